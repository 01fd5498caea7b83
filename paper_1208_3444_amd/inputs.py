"""Seeded synthetic inputs shaped like the paper's runs.

This module only draws and lays out input arrays: lattices, displacement
fields, masses and the parameters of each workload.  It holds none of the
method's arithmetic (no forces, no Friedmann equation, no integrator); where
an input depends on the method (the initial velocity v = H(a_i) psi needs
H from Eq. (2)), the caller supplies that factor.  Both the HIP path and the
oracle take their inputs from here.

The paper's own initial conditions (a glass perturbed with an Eisenstein-Hu
spectrum at z = 50 in a 100 Mpc box) are not reproducible without its data,
so these recipes stand in for them at the paper's scale (up to 32^3
particles, a from 1/51 to 1):

* ``lattice_gaussian`` -- cell-centred n^3 lattice of spacing d = 1/n in the
  unit box, plus i.i.d. Gaussian displacements of sigma per component.
* ``lattice_grf``      -- the same lattice displaced by an irrotational
  Gaussian random field with displacement power spectrum P(k) ~ k^-2,
  psi_hat(k) = i k/|k|^2 W_hat(k) for white noise W, k = 0 and Nyquist
  planes zeroed, rescaled to a given rms per component.
* ``ragged_ensemble``  -- independent boxes with N log-uniform in a range,
  each a random subset of a cell-centred lattice plus Gaussian displacements.

Particles are emitted in Morton (Z-curve) order of their lattice site, so
that consecutive particles are spatially compact.  Random numbers come from
``numpy.random.Generator(PCG64(seed))``.
"""
from dataclasses import dataclass, field
import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def morton_codes(ijk: np.ndarray) -> np.ndarray:
    """Interleave the bits of integer lattice indices (M, 3) -> (M,) uint64."""
    ijk = np.asarray(ijk, dtype=np.uint64)
    code = np.zeros(ijk.shape[0], dtype=np.uint64)
    for bit in range(21):
        for axis in range(3):
            b = (ijk[:, axis] >> np.uint64(bit)) & np.uint64(1)
            code |= b << np.uint64(3 * bit + axis)
    return code


def lattice_sites(n: int) -> np.ndarray:
    """All (i, j, k) sites of an n^3 lattice, (n^3, 3), in C order."""
    g = np.arange(n)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def _morton_sort(ijk):
    return np.argsort(morton_codes(ijk), kind="stable")


def _positions(ijk, d):
    """Cell-centred comoving positions (3, M) of lattice sites."""
    return ((ijk.astype(np.float64) + 0.5) * d).T.copy()


def grf_displacement(n: int, rms: float, rng) -> np.ndarray:
    """Irrotational Gaussian displacement field on an n^3 grid, (3, n, n, n).

    psi_hat(k) = i k / |k|^2 W_hat(k), W white noise; the k = 0 mode and the
    Nyquist planes are zeroed, and the field is rescaled so that the rms
    over all 3 n^3 components equals ``rms``.
    """
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2[0, 0, 0] = 1.0
    mask = np.ones_like(k2)
    mask[0, 0, 0] = 0.0
    if n % 2 == 0:
        mask[n // 2, :, :] = 0.0
        mask[:, n // 2, :] = 0.0
        mask[:, :, n // 2] = 0.0
    psi = np.empty((3, n, n, n))
    for axis, K in enumerate((KX, KY, KZ)):
        psi[axis] = np.fft.irfftn(1j * K / k2 * wk * mask, s=(n, n, n), axes=(0, 1, 2))
    psi *= rms / np.sqrt(np.mean(psi ** 2))
    return psi


@dataclass
class Workload:
    """One synthetic workload: state, model parameters and time grid.

    ``x`` and ``psi`` are (3, N) float64; the initial comoving velocity is
    ``v_scale * psi`` with v_scale = H(a_begin) supplied by the caller.
    For ensembles, ``box_offsets`` (B+1,) and ``box_eps`` (B,) describe the
    concatenated boxes and ``eps`` is unused.
    """
    name: str
    x: np.ndarray
    psi: np.ndarray
    m: np.ndarray
    eps: float
    G: float
    cosmo: dict
    a_begin: float
    a_end: float
    n_steps: int
    seed: int
    extra: dict = field(default_factory=dict)
    box_offsets: np.ndarray = None
    box_eps: np.ndarray = None

    @property
    def N(self) -> int:
        return int(self.m.shape[0])

    def velocities(self, v_scale: float) -> np.ndarray:
        return v_scale * self.psi


def lattice_gaussian(n: int, sigma_over_d: float, seed: int):
    """(x, psi, d) for a Morton-ordered cell-centred lattice + Gaussian psi."""
    d = 1.0 / n
    ijk = lattice_sites(n)
    order = _morton_sort(ijk)
    ijk = ijk[order]
    rng = _rng(seed)
    psi = rng.normal(0.0, sigma_over_d * d, size=(3, n ** 3))
    return _positions(ijk, d) + psi, psi, d


def lattice_grf(n: int, rms_over_d: float, seed: int):
    """(x, psi, d) for a Morton-ordered lattice displaced by the k^-2 field."""
    d = 1.0 / n
    rng = _rng(seed)
    field_ = grf_displacement(n, rms_over_d * d, rng).reshape(3, -1)
    ijk = lattice_sites(n)
    order = _morton_sort(ijk)
    psi = field_[:, order].copy()
    return _positions(ijk[order], d) + psi, psi, d


EDS = dict(H0=math.sqrt(8.0 * math.pi / 3.0), Om_R=0.0, Om_M=1.0, Om_K=0.0, Om_L=0.0)
LCDM = dict(H0=math.sqrt(8.0 * math.pi / (3.0 * 0.3)), Om_R=0.0, Om_M=0.3, Om_K=0.0,
            Om_L=0.7)


def eds_lattice(n: int = 16, seed: int = 1, a_begin: float = 0.1, a_end: float = 1.0,
                n_steps: int = 64) -> Workload:
    """Plain-method FP64 workload: n^3 equal-mass particles, EdS, sigma = 0.02 d."""
    x, psi, d = lattice_gaussian(n, 0.02, seed)
    N = n ** 3
    return Workload(f"eds_lattice_{n}^3", x, psi, np.full(N, 1.0 / N), 0.05 * d, 1.0,
                    dict(EDS), a_begin, a_end, n_steps, seed)


def lcdm_grf(n: int = 32, seed: int = 2, a_begin: float = 1.0 / 51.0, a_end: float = 1.0,
             n_steps: int = 1000) -> Workload:
    """Paper-scale LCDM workload: n^3 particles, k^-2 displacement field, rms 0.1 d."""
    x, psi, d = lattice_grf(n, 0.1, seed)
    N = n ** 3
    return Workload(f"lcdm_grf_{n}^3", x, psi, np.full(N, 1.0 / N), 0.05 * d, 1.0,
                    dict(LCDM), a_begin, a_end, n_steps, seed)


def precision_sweep(n: int = 64, seed: int = 3, n_targets: int = 4096,
                    target_seed: int = 33) -> Workload:
    """Single force evaluation at a = 0.5 on the LCDM recipe, with sampled targets."""
    w = lcdm_grf(n, seed, a_begin=0.5, a_end=0.5, n_steps=1)
    w.name = f"precision_sweep_{n}^3"
    w.extra["targets"] = np.sort(_rng(target_seed).choice(w.N, size=min(n_targets, w.N),
                                                           replace=False))
    w.extra["a"] = 0.5
    return w


def adjoint_run(n: int = 32, seed: int = 4, n_steps: int = 200, n_tracers: int = 64,
                tracer_seed: int = 44, n_dirs: int = 16, dir_seed: int = 444,
                checkpoint_every: int = 20) -> Workload:
    """LCDM recipe from a = 0.2 to 1, tracers and finite-difference directions."""
    w = lcdm_grf(n, seed, a_begin=0.2, a_end=1.0, n_steps=n_steps)
    w.name = f"adjoint_{n}^3"
    rng = _rng(tracer_seed)
    w.extra["tracers"] = np.sort(rng.choice(w.N, size=min(n_tracers, w.N), replace=False))
    w.extra["checkpoint_every"] = checkpoint_every
    drng = _rng(dir_seed)
    dirs = drng.standard_normal((n_dirs, 2, 3, w.N))
    dirs /= np.sqrt((dirs ** 2).sum(axis=(1, 2, 3), keepdims=True))
    w.extra["fd_directions"] = dirs
    return w


def ragged_ensemble(n_boxes: int = 256, n_min: int = 512, n_max: int = 8192, seed: int = 5,
                    a_begin: float = 0.1, a_end: float = 1.0, n_steps: int = 500) -> Workload:
    """Independent open unit boxes with N log-uniform in [n_min, n_max].

    Box b: n = ceil(N^(1/3)); a random subset of N sites of the cell-centred
    n^3 lattice of spacing 1/n (seed 5000 + b), Morton ordered; Gaussian
    displacements with sigma = 0.02 d_box, eps = 0.05 d_box, m = 1/N, where
    d_box = N^(-1/3).  EdS cosmology as for the lattice workload.
    """
    rng = _rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_boxes)))
    sizes = sizes.astype(np.int64)
    xs, psis, ms, epss = [], [], [], []
    for b, nb in enumerate(sizes):
        nb = int(nb)
        n = int(round(nb ** (1.0 / 3.0)))
        while n ** 3 < nb:
            n += 1
        while (n - 1) ** 3 >= nb:
            n -= 1
        brng = _rng(5000 + b)
        sites = lattice_sites(n)
        pick = np.sort(brng.choice(n ** 3, size=nb, replace=False))
        ijk = sites[pick]
        ijk = ijk[_morton_sort(ijk)]
        d_box = nb ** (-1.0 / 3.0)
        psi = brng.normal(0.0, 0.02 * d_box, size=(3, nb))
        xs.append(_positions(ijk, 1.0 / n) + psi)
        psis.append(psi)
        ms.append(np.full(nb, 1.0 / nb))
        epss.append(0.05 * d_box)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    w = Workload(f"ragged_ensemble_{n_boxes}", np.concatenate(xs, axis=1),
                 np.concatenate(psis, axis=1), np.concatenate(ms), float("nan"), 1.0,
                 dict(EDS), a_begin, a_end, n_steps, seed)
    w.box_offsets = offsets
    w.box_eps = np.asarray(epss)
    return w


def random_cloud(N: int, seed: int, scale: float = 1.0, mass_spread: bool = True):
    """Small irregular test cloud: (x (3,N), m (N,)) with unequal masses."""
    rng = _rng(seed)
    x = rng.uniform(-scale, scale, size=(3, N))
    m = rng.uniform(0.5, 1.5, size=N) / N if mass_spread else np.full(N, 1.0 / N)
    return x, m
