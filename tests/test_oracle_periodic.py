"""Pins of the oracle's periodic field (Ewald summation), independent of the
implementation:

* a single particle in a box feels no force, and its potential is minus G m
  times the simple cubic lattice's Madelung constant (with the neutralising
  background), -2.8372974794806 / L (Nijboer and de Wette 1957): pins the
  reciprocal sum's normalisation, the background constant and the self
  terms together;
* a particle on a perfect cubic lattice of n^3 sites feels no force and has
  the potential of that lattice: -G m (-2.83729...) n / L;
* the splitting parameter alpha is arbitrary: results at alpha L = 4, 6, 9
  (real and reciprocal parts in very different proportions) agree to
  roundoff, which fails for any wrong factor or sign in either part;
* a compact cluster far smaller than the box feels its own open-box field
  (Eq. (1), softened) plus the near-field of its images and the removed
  background, which for a cubic lattice is isotropic:
  -(4 pi G / (3 L^3)) sum_j m_j (x_j - x_k)  (background density M / L^3,
  divergence +4 pi G rho), up to O(s^3 / L^5);
* periodicity (a shift by any vector, positions left unwrapped), momentum
  (sum m g = 0), the potential energy's gradient (W = 1/2 sum m phi,
  m_k g_k = -dW/dx_k by central differences), and the target-subset form.
"""
import numpy as np
import pytest

import oracle
from paper_1208_3444_amd import inputs

MADELUNG_SC = -2.8372974794806


def _cloud(n, seed, L):
    x, m = inputs.random_cloud(n, seed, scale=L)
    return x, m


@pytest.mark.parametrize("L", [1.0, 2.5])
def test_single_particle_madelung(L):
    x = np.array([[0.3], [0.6], [0.1]]) * L
    for aL in (4.0, 6.0, 9.0):
        acc, phi = oracle.forces_periodic(x, np.array([2.0]), 0.01 * L, L, G=1.5,
                                          with_phi=True, alpha=aL / L)
        assert np.all(acc == 0.0)
        assert phi[0] == pytest.approx(-1.5 * 2.0 * MADELUNG_SC / L, rel=1e-12)


def test_cubic_lattice_no_force_madelung_potential():
    n, L = 4, 2.0
    g = (np.arange(n) + 0.5) * L / n
    x = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    m = np.full(n ** 3, 0.7)
    acc, phi = oracle.forces_periodic(x, m, 0.0, L, with_phi=True)
    scale = 0.7 / (L / n) ** 2
    assert np.max(np.abs(acc)) <= 1e-13 * scale
    assert np.allclose(phi, -0.7 * MADELUNG_SC * n / L, rtol=1e-12, atol=0)


def test_splitting_parameter_independence():
    L = 1.0
    x, m = _cloud(40, 3, L)
    ref = oracle.forces_periodic(x, m, 0.02, L, with_phi=True, alpha=6.0)
    for aL in (4.0, 9.0):
        acc, phi = oracle.forces_periodic(x, m, 0.02, L, with_phi=True, alpha=aL)
        assert np.max(np.abs(acc - ref[0])) <= 1e-13 * np.abs(ref[0]).max()
        assert np.max(np.abs(phi - ref[1])) <= 1e-13 * np.abs(ref[1]).max()


def test_compact_cluster_open_box_limit():
    """The same 12-particle cluster shrunk about the box centre: the periodic
    field minus the open-box field minus the background term is the image
    lattice's next (l = 4) term, which scales as the cube of the cluster's
    size, while the background term scales as its size."""
    L = 1.0
    rng = np.random.default_rng(8)
    u = rng.uniform(-1, 1, size=(3, 12))
    m = rng.uniform(0.5, 1.5, 12)
    c = np.array([0.5, 0.5, 0.5])[:, None]
    res, bgs = [], []
    for s in (0.004, 0.002, 0.001):
        x = c + s * u
        eps = 0.3 * s
        per = oracle.forces_periodic(x, m, eps, L)
        opn = oracle.forces(x, m, eps)
        d = (m[None, :, None] * (x[:, :, None] - x[:, None, :])).sum(axis=1)
        bg = -(4.0 * np.pi / (3.0 * L ** 3)) * d
        res.append(np.max(np.abs(per - opn - bg)))
        bgs.append(np.max(np.abs(bg)))
    assert 6.0 <= res[0] / res[1] <= 10.0 and 6.0 <= res[1] / res[2] <= 10.0, res
    assert 1.8 <= bgs[0] / bgs[1] <= 2.2
    assert bgs[2] >= 1e4 * res[2]


def test_periodicity_momentum_and_gradient():
    L = 1.3
    x, m = _cloud(25, 11, L)
    eps = 0.01
    acc, phi = oracle.forces_periodic(x, m, eps, L, with_phi=True)
    scale = np.abs(acc).max()
    # a shift by any vector (not wrapped back): the same field
    shift = np.array([0.37, -1.21, 2.5])[:, None] * L
    acc2 = oracle.forces_periodic(x + shift, m, eps, L)
    assert np.max(np.abs(acc2 - acc)) <= 1e-12 * scale
    # momentum
    assert np.max(np.abs((m[None, :] * acc).sum(axis=1))) <= 1e-14 * (m.sum() * scale)
    # m_k g_k = -dW/dx_k, W = 1/2 sum m phi
    def W(xx):
        return 0.5 * np.sum(m * oracle.forces_periodic(xx, m, eps, L, with_phi=True)[1])
    h = 1e-6
    for k in (0, 7, 19):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[c, k] += h
            xm[c, k] -= h
            fd = -(W(xp) - W(xm)) / (2 * h)
            assert fd == pytest.approx(m[k] * acc[c, k], rel=1e-6, abs=1e-9 * scale)
    # target subset
    t = np.array([3, 0, 24, 11])
    acc_t, phi_t = oracle.forces_periodic(x, m, eps, L, with_phi=True, targets=t)
    assert np.array_equal(acc_t, acc[:, t]) and np.array_equal(phi_t, phi[t])


def test_periodic_run_energy_second_order_and_momentum():
    """Static limit (a = 1, H0 = 0): the kick-drift-kick run with the
    periodic field conserves total momentum to roundoff, and its energy
    error, K + W with W = 1/2 sum m phi, falls by 4 when the step halves
    (second order: the field is the gradient of that potential)."""
    static = dict(H0=0.0, Om_R=0.0, Om_M=0.0, Om_K=0.0, Om_L=0.0)
    x, m = inputs.random_cloud(120, 77, scale=1.0)
    v = 0.05 * np.random.default_rng(77).standard_normal((3, 120))

    def energy(xx, vv):
        _, phi = oracle.forces_periodic(xx, m, 0.02, 1.0, with_phi=True)
        return 0.5 * np.sum(m * (vv ** 2).sum(axis=0)) + 0.5 * np.sum(m * phi)

    E0 = energy(x, v)
    err = []
    for n in (50, 100):
        xe, ve = oracle.run_periodic(x, v, m, 0.02, 1.0, static, 1.0, 1.0, 0.1, n)
        assert np.all((xe >= 0.0) & (xe < 1.0))
        assert np.abs((m * ve).sum(axis=1) - (m * v).sum(axis=1)).max() <= 1e-15
        err.append(abs(energy(xe, ve) - E0))
    assert 3.6 <= err[0] / err[1] <= 4.4, err
