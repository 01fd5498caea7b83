"""Pins of the oracle's tracer tracks and single-particle velocity power
spectrum (the introduction's stated goal: a particle's velocity at every
step and the power spectrum of that series).

* A track's row r is the state a run over [first, first + r) ends in
  (bitwise, both schemes): the row index, the position/velocity columns and
  the p -> v conversion are the run's own.
* Free particles under the kick-drift-kick run: every row's velocity is the
  exact a^-2 decay; with every particle traced, 1/2 sum m a^2 |v|^2 of each
  row is the diagnostics' K.
* The spectrum against numpy's FFT (a different routine from the oracle's
  direct sum), Parseval's identity over the full two-sided periodogram, a
  pure cosine at a bin frequency and at the Nyquist frequency, a constant
  (all power at k = 0, none once the mean is removed), components summed.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1208_3444_amd.inputs import EDS, LCDM, eds_lattice, random_cloud


@pytest.mark.parametrize("scheme", ["kdk", "he"])
def test_track_rows_are_run_end_states(scheme):
    fn = oracle.run if scheme == "kdk" else oracle.run_he
    x0, m = random_cloud(30, 11, scale=0.4)
    v0 = 0.2 * np.random.default_rng(12).standard_normal((3, 30))
    tr = np.array([4, 0, 29, 17])
    args = (m, 0.03, 1.0, LCDM, 0.2, 1.0, 12)
    first, last = 3, 9
    xs, vs = fn(x0, v0, *args, last_step=first)
    x, v, track = fn(xs, vs, *args, first_step=first, last_step=last, tracers=tr)
    assert track.shape == (last - first + 1, 2, 3, 4)
    assert np.array_equal(track[0, 0], xs[:, tr]) and np.array_equal(track[0, 1], vs[:, tr])
    assert np.array_equal(track[-1, 0], x[:, tr]) and np.array_equal(track[-1, 1], v[:, tr])
    for r in (1, 4):
        xr, vr = fn(xs, vs, *args, first_step=first, last_step=first + r)
        assert np.array_equal(track[r, 0], xr[:, tr]) and np.array_equal(track[r, 1], vr[:, tr])
    # the track does not change the run
    x2, v2 = fn(xs, vs, *args, first_step=first, last_step=last)
    assert np.array_equal(x, x2) and np.array_equal(v, v2)


def test_free_particles_and_kinetic_energy():
    x0, m = random_cloud(6, 2, scale=0.5)
    v0 = np.random.default_rng(3).standard_normal((3, 6))
    a0, a1, n = 0.1, 1.0, 16
    _, _, track = oracle.run(x0, v0, m, 0.01, 0.0, EDS, a0, a1, n, tracers=np.arange(6))
    a = a0 * (a1 / a0) ** (np.arange(n + 1) / n)
    for r in range(n + 1):
        assert np.allclose(track[r, 1], v0 * (a0 / a[r]) ** 2, rtol=1e-14, atol=0)
    w = eds_lattice(4, n_steps=8)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    for fn in (oracle.run, oracle.run_he):
        _, _, d, track = fn(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 8,
                            diag=True, tracers=np.arange(w.N))
        K = 0.5 * np.einsum("k,rck->r", w.m, track[:, 1] ** 2) * d["a"] ** 2
        assert np.allclose(K, d["K"], rtol=1e-13, atol=0)


def _track_from_velocity(vel):
    """vel (M, 3, T) -> a track with zero positions."""
    M, _, T = vel.shape
    tr = np.zeros((M, 2, 3, T))
    tr[:, 1] = vel
    return tr


@pytest.mark.parametrize("M", [1, 2, 7, 64, 101])
@pytest.mark.parametrize("remove_mean", [False, True])
def test_spectrum_against_fft_and_parseval(M, remove_mean):
    rng = np.random.default_rng(M)
    vel = rng.standard_normal((M, 3, 5)) + 0.7
    E = oracle.velocity_spectrum(_track_from_velocity(vel), remove_mean=remove_mean)
    assert E.shape == (5, M // 2 + 1)
    w = vel - vel.mean(axis=0) if remove_mean else vel
    ref = (np.abs(np.fft.fft(w, axis=0)) ** 2).sum(axis=1).T[:, : M // 2 + 1] / M
    energy = (w ** 2).sum(axis=(0, 1))
    assert np.all(np.abs(E - ref) <= 1e-13 * energy[:, None])
    # Parseval over the two-sided periodogram P(k) = P(M - k)
    full = E[:, 0] + 2 * E[:, 1:(M + 1) // 2].sum(axis=1)
    if M % 2 == 0:
        full = full + E[:, M // 2]
    assert np.allclose(full, energy, rtol=1e-13, atol=1e-300)


def test_spectrum_pure_tones_and_constant():
    M = 96
    n = np.arange(M)
    vel = np.zeros((M, 3, 4))
    vel[:, 0, 0] = 1.5 * np.cos(2 * math.pi * 5 * n / M + 0.3)  # bin 5
    vel[:, 1, 1] = 1.5 * np.cos(2 * math.pi * 5 * n / M + 0.3)  # same tone in y
    vel[:, 2, 2] = 0.8 * np.cos(math.pi * n)                     # Nyquist
    vel[:, 2, 3] = -2.0                                          # constant
    E = oracle.velocity_spectrum(_track_from_velocity(vel))
    tiny = 1e-24
    assert E[0, 5] == pytest.approx(M * 1.5 ** 2 / 4, rel=1e-13)
    assert np.all(np.delete(E[0], 5) < tiny)
    assert np.array_equal(E[0], E[1]) or np.allclose(E[0], E[1], rtol=1e-14, atol=tiny)
    assert E[2, M // 2] == pytest.approx(M * 0.8 ** 2, rel=1e-13)
    assert np.all(E[2, : M // 2] < tiny)
    assert E[3, 0] == pytest.approx(M * 4.0, rel=1e-14)
    assert np.all(E[3, 1:] < tiny)
    Em = oracle.velocity_spectrum(_track_from_velocity(vel), remove_mean=True)
    assert np.all(Em[3] < tiny)
    assert Em[0, 5] == pytest.approx(E[0, 5], rel=1e-13)  # a tone has zero mean


def test_spectrum_at_chosen_bins():
    rng = np.random.default_rng(5)
    M = 77
    vel = rng.standard_normal((M, 3, 3)) - 0.4
    tr = _track_from_velocity(vel)
    bins = [0, 1, 38, 12]
    for rm in (False, True):
        full = oracle.velocity_spectrum(tr, remove_mean=rm)
        assert np.array_equal(oracle.velocity_spectrum_bins(tr, bins, remove_mean=rm),
                              full[:, bins])
    # a long series (the GPU limit) against numpy's FFT at a few bins
    M = 1 << 17
    vel = rng.standard_normal((M, 3, 1))
    tr = _track_from_velocity(vel)
    bins = [0, 1, 4097, M // 2]
    got = oracle.velocity_spectrum_bins(tr, bins)
    ref = (np.abs(np.fft.fft(vel, axis=0)) ** 2).sum(axis=1).T[:, bins] / M
    assert np.allclose(got, ref, rtol=1e-9, atol=1e-12 * (vel ** 2).sum())
