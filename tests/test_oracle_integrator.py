"""Pins of the oracle's kick-drift-kick run (Eq. (9) operators, Eq. (1) forces).

* free particles: the 2(da/dt/a) v drag makes v fall as a^-2 exactly, and
  x moves by a0^2 v0 times the drift integral,
* static limit (a = 1, H = 0): the two-body Kepler orbit against the closed
  form from Kepler's equation, with second-order convergence, bounded energy
  error and conserved angular momentum,
* time reversibility, conservation of total momentum and angular momentum,
* the Layzer-Irvine equation dE/d ln a = -(2K + U) for the expanding run,
  whose residual converges at second order,
* the reverse-mode gradient against central finite differences of the run,
* the finite-time Lyapunov exponent in closed-form limits.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1208_3444_amd.inputs import EDS, LCDM, eds_lattice, random_cloud

STATIC = dict(H0=0.0, Om_R=0.0, Om_M=0.0, Om_K=0.0, Om_L=0.0)


def test_free_particle_drag_and_drift():
    x0 = np.array([[0.1, 0.4], [0.2, -0.3], [0.3, 0.7]])
    v0 = np.array([[1.0, -2.0], [0.5, 0.25], [-0.75, 3.0]])
    m = np.array([0.5, 0.5])
    a0, a1 = 0.1, 1.0
    x, v = oracle.run(x0, v0, m, 0.01, 0.0, LCDM, a0, a1, 37)  # G = 0: no pair force
    D = oracle.time_integral("drift", a0, a1, LCDM["H0"], 0, 0.3, 0, 0.7)
    assert np.allclose(v, v0 * (a0 / a1) ** 2, rtol=1e-14, atol=0)
    assert np.allclose(x, x0 + a0 ** 2 * v0 * D, rtol=1e-13, atol=1e-15)
    # single particle with gravity on: no pair, same result
    x1, v1 = oracle.run(x0[:, :1], v0[:, :1], m[:1], 0.01, 1.0, LCDM, a0, a1, 5)
    assert np.allclose(v1, v0[:, :1] * (a0 / a1) ** 2, rtol=1e-14, atol=0)
    # the paper's H&E drag factor (1 - H tau)/(1 + H tau) is the Pade
    # approximant of this exact decay: per-step ratio differs at O(tau^3)
    h0 = EDS["H0"]
    for tau in (1e-2, 5e-3):
        a = 0.5
        t0 = 2 * a ** 1.5 / (3 * h0)
        a_next = (1.5 * h0 * (t0 + tau)) ** (2 / 3)
        hh = h0 * ((a * a_next) ** 0.5) ** -1.5
        exact = (a / a_next) ** 2
        pade = (1 - hh * tau) / (1 + hh * tau)
        assert abs(exact - pade) < 10 * (hh * tau) ** 3


def _kepler_state(e, t):
    """Two equal masses (total 1), G = 1, semi-major axis 1, pericentre at t=0."""
    Mn = t  # mean motion sqrt(G M / A^3) = 1
    E = Mn
    for _ in range(60):
        E -= (E - e * math.sin(E) - Mn) / (1 - e * math.cos(E))
    r = np.array([math.cos(E) - e, math.sqrt(1 - e * e) * math.sin(E), 0.0])
    Edot = 1.0 / (1 - e * math.cos(E))
    rv = np.array([-math.sin(E) * Edot, math.sqrt(1 - e * e) * math.cos(E) * Edot, 0.0])
    x = np.stack([-0.5 * r, 0.5 * r], axis=1)
    v = np.stack([-0.5 * rv, 0.5 * rv], axis=1)
    return x, v


@pytest.mark.parametrize("e", [0.0, 0.5])
def test_kepler_second_order(e):
    m = np.array([0.5, 0.5])
    T = 2 * math.pi
    x0, v0 = _kepler_state(e, 0.0)
    xT, vT = _kepler_state(e, T)
    errs = []
    for n in (200, 400, 800):
        x, v = oracle.run(x0, v0, m, 0.0, 1.0, STATIC, 1.0, T, n)
        errs.append(np.linalg.norm(x - xT))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs
    assert errs[-1] < 2e-3


def test_kepler_energy_bounded_angular_momentum_conserved():
    m = np.array([0.5, 0.5])
    x0, v0 = _kepler_state(0.5, 0.0)
    n = 4000
    x, v, d = oracle.run(x0, v0, m, 0.0, 1.0, STATIC, 1.0, 20 * 2 * math.pi, n, diag=True)
    E = d["K"] + d["U"]
    # no secular drift: the error in the last period is no larger than in the first
    assert np.max(np.abs(E - E[0])) < 1e-2 * abs(E[0])
    first, last = np.abs(E[: n // 20] - E[0]).max(), np.abs(E[-n // 20:] - E[0]).max()
    assert last < 1.5 * first
    assert np.allclose(d["LI"], E - E[0], atol=1e-15)
    L = np.stack([d["Lx"], d["Ly"], d["Lz"]])
    assert np.max(np.abs(L - L[:, :1])) < 1e-14
    P = np.stack([d["Px"], d["Py"], d["Pz"]])
    assert np.max(np.abs(P)) < 1e-15
    assert d["t"][-1] == pytest.approx(40 * math.pi, rel=1e-13)


def test_time_reversibility_expanding():
    x0, m = random_cloud(32, 21, scale=0.3)
    v0 = 0.2 * np.random.default_rng(1).standard_normal((3, 32))
    eps = 0.02
    x1, v1 = oracle.run(x0, v0, m, eps, 1.0, LCDM, 0.2, 0.5, 40)
    xb, vb = oracle.run(x1, v1, m, eps, 1.0, LCDM, 0.5, 0.2, 40)
    assert np.max(np.abs(xb - x0)) < 1e-12
    assert np.max(np.abs(vb - v0)) < 1e-11


def test_momentum_and_angular_momentum_conserved():
    x0, m = random_cloud(48, 22, scale=0.3)
    v0 = 0.3 * np.random.default_rng(2).standard_normal((3, 48))
    x, v, d = oracle.run(x0, v0, m, 0.02, 1.0, LCDM, 0.1, 1.0, 30, diag=True)
    P = np.stack([d["Px"], d["Py"], d["Pz"]])
    L = np.stack([d["Lx"], d["Ly"], d["Lz"]])
    # roundoff scale: the sums of |m p| and |m x x p| over particles
    p_scale = np.sum(m * np.linalg.norm(v, axis=0))
    l_scale = np.sum(m * np.linalg.norm(x, axis=0) * np.linalg.norm(v, axis=0))
    assert np.max(np.abs(P - P[:, :1])) < 1e-13 * p_scale
    assert np.max(np.abs(L - L[:, :1])) < 1e-13 * l_scale


def test_run_resume_matches_single_run():
    w = eds_lattice(4, seed=1, n_steps=12)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    args = (w.m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, w.n_steps)
    xa, va = oracle.run(w.x, v0, *args)
    xh, vh = oracle.run(w.x, v0, *args, first_step=0, last_step=5)
    xb, vb = oracle.run(xh, vh, *args, first_step=5, last_step=12)
    assert np.max(np.abs(xb - xa)) < 1e-13
    assert np.max(np.abs(vb - va)) < 1e-12 * np.abs(va).max()


def test_layzer_irvine_second_order():
    # a from 0.1 to 0.4: before the open box's mean-field collapse, where
    # close encounters (not the step size) would dominate the residual
    w = eds_lattice(6, seed=1)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    res = []
    for n in (16, 32, 64):
        _, _, d = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 0.4, n,
                             diag=True)
        assert d["a"][-1] == 0.4
        res.append(abs(d["LI"][-1]))
    r1, r2 = res[0] / res[1], res[1] / res[2]
    assert 3.8 < r1 < 4.2 and 3.9 < r2 < 4.1, res
    assert res[-1] < 1e-3 * abs(d["U"][-1])
    # the rows are consistent: E - E0 + trapezoid of (2K + U) in ln a
    E = d["K"] + d["U"]
    src = 2 * d["K"] + d["U"]
    trap = np.concatenate([[0.0], np.cumsum(0.5 * (src[1:] + src[:-1]) * np.diff(np.log(d["a"])))])
    assert np.allclose(d["LI"], E - E[0] + trap, rtol=0, atol=1e-12 * np.abs(E).max())


def _loss_and_grad(x0, v0, m, eps, G, cos, a_b, a_e, n, tracers):
    xN, vN = oracle.run(x0, v0, m, eps, G, cos, a_b, a_e, n)
    L = float(np.sum(vN[:, tracers] ** 2))
    lam_v = np.zeros_like(vN)
    lam_v[:, tracers] = 2 * vN[:, tracers]
    gx, gv, xN2, vN2 = oracle.adjoint(x0, v0, m, eps, G, cos, a_b, a_e, n,
                                      np.zeros_like(xN), lam_v)
    assert np.array_equal(xN2, xN) and np.array_equal(vN2, vN)
    return L, gx, gv


def test_adjoint_matches_central_differences():
    # a mild cloud (G = 0.2) keeps the map close to linear over h
    x0, m = random_cloud(40, 31, scale=0.5)
    v0 = 0.3 * np.random.default_rng(3).standard_normal((3, 40))
    tracers = np.array([0, 5, 9, 33])
    args = (m, 0.03, 0.2, LCDM, 0.2, 1.0, 12)
    L, gx, gv = _loss_and_grad(x0, v0, *args, tracers)
    rng = np.random.default_rng(4)
    for _ in range(4):
        ux = rng.standard_normal(x0.shape)
        uv = rng.standard_normal(v0.shape)
        nrm = math.sqrt(np.sum(ux ** 2) + np.sum(uv ** 2))
        ux /= nrm
        uv /= nrm
        fd = []
        for h in (1e-5, 5e-6):
            Lp = np.sum(oracle.run(x0 + h * ux, v0 + h * uv, *args)[1][:, tracers] ** 2)
            Lm = np.sum(oracle.run(x0 - h * ux, v0 - h * uv, *args)[1][:, tracers] ** 2)
            fd.append((Lp - Lm) / (2 * h))
        rich = (4 * fd[1] - fd[0]) / 3  # Richardson: O(h^4)
        ad = np.sum(gx * ux) + np.sum(gv * uv)
        assert abs(fd[1] - fd[0]) < 1e-5 * abs(rich)
        assert abs(ad - rich) <= 1e-8 * abs(rich), (ad, fd)


def test_adjoint_multi_cotangent_is_batch_of_single():
    x0, m = random_cloud(16, 41, scale=0.3)
    v0 = 0.1 * np.random.default_rng(5).standard_normal((3, 16))
    rng = np.random.default_rng(6)
    lx = rng.standard_normal((3, 3, 16))
    lv = rng.standard_normal((3, 3, 16))
    args = (m, 0.05, 1.0, EDS, 0.1, 1.0, 6)
    gx, gv, _, _ = oracle.adjoint(x0, v0, *args, lx, lv)
    for c in range(3):
        gx1, gv1, _, _ = oracle.adjoint(x0, v0, *args, lx[c], lv[c])
        assert np.array_equal(gx1, gx[c]) and np.array_equal(gv1, gv[c])


def test_ftle_limits():
    x0, m = random_cloud(12, 51, scale=0.3)
    v0 = 0.1 * np.random.default_rng(7).standard_normal((3, 12))
    # no gravity: the flow map is x0 + const * v0, so d x_N / d x_0 = I
    lam_t, lam_lna, phi = oracle.ftle(x0, v0, m, 0.05, 0.0, EDS, 0.1, 1.0, 8, [1, 4])
    assert np.allclose(phi, np.eye(3)[None], atol=1e-15)
    assert np.allclose(lam_t, 0.0, atol=1e-15)
    # with gravity: the block matches central differences of the forward map
    # (Richardson-extrapolated; this dense cloud is strongly nonlinear)
    args = (m, 0.05, 1.0, EDS, 0.1, 1.0, 8)
    _, _, phi = oracle.ftle(x0, v0, m, 0.05, 1.0, EDS, 0.1, 1.0, 8, [4])

    def col(j, h):
        xp = x0.copy(); xp[j, 4] += h
        xm = x0.copy(); xm[j, 4] -= h
        return (oracle.run(xp, v0, *args)[0][:, 4] - oracle.run(xm, v0, *args)[0][:, 4]) / (2 * h)

    for j in range(3):
        rich = (4 * col(j, 5e-7) - col(j, 1e-6)) / 3
        assert np.allclose(phi[0][:, j], rich, rtol=1e-7, atol=1e-7 * np.abs(rich).max())
