"""Pins of the oracle's Hockney-Eastwood difference equations (Eqs. (3)-(5)):
drift half a step, kick with the drag factor (1 - H tau)/(1 + H tau) and the
force at the half step over a^3 (1 + H tau), drift the other half, with H
and a at the step's half time.

* The step's tau is the cosmic time between grid points and a_h solves
  t(a_h) = t_n + tau / 2 (against the pinned time integral).
* Free particles: v and x converge at second order to the exact a^-2 decay
  and drift integral.
* Static limit: the scheme is the leapfrog; a Kepler orbit converges at
  second order and the map is time-reversible.
* Expanding background: the Layzer-Irvine residual converges at second order,
  and the scheme converges to the same trajectory as the (pinned)
  kick-drift-kick run.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1208_3444_amd.inputs import EDS, LCDM, eds_lattice, random_cloud

STATIC = {"H0": 0.0, "Om_R": 0.0, "Om_M": 0.0, "Om_K": 0.0, "Om_L": 0.0}


def _c(cos):
    return cos["H0"], cos["Om_R"], cos["Om_M"], cos["Om_K"], cos["Om_L"]


@pytest.mark.parametrize("cos", [EDS, LCDM])
def test_step_time_and_half_time(cos):
    a0, a1, n = 0.1, 1.0, 7
    for k in (0, 3, 6):
        tau, ah, Hh = oracle.he_coefficients(cos, a0, a1, n, k)
        an = a0 * (a1 / a0) ** (k / n)
        an1 = a0 * (a1 / a0) ** ((k + 1) / n)
        assert tau == pytest.approx(oracle.time_integral("time", an, an1, *_c(cos)), rel=1e-13)
        half = oracle.time_integral("time", an, ah, *_c(cos))
        assert half == pytest.approx(0.5 * tau, rel=1e-11)
        assert an < ah < an1
        assert Hh == pytest.approx(oracle.hubble(ah, *_c(cos)), rel=1e-14)
    # EdS closed form: t ~ a^{3/2}, so a_h = ((a_n^1.5 + a_n+1^1.5)/2)^{2/3}
    tau, ah, _ = oracle.he_coefficients(EDS, 0.1, 1.0, 1, 0)
    assert ah == pytest.approx(((0.1 ** 1.5 + 1.0) / 2) ** (2 / 3), rel=1e-11)
    assert oracle.he_coefficients(STATIC, 2.0, 3.0, 6, 2) == (0.5, 2.0, 0.0)


def test_free_particles_second_order():
    x0, m = random_cloud(5, 1, scale=0.5)
    v0 = np.random.default_rng(2).standard_normal((3, 5))
    a0, a1 = 0.1, 1.0
    v_exact = v0 * (a0 / a1) ** 2
    x_exact = x0 + v0 * a0 ** 2 * oracle.time_integral("drift", a0, a1, *_c(EDS))
    ev, ex = [], []
    for n in (20, 40, 80):
        x, v = oracle.run_he(x0, v0, m, 0.01, 0.0, EDS, a0, a1, n)
        ev.append(np.abs(v - v_exact).max())
        ex.append(np.abs(x - x_exact).max())
    for e in (ev, ex):
        r1, r2 = e[0] / e[1], e[1] / e[2]
        assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, e


def _kepler_state(e, t):
    Mn = t
    E = Mn
    for _ in range(60):
        E -= (E - e * math.sin(E) - Mn) / (1 - e * math.cos(E))
    r = np.array([math.cos(E) - e, math.sqrt(1 - e * e) * math.sin(E), 0.0])
    Edot = 1.0 / (1 - e * math.cos(E))
    rv = np.array([-math.sin(E) * Edot, math.sqrt(1 - e * e) * math.cos(E) * Edot, 0.0])
    return np.stack([-0.5 * r, 0.5 * r], axis=1), np.stack([-0.5 * rv, 0.5 * rv], axis=1)


def test_static_limit_kepler_and_reversibility():
    m = np.array([0.5, 0.5])
    x0, v0 = _kepler_state(0.5, 0.0)
    xT, _ = _kepler_state(0.5, 2 * math.pi)
    errs = []
    for n in (200, 400, 800):
        x, v = oracle.run_he(x0, v0, m, 0.0, 1.0, STATIC, 1.0, 2 * math.pi, n)
        errs.append(np.linalg.norm(x - xT))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs
    # reverse the velocities and step back: the start returns to roundoff
    x1, v1 = oracle.run_he(x0, v0, m, 0.0, 1.0, STATIC, 1.0, 3.0, 300)
    xb, vb = oracle.run_he(x1, -v1, m, 0.0, 1.0, STATIC, 1.0, 3.0, 300)
    assert np.max(np.abs(xb - x0)) < 1e-12 and np.max(np.abs(vb + v0)) < 1e-12


def test_layzer_irvine_second_order_and_agreement_with_kdk():
    w = eds_lattice(6, seed=1)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    res, diff = [], []
    for n in (16, 32, 64):
        x, v, d = oracle.run_he(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 0.4, n,
                                diag=True)
        res.append(abs(d["LI"][-1]))
        xk, vk = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 0.4, n)
        diff.append(np.abs(x - xk).max())
    for e in (res, diff):
        r1, r2 = e[0] / e[1], e[1] / e[2]
        assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, e
    # the rows are consistent: E - E0 + trapezoid of (2K + U) in ln a
    E = d["K"] + d["U"]
    src = 2 * d["K"] + d["U"]
    trap = np.concatenate([[0.0], np.cumsum(0.5 * (src[1:] + src[:-1]) * np.diff(np.log(d["a"])))])
    assert np.allclose(d["LI"], E - E[0] + trap, rtol=0, atol=1e-12 * np.abs(E).max())


def test_resume_matches_single_run():
    x0, m = random_cloud(20, 7, scale=0.3)
    v0 = 0.2 * np.random.default_rng(8).standard_normal((3, 20))
    args = (m, 0.03, 1.0, LCDM, 0.2, 1.0, 10)
    xa, va = oracle.run_he(x0, v0, *args)
    xh, vh = oracle.run_he(x0, v0, *args, first_step=0, last_step=4)
    xb, vb = oracle.run_he(xh, vh, *args, first_step=4, last_step=10)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
