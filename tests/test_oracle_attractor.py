"""Pins of the oracle's Eq. (10) deformation attractor (fixed point of
strength S = C psi at x_psi, softened with eps, attractive sign of Eq. (1)).

* The paper notes the term acts like a mass particle at a fixed position: the
  attractor's field, potential and transpose Jacobian equal the pair sum's
  for a phantom particle of mass S/G at x_psi (with zero cotangent), rows of
  the real particles -- the pair sum being pinned on its own elsewhere.  G is
  not 1 so that a stray G in the attractor would show.
* The transpose Jacobian against central differences of the field.
* A particle on a circular orbit about the attractor (static limit) returns
  after one period with second-order convergence; its energy K + U, with the
  external potential counted once (not halved), has no secular drift.
* Expanding background: the Layzer-Irvine residual still converges at second
  order with the attractor on (the external potential scales as 1/a too).
* The adjoint, including d/dS and d/dx_psi, against Richardson-extrapolated
  central differences of the oracle run.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1208_3444_amd.inputs import EDS, LCDM, eds_lattice, random_cloud

STATIC = {"H0": 0.0, "Om_R": 0.0, "Om_M": 0.0, "Om_K": 0.0, "Om_L": 0.0}
ATT = (0.37, (0.11, -0.23, 0.05))


def _phantom(x, m, att, G):
    S, xp = att
    xe = np.concatenate([x, np.asarray(xp, float).reshape(3, 1)], axis=1)
    me = np.concatenate([m, [S / G]])
    return xe, me


@pytest.mark.parametrize("eps", [0.02, 0.0])
def test_field_and_potential_equal_a_fixed_phantom_particle(eps):
    x, m = random_cloud(60, 3, scale=0.5)
    G, a = 1.7, 0.6
    xe, me = _phantom(x, m, ATT, G)
    got = oracle.forces(x, m, eps, G=G, a=a, attractor=ATT)
    ref = oracle.forces(xe, me, eps, G=G, a=a)[:, :60]
    assert np.allclose(got, ref, rtol=1e-13, atol=0)
    phi = oracle.potential(x, m, eps, G=G, attractor=ATT)
    pref = oracle.potential(xe, me, eps, G=G)[:60]
    assert np.allclose(phi, pref, rtol=1e-13, atol=0)
    # the field alone: attractive, strength S, 1/r^2 far away
    f, ph = oracle.attractor_field(np.array([[10.0], [0.0], [0.0]]), 0.0, (2.0, (0.0, 0.0, 0.0)))
    assert f[0, 0] == pytest.approx(-2.0 / 100.0, rel=1e-15) and ph[0] == pytest.approx(-0.2)


def test_vjp_equals_phantom_pair_vjp_and_finite_differences():
    x, m = random_cloud(40, 4, scale=0.5)
    G, eps = 1.3, 0.03
    lam = np.random.default_rng(1).standard_normal((3, 40))
    xe, me = _phantom(x, m, ATT, G)
    le = np.concatenate([lam, np.zeros((3, 1))], axis=1)
    got = oracle.force_vjp(x, m, lam, eps, G=G, attractor=ATT)
    ref = oracle.force_vjp(xe, me, le, eps, G=G)[:, :40]
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # attractor part alone against central differences of its field
    av = oracle.attractor_vjp(x, lam, eps, ATT)
    h = 1e-6
    for k in (0, 7, 39):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[c, k] += h
            xm[c, k] -= h
            fp = oracle.attractor_field(xp, eps, ATT)[0]
            fm = oracle.attractor_field(xm, eps, ATT)[0]
            fd = np.sum(lam * (fp - fm)) / (2 * h)
            assert av[c, k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def _circular(r, S):
    w = math.sqrt(S / r ** 3)
    return np.array([[r], [0.0], [0.0]]), np.array([[0.0], [r * w], [0.0]]), 2 * math.pi / w


def test_circular_orbit_second_order_and_energy():
    S, r = 1.5, 0.8
    att = (S, (0.0, 0.0, 0.0))
    x0, v0, T = _circular(r, S)
    m = np.array([1e-3])
    errs = []
    for n in (100, 200, 400):
        x, v = oracle.run(x0, v0, m, 0.0, 0.0, STATIC, 1.0, T, n, attractor=att)
        errs.append(np.linalg.norm(x - x0))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs
    # energy of an eccentric orbit over ten periods: bounded, no drift; with
    # the external potential halved it would not be conserved at all
    v0e = 0.8 * v0
    n = 4000
    _, _, d = oracle.run(x0, v0e, m, 0.0, 0.0, STATIC, 1.0, 10 * T, n, diag=True, attractor=att)
    E = d["K"] + d["U"]
    E0 = 0.5 * m[0] * np.sum(v0e ** 2) - m[0] * S / r
    assert E[0] == pytest.approx(E0, rel=1e-14)
    assert np.max(np.abs(E - E0)) < 1e-3 * abs(E0)
    first, last = np.abs(E[: n // 10] - E0).max(), np.abs(E[-n // 10:] - E0).max()
    assert last < 1.5 * first
    assert np.allclose(d["LI"], E - E[0], atol=1e-15)
    Lz = d["Lz"]
    assert np.max(np.abs(Lz - Lz[0])) < 1e-15  # central force about the origin


def test_layzer_irvine_second_order_with_attractor():
    w = eds_lattice(6, seed=1)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    # outside the box: a smooth tidal pull (an attractor inside would be
    # met at close range, where encounters, not the step, set the residual)
    att = (0.3, (1.6, 0.4, 0.5))
    res = []
    for n in (16, 32, 64):
        _, _, d = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 0.4, n,
                             diag=True, attractor=att)
        res.append(abs(d["LI"][-1]))
    r1, r2 = res[0] / res[1], res[1] / res[2]
    assert 3.7 < r1 < 4.3 and 3.85 < r2 < 4.15, res
    # the attractor's energy is in U (a run without it differs)
    _, _, d0 = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 0.4, 16, diag=True)
    assert abs(d0["U"][0] - d["U"][0]) > 0.1 * abs(d0["U"][0])


def test_adjoint_with_attractor_matches_central_differences():
    x0, m = random_cloud(24, 31, scale=0.5)
    v0 = 0.3 * np.random.default_rng(3).standard_normal((3, 24))
    tracers = np.array([0, 5, 9, 17])
    eps, G, n = 0.03, 0.2, 10
    S, xp = 0.15, np.array([0.1, -0.2, 0.05])

    def loss(x, v, S_, xp_):
        _, vN = oracle.run(x, v, m, eps, G, LCDM, 0.2, 1.0, n, attractor=(S_, xp_))
        return float(np.sum(vN[:, tracers] ** 2))

    xN, vN = oracle.run(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n, attractor=(S, xp))
    lv = np.zeros_like(vN)
    lv[:, tracers] = 2 * vN[:, tracers]
    gx, gv, xN2, vN2, ga = oracle.adjoint(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n,
                                          np.zeros_like(xN), lv, attractor=(S, xp))
    assert np.array_equal(xN2, xN) and np.array_equal(vN2, vN)

    def rich(fun):
        fd = [(fun(h) - fun(-h)) / (2 * h) for h in (1e-5, 5e-6)]
        assert abs(fd[1] - fd[0]) < 1e-4 * max(abs(fd[1]), 1e-12)
        return (4 * fd[1] - fd[0]) / 3

    rng = np.random.default_rng(4)
    ux, uv = rng.standard_normal(x0.shape), rng.standard_normal(v0.shape)
    nrm = math.sqrt(np.sum(ux ** 2) + np.sum(uv ** 2))
    ux, uv = ux / nrm, uv / nrm
    r = rich(lambda h: loss(x0 + h * ux, v0 + h * uv, S, xp))
    assert np.sum(gx * ux) + np.sum(gv * uv) == pytest.approx(r, rel=1e-7)
    r = rich(lambda h: loss(x0, v0, S + h, xp))
    assert ga[0] == pytest.approx(r, rel=1e-7)
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1.0
        r = rich(lambda h: loss(x0, v0, S, xp + h * e))
        assert ga[1 + c] == pytest.approx(r, rel=1e-6, abs=1e-10)


def test_no_attractor_is_the_plain_run():
    x0, m = random_cloud(16, 5, scale=0.3)
    v0 = 0.1 * np.random.default_rng(5).standard_normal((3, 16))
    a = oracle.run(x0, v0, m, 0.05, 1.0, EDS, 0.1, 1.0, 6)
    b = oracle.run(x0, v0, m, 0.05, 1.0, EDS, 0.1, 1.0, 6, attractor=(0.0, (0.0, 0.0, 0.0)))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
