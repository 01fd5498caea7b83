"""Pins of the oracle's Eq. (6) background term, b (x - c) added to the
comoving sum with b = Om_M H0^2 / 2 (the mean matter density's pull
removed about the centre c).

* Shell theorem: inside a uniform sphere of the background density the pair
  field is -b (x - c), so with the term the field and the potential's
  variation vanish (up to the lattice's discreteness), and the unperturbed
  sphere stays where it is over an EdS or Lambda-CDM run, while without the
  term it collapses.
* Linear growth: a uniform compression of that sphere is a top-hat
  perturbation; with the growing-mode velocity f H psi it grows as D(a),
  the growing solution of the linear growth equation, integrated here with
  scipy from Eq. (2) (EdS: D = a).
* The Layzer-Irvine residual, with the term's energy in U, still converges
  at second order; the transpose Jacobian (b I) against central differences
  of the field; the adjoint against Richardson differences of the run.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_1208_3444_amd.inputs import EDS, LCDM, eds_lattice, random_cloud

D_SPACING = 1.0 / 16


def _sphere(nR):
    """Cubic lattice points (spacing d) within radius nR d of the origin, unit
    comoving density; returns x, m, r."""
    g = np.arange(-nR, nR + 1) * D_SPACING
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    r = np.sqrt((pts ** 2).sum(axis=0))
    keep = r <= nR * D_SPACING
    x = pts[:, keep]
    return x, np.full(x.shape[1], D_SPACING ** 3), r[keep]


def _cos(cos):
    return tuple(cos[k] for k in ("H0", "Om_R", "Om_M", "Om_K", "Om_L"))


def test_coefficient_is_the_mean_density_pull():
    # both recipes have unit comoving mean density with G = 1
    for cos in (EDS, LCDM):
        assert oracle.background_coefficient(cos) == pytest.approx(4 * math.pi / 3, rel=1e-14)
    f, phi = oracle.background_field(np.array([[1.0, 0.5], [0.0, 0.5], [0.0, 0.5]]),
                                     (2.0, (0.5, 0.5, 0.5)))
    # pushes away from the centre, potential a downward parabola
    assert f[0, 0] > 0 and np.all(f[:, 1] == 0) and phi[0] < 0 and phi[1] == 0


def test_shell_theorem_cancellation():
    x, m, r = _sphere(8)
    b = 4 * math.pi / 3
    inner = r < 0.5 * 8 * D_SPACING
    eps = 0.5 * D_SPACING
    g0 = oracle.forces(x, m, eps)
    g = oracle.forces(x, m, eps, background=(b, (0.0, 0.0, 0.0)))
    n0 = np.linalg.norm(g0[:, inner], axis=0)
    n1 = np.linalg.norm(g[:, inner], axis=0)
    assert n1.max() < 0.02 * n0.mean()
    p0 = oracle.potential(x, m, eps)
    p1 = oracle.potential(x, m, eps, background=(b, (0.0, 0.0, 0.0)))
    assert np.ptp(p1[inner]) < 0.01 * np.ptp(p0[inner])
    # a = 2 scales both terms alike
    g2 = oracle.forces(x, m, eps, a=2.0, background=(b, (0.0, 0.0, 0.0)))
    assert np.allclose(g2, g / 8, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("cos,a0", [(EDS, 0.1), (LCDM, 0.2)])
def test_unperturbed_sphere_stays_and_compression_grows_as_D(cos, a0):
    x, m, r = _sphere(8)
    inner = r < 0.6 * 8 * D_SPACING
    eps = 0.1 * D_SPACING
    bg = (oracle.background_coefficient(cos), (0.0, 0.0, 0.0))
    a1, n = 1.0 if cos is LCDM else 0.4, 32
    v0 = np.zeros_like(x)
    xs, _ = oracle.run(x, v0, m, eps, 1.0, cos, a0, a1, n, background=bg)
    assert np.abs(xs - x)[:, inner].max() < 0.1 * D_SPACING
    xc, _ = oracle.run(x, v0, m, eps, 1.0, cos, a0, a1, n)
    assert np.abs(xc - x)[:, inner].max() > 1.0 * D_SPACING  # collapses without it

    # linear growth equation in ln a, H from Eq. (2):
    # D'' + (2 + dlnH/dlna) D' = (3/2) Om_M H0^2 / (a^3 H^2) D
    H0, Om = cos["H0"], cos["Om_M"]

    def H(a):
        return H0 * math.sqrt(cos["Om_R"] / a ** 4 + Om / a ** 3 + cos["Om_K"] / a ** 2
                              + cos["Om_L"])

    def rhs(s, y):
        a = math.exp(s)
        h = 1e-6
        dlnH = (math.log(H(a * math.exp(h))) - math.log(H(a * math.exp(-h)))) / (2 * h)
        return [y[1], -(2 + dlnH) * y[1] + 1.5 * Om * H0 ** 2 / (a ** 3 * H(a) ** 2) * y[0]]

    sol = solve_ivp(rhs, [math.log(1e-3), 0.0], [1e-3, 1e-3], rtol=1e-11, atol=1e-16,
                    dense_output=True)
    D0, dD0 = sol.sol(math.log(a0))
    D1 = sol.sol(math.log(a1))[0]
    if cos is EDS:
        assert D1 / D0 == pytest.approx(a1 / a0, rel=1e-6)
    A = 1e-3
    psi = -A * x
    xp, _ = oracle.run(x + psi, (dD0 / D0) * H(a0) * psi, m, eps, 1.0, cos, a0, a1, n,
                       background=bg)
    dd = xp - xs
    ratio = (dd[:, inner] * psi[:, inner]).sum() / (psi[:, inner] ** 2).sum()
    assert ratio == pytest.approx(D1 / D0, rel=2e-3)


def test_layzer_irvine_second_order_with_background():
    w = eds_lattice(6, seed=1)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    bg = (oracle.background_coefficient(w.cosmo), (0.5, 0.5, 0.5))
    res = []
    for n in (16, 32, 64):
        _, _, d = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 1.0, n, diag=True,
                             background=bg)
        res.append(abs(d["LI"][-1]))
    r1, r2 = res[0] / res[1], res[1] / res[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, res
    # with the term the open lattice no longer collapses by a = 1, so the
    # whole run is smooth; its energy is in U
    _, _, d0 = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, 1.0, 16, diag=True)
    assert abs(d0["U"][0] - d["U"][0]) > 1e-3 * abs(d0["U"][0])


def test_vjp_against_central_differences():
    x, m = random_cloud(30, 6, scale=0.5)
    lam = np.random.default_rng(2).standard_normal((3, 30))
    bg = (1.7, (0.2, -0.1, 0.3))
    got = oracle.force_vjp(x, m, lam, 0.03, G=0.8, background=bg)
    h = 1e-6
    for k in (0, 11, 29):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[c, k] += h
            xm[c, k] -= h
            fp = oracle.forces(xp, m, 0.03, G=0.8, background=bg)
            fm = oracle.forces(xm, m, 0.03, G=0.8, background=bg)
            fd = np.sum(lam * (fp - fm)) / (2 * h)
            assert got[c, k] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_adjoint_with_background_matches_central_differences():
    x0, m = random_cloud(20, 21, scale=0.5)
    v0 = 0.3 * np.random.default_rng(5).standard_normal((3, 20))
    eps, G, n = 0.03, 0.2, 8
    bg = (0.9, (0.1, 0.0, -0.1))
    tracers = np.array([1, 7, 13])

    def loss(x, v):
        xN, vN = oracle.run(x, v, m, eps, G, LCDM, 0.2, 1.0, n, background=bg)
        return float(np.sum(xN[:, tracers] ** 2) + np.sum(vN[:, tracers] ** 2))

    xN, vN = oracle.run(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n, background=bg)
    lx, lv = np.zeros_like(xN), np.zeros_like(vN)
    lx[:, tracers] = 2 * xN[:, tracers]
    lv[:, tracers] = 2 * vN[:, tracers]
    gx, gv, xN2, _ = oracle.adjoint(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n, lx, lv,
                                    background=bg)
    assert np.array_equal(xN2, xN)
    rng = np.random.default_rng(6)
    ux, uv = rng.standard_normal(x0.shape), rng.standard_normal(v0.shape)
    nrm = math.sqrt(np.sum(ux ** 2) + np.sum(uv ** 2))
    ux, uv = ux / nrm, uv / nrm
    fd = [(loss(x0 + h * ux, v0 + h * uv) - loss(x0 - h * ux, v0 - h * uv)) / (2 * h)
          for h in (1e-5, 5e-6)]
    rich = (4 * fd[1] - fd[0]) / 3
    assert np.sum(gx * ux) + np.sum(gv * uv) == pytest.approx(rich, rel=1e-7)
    # the term changes the gradient (it is really in the reverse sweep)
    gx0 = oracle.adjoint(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n, lx, lv)[0]
    assert np.abs(gx0 - gx).max() > 1e-3 * np.abs(gx).max()
