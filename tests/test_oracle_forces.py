"""Pins of the oracle's pair sums (Eq. (1)) to things other than itself.

* the negative gradient of the softened potential energy, differentiated
  numerically in 50-digit arithmetic (fixes the sign and the formula),
* closed forms: two bodies, eight bodies on the vertices of a cube, the
  large-softening harmonic limit,
* invariants: total momentum, translation, scaling, linearity in G and m,
  permutation equivariance, the a^-3 factor,
* the transpose-Jacobian product against finite differences of the forces
  (dot-product test) and its symmetry at equal masses.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_1208_3444_amd.inputs import random_cloud


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _mp_energy(X, m, eps, G):
    """Softened pair potential energy -G sum_{j<k} m_j m_k / sqrt(r^2 + eps^2)."""
    N = len(m)
    W = mp.mpf(0)
    for k in range(N):
        for j in range(k + 1, N):
            r2 = sum((X[c][j] - X[c][k]) ** 2 for c in range(3)) + mp.mpf(eps) ** 2
            W -= G * m[j] * m[k] / mp.sqrt(r2)
    return W


@pytest.mark.parametrize("N,eps,seed", [(2, 0.1, 0), (5, 0.05, 1), (8, 0.02, 2), (7, 0.0, 3)])
def test_force_equals_minus_gradient_of_energy(N, eps, seed):
    mp.mp.dps = 50
    x, m = random_cloud(N, seed, scale=0.5)
    G = 1.3
    X = [[mp.mpf(float(v)) for v in x[c]] for c in range(3)]
    M = [mp.mpf(float(v)) for v in m]
    ref = np.zeros((3, N))
    for k in range(N):
        for c in range(3):
            def W_of(t, k=k, c=c):
                Y = [row[:] for row in X]
                Y[c][k] = t
                return _mp_energy(Y, M, eps, G)
            ref[c, k] = float(-mp.diff(W_of, X[c][k]) / M[k])
    got = oracle.forces(x, m, eps, G=G)
    for k in range(N):
        assert np.linalg.norm(got[:, k] - ref[:, k]) <= 1e-14 * np.linalg.norm(ref[:, k])


def test_two_body_closed_form():
    eps = 0.3
    x = np.array([[0.1, 0.9], [0.2, -0.4], [-0.3, 0.5]])
    m = np.array([0.7, 0.2])
    G, a = 2.0, 0.5
    acc = oracle.forces(x, m, eps, G=G, a=a)
    d = x[:, 1] - x[:, 0]
    r = np.linalg.norm(d)
    mag0 = G * m[1] * r / (r * r + eps * eps) ** 1.5 / a ** 3
    mag1 = G * m[0] * r / (r * r + eps * eps) ** 1.5 / a ** 3
    assert _rel(acc[:, 0], mag0 * d / r) < 1e-15
    assert _rel(acc[:, 1], -mag1 * d / r) < 1e-15


def test_cube_vertices_closed_form():
    s, eps, m0, G = 0.7, 0.11, 0.125, 1.0
    verts = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float).T * s
    m = np.full(8, m0)
    acc = oracle.forces(verts, m, eps, G=G)
    mag = G * m0 * s * (math.sqrt(3) / (s * s + eps * eps) ** 1.5
                        + 2 * math.sqrt(3) / (2 * s * s + eps * eps) ** 1.5
                        + math.sqrt(3) / (3 * s * s + eps * eps) ** 1.5)
    centre = np.full(3, 0.5 * s)
    for k in range(8):
        to_c = centre - verts[:, k]
        expect = mag * to_c / np.linalg.norm(to_c)
        assert _rel(acc[:, k], expect) < 1e-15
    # potential closed form: each vertex sees 3 edges, 3 face and 1 body diagonal
    phi = oracle.potential(verts, m, eps, G=G)
    expect_phi = -G * m0 * (3 / math.sqrt(s * s + eps * eps) + 3 / math.sqrt(2 * s * s + eps * eps)
                            + 1 / math.sqrt(3 * s * s + eps * eps))
    assert np.allclose(phi, expect_phi, rtol=1e-15, atol=0)


def test_large_softening_harmonic_limit():
    x, m = random_cloud(12, 5, scale=1e-2)
    G = 1.0
    errs = []
    for eps in (1.0, 2.0, 4.0):
        acc = oracle.forces(x, m, eps, G=G)
        harm = np.zeros_like(acc)
        for k in range(12):
            for j in range(12):
                if j != k:
                    harm[:, k] += G * m[j] * (x[:, j] - x[:, k]) / eps ** 3
        errs.append(_rel(acc, harm))
    # relative correction is O(r^2/eps^2): quarter per doubling of eps
    assert errs[0] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_momentum_and_invariances():
    x, m = random_cloud(64, 7, scale=0.5)
    eps, G = 0.03, 1.0
    g = oracle.forces(x, m, eps, G=G)
    term_scale = np.abs(g).sum() * m.max()
    assert np.all(np.abs((m * g).sum(axis=1)) < 1e-14 * term_scale)
    # translation
    g_t = oracle.forces(x + np.array([[0.37], [-0.21], [1.5]]), m, eps, G=G)
    assert _rel(g_t, g) < 1e-13
    # scaling x -> lam x, eps -> lam eps  =>  g -> g / lam^2
    lam = 2.5
    assert _rel(oracle.forces(lam * x, m, lam * eps, G=G), g / lam ** 2) < 1e-14
    # linear in G and in m
    assert _rel(oracle.forces(x, m, eps, G=3.0), 3.0 * g) < 1e-15
    assert _rel(oracle.forces(x, 0.25 * m, eps, G=G), 0.25 * g) < 1e-15
    # a^-3 factor
    assert _rel(oracle.forces(x, m, eps, G=G, a=0.2), g / 0.2 ** 3) < 1e-14
    # permutation equivariance
    perm = np.random.default_rng(0).permutation(64)
    assert _rel(oracle.forces(x[:, perm], m[perm], eps, G=G), g[:, perm]) < 1e-14
    # the subset entry point gives the same targets
    t = np.array([3, 17, 40, 63])
    assert _rel(oracle.forces_targets(x, m, t, eps, G=G, a=0.4), g[:, t] / 0.4 ** 3) < 1e-14


def test_potential_gradient_matches_force():
    x, m = random_cloud(16, 9, scale=0.5)
    eps, G = 0.05, 1.0
    g = oracle.forces(x, m, eps, G=G)

    def W(xx):
        return 0.5 * np.sum(m * oracle.potential(xx, m, eps, G=G))

    h = 1e-5
    for k in (0, 7, 15):
        for c in range(3):
            xp = x.copy(); xp[c, k] += h
            xm = x.copy(); xm[c, k] -= h
            dW = (W(xp) - W(xm)) / (2 * h)
            assert abs(-dW / m[k] - g[c, k]) < 1e-7 * np.linalg.norm(g[:, k])


def _jvp_fd(x, m, eps, G, u, h=1e-6):
    return (oracle.forces(x + h * u, m, eps, G=G) - oracle.forces(x - h * u, m, eps, G=G)) / (2 * h)


def test_force_vjp_dot_product():
    x, m = random_cloud(24, 11, scale=0.5)
    eps, G = 0.05, 1.7
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal((3, 24))
        w = rng.standard_normal((3, 24))
        lhs = np.sum(_jvp_fd(x, m, eps, G, u) * w)
        rhs = np.sum(u * oracle.force_vjp(x, m, w, eps, G=G))
        assert abs(lhs - rhs) <= 1e-7 * abs(rhs)


def test_force_vjp_columns_by_finite_differences():
    x, m = random_cloud(6, 12, scale=0.5)
    eps, G = 0.1, 1.0
    N = 6
    J = np.zeros((3 * N, 3 * N))
    for k in range(N):
        for c in range(3):
            u = np.zeros((3, N)); u[c, k] = 1.0
            J[:, c * N + k] = _jvp_fd(x, m, eps, G, u).reshape(-1)
    lam = np.random.default_rng(5).standard_normal((3, N))
    vjp = oracle.force_vjp(x, m, lam, eps, G=G).reshape(-1)
    assert _rel(vjp, J.T @ lam.reshape(-1)) < 1e-8


def test_force_jacobian_symmetric_at_equal_mass():
    x, _ = random_cloud(10, 13, scale=0.5)
    m = np.full(10, 0.1)
    eps, G = 0.05, 1.0
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((3, 10))
    # J symmetric  =>  J^T lam == J lam
    assert _rel(oracle.force_vjp(x, m, lam, eps, G=G), _jvp_fd(x, m, eps, G, lam)) < 1e-7
