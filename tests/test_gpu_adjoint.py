"""GPU parity of the hand-written adjoint: the transpose-Jacobian pair sweep
and the checkpointed reverse sweep of the run, against the FP64 oracle and
central finite differences of the GPU forward, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import to_dev

pytestmark = pytest.mark.gpu

LCDM = inputs.LCDM


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("C", [1, 4, 11])
def test_force_vjp_matches_oracle(dev, C):
    x, m = inputs.random_cloud(700, 8, scale=0.5)
    eps, G = 0.02, 1.3
    lam = np.random.default_rng(C).standard_normal((C, 3, 700))
    xt, mt, lt = to_dev(x, dev), to_dev(m, dev), to_dev(lam, dev)
    got64 = colatus.force_vjp(xt, mt, lt, eps, G, precision="fp64").cpu().numpy()
    gotmx = colatus.force_vjp(xt, mt, lt, eps, G, precision="mixed_f64acc").cpu().numpy()
    for c in range(C):
        ref = oracle.force_vjp(x, m, lam[c], eps, G=G)
        assert _rel(got64[c], ref) <= 1e-12
        assert _rel(gotmx[c], ref) <= 1e-5


def test_adjoint_fp64_matches_oracle_and_checkpoints_are_exact(dev):
    x0, m = inputs.random_cloud(96, 12, scale=0.5)
    v0 = 0.3 * np.random.default_rng(1).standard_normal((3, 96))
    eps, G, n = 0.03, 0.5, 12
    rng = np.random.default_rng(2)
    lx = rng.standard_normal((2, 3, 96))
    lv = rng.standard_normal((2, 3, 96))
    gx_r, gv_r, xN_r, vN_r = oracle.adjoint(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n, lx, lv)
    args = [to_dev(a, dev) for a in (x0, v0, m)]
    outs = []
    for K in (1, 5, 12, 0, -1):  # 0: every position kept; -1: the library chooses
        gx, gv, xN, vN = colatus.adjoint(*args, eps, G, LCDM, 0.2, 1.0, n, to_dev(lx, dev),
                                         to_dev(lv, dev), checkpoint_every=K, precision="fp64",
                                         return_state=True)
        outs.append((gx.cpu().numpy(), gv.cpu().numpy()))
        assert np.max(np.abs(xN.cpu().numpy() - xN_r)) <= 1e-12
        assert np.max(np.abs(vN.cpu().numpy() - vN_r)) <= 1e-11 * np.abs(vN_r).max()
    for gx, gv in outs:
        assert _rel(gx, gx_r) <= 1e-10 and _rel(gv, gv_r) <= 1e-10
    # recomputation from checkpoints is bitwise: any K gives the same bits
    for gx, gv in outs[1:]:
        assert np.array_equal(gx, outs[0][0]) and np.array_equal(gv, outs[0][1])


def test_adjoint_mixed_close_to_fp64_gradient(dev):
    w = inputs.lcdm_grf(8, seed=4, a_begin=0.2, n_steps=20)
    v0 = w.velocities(oracle.hubble(0.2, *w.cosmo.values()))
    tr = np.arange(0, w.N, 37)
    xN, vN = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, 0.2, 1.0, 20)
    lv = np.zeros((3, w.N))
    lv[:, tr] = 2 * vN[:, tr]
    lx = np.zeros((3, w.N))
    gx_r, gv_r, _, _ = oracle.adjoint(w.x, v0, w.m, w.eps, w.G, w.cosmo, 0.2, 1.0, 20, lx, lv)
    args = [to_dev(a, dev) for a in (w.x, v0, w.m)]
    for prec, tol in (("fp64", 1e-9), ("mixed_twosum", 1e-3)):
        gx, gv = colatus.adjoint(*args, w.eps, w.G, w.cosmo, 0.2, 1.0, 20, to_dev(lx, dev),
                                 to_dev(lv, dev), checkpoint_every=6, precision=prec)
        assert _rel(gx.cpu().numpy(), gx_r) <= tol, prec
        assert _rel(gv.cpu().numpy(), gv_r) <= tol, prec


def test_adjoint_matches_finite_differences_of_gpu_forward(dev):
    x0, m = inputs.random_cloud(200, 5, scale=0.5)
    v0 = 0.2 * np.random.default_rng(6).standard_normal((3, 200))
    eps, G, n = 0.03, 0.2, 16
    tr = np.array([3, 50, 120, 199])

    def loss(x, v):
        xt, vt, mt = to_dev(x, dev), to_dev(v, dev), to_dev(m, dev)
        colatus.run(xt, vt, mt, eps, G, LCDM, 0.2, 1.0, n, precision="fp64")
        vN = vt.cpu().numpy()
        return float(np.sum(vN[:, tr] ** 2)), vN

    L0, vN = loss(x0, v0)
    lv = np.zeros((3, 200))
    lv[:, tr] = 2 * vN[:, tr]
    gx, gv = colatus.adjoint(to_dev(x0, dev), to_dev(v0, dev), to_dev(m, dev), eps, G, LCDM,
                             0.2, 1.0, n, to_dev(np.zeros((3, 200)), dev), to_dev(lv, dev),
                             checkpoint_every=4, precision="fp64")
    gx, gv = gx.cpu().numpy(), gv.cpu().numpy()
    rng = np.random.default_rng(7)
    for _ in range(4):
        ux, uv = rng.standard_normal((3, 200)), rng.standard_normal((3, 200))
        nrm = math.sqrt(np.sum(ux ** 2) + np.sum(uv ** 2))
        ux, uv = ux / nrm, uv / nrm
        fd = []
        for h in (1e-5, 5e-6):
            fd.append((loss(x0 + h * ux, v0 + h * uv)[0] - loss(x0 - h * ux, v0 - h * uv)[0])
                      / (2 * h))
        rich = (4 * fd[1] - fd[0]) / 3
        ad = np.sum(gx * ux) + np.sum(gv * uv)
        assert abs(ad - rich) <= 1e-7 * abs(rich), (ad, fd)


def test_autograd_function(dev):
    x0, m = inputs.random_cloud(64, 9, scale=0.5)
    v0 = 0.1 * np.random.default_rng(3).standard_normal((3, 64))
    P = dict(eps=0.03, G=0.5, cosmo=LCDM, a_begin=0.2, a_end=1.0, n_steps=10,
             checkpoint_every=3, precision="fp64")
    xt = to_dev(x0, dev).requires_grad_(True)
    vt = to_dev(v0, dev).requires_grad_(True)
    mt = to_dev(m, dev)
    xN, vN = colatus.ColatusRun.apply(xt, vt, mt, P)
    L = (vN[:, :5] ** 2).sum() + xN[0].sum()
    L.backward()
    lx = np.zeros((3, 64)); lx[0] = 1.0
    lv = np.zeros((3, 64)); lv[:, :5] = 2 * vN[:, :5].detach().cpu().numpy()
    gx_r, gv_r, _, _ = oracle.adjoint(x0, v0, m, 0.03, 0.5, LCDM, 0.2, 1.0, 10, lx, lv)
    assert _rel(xt.grad.cpu().numpy(), gx_r) <= 1e-10
    assert _rel(vt.grad.cpu().numpy(), gv_r) <= 1e-10


def test_ftle_matches_oracle(dev):
    w = inputs.lcdm_grf(6, seed=4, a_begin=0.2, n_steps=12)
    v0 = w.velocities(oracle.hubble(0.2, *w.cosmo.values()))
    tracers = [0, 17, 100, 201]
    lt_r, ll_r, phi_r = oracle.ftle(w.x, v0, w.m, w.eps, w.G, w.cosmo, 0.2, 1.0, 12, tracers)
    args = [to_dev(a, dev) for a in (w.x, v0, w.m)]
    lt, ll, phi = (t.cpu().numpy() for t in colatus.ftle(*args, w.eps, w.G, w.cosmo, 0.2, 1.0,
                                                          12, tracers, checkpoint_every=5,
                                                          precision="fp64"))
    assert np.allclose(phi, phi_r, rtol=1e-9, atol=1e-12)
    assert np.allclose(lt, lt_r, rtol=1e-9) and np.allclose(ll, ll_r, rtol=1e-9)
    ltm = colatus.ftle(*args, w.eps, w.G, w.cosmo, 0.2, 1.0, 12, tracers, checkpoint_every=5,
                       precision="mixed_twosum")[0].cpu().numpy()
    assert np.max(np.abs(ltm - lt_r)) <= 1e-3 * max(1.0, np.abs(lt_r).max())


def test_ftle_singular_value_and_time_span_in_the_library(dev):
    """colatus_ftle's sigma_max (Jacobi on B^T B) against numpy's SVD of the
    blocks it returns, its time span against the diagnostics' t of the same
    run and against colatus_cosmic_time; the static limit; a tracer whose
    block is the identity (G = 0: free particles) has lambda = 0."""
    w = inputs.lcdm_grf(6, seed=4, a_begin=0.2, n_steps=12)
    v0 = w.velocities(oracle.hubble(0.2, *w.cosmo.values()))
    args = [to_dev(a, dev) for a in (w.x, v0, w.m)]
    tracers = [3, 50, 101, 150, 215]
    lt, ll, phi = (t.cpu().numpy() for t in colatus.ftle(*args, w.eps, w.G, w.cosmo, 0.2, 1.0,
                                                          12, tracers, checkpoint_every=4,
                                                          precision="fp64"))
    ls = np.log(np.linalg.svd(phi, compute_uv=False)[:, 0])
    d = colatus.run(args[0].clone(), args[1].clone(), args[2], w.eps, w.G, w.cosmo, 0.2, 1.0, 12,
                    precision="fp64", diag=True)
    span = colatus.cosmic_time(w.cosmo, 0.2, 1.0, 12)
    assert span == d["t"][-1]
    assert span == pytest.approx(oracle.time_integral("time", 0.2, 1.0, *w.cosmo.values()),
                                 rel=1e-13)
    assert np.allclose(lt, ls / span, rtol=1e-12, atol=0)
    assert np.allclose(ll, ls / math.log(1.0 / 0.2), rtol=1e-12, atol=0)
    # free particles: the flow map block is the identity
    lt0, ll0, phi0 = (t.cpu().numpy() for t in colatus.ftle(*args, w.eps, 0.0, w.cosmo, 0.2, 1.0,
                                                             12, tracers, precision="fp64"))
    assert np.allclose(phi0, np.broadcast_to(np.eye(3), phi0.shape), rtol=0, atol=1e-15)
    assert np.all(np.abs(lt0) <= 1e-14)
    # static limit: a held fixed, the span is the elapsed time, no ln a
    static = dict(H0=0.0, Om_R=0.0, Om_M=0.0, Om_K=0.0, Om_L=0.0)
    assert colatus.cosmic_time(static, 1.0, 2.5, 10) == pytest.approx(2.5, rel=1e-15)
    lts, lls, phis = (t.cpu().numpy() for t in colatus.ftle(*args, w.eps, w.G, static, 1.0, 0.3,
                                                             10, tracers, precision="fp64"))
    lr, _, phir = oracle.ftle(w.x, v0, w.m, w.eps, w.G, static, 1.0, 0.3, 10, tracers)
    assert np.allclose(phis, phir, rtol=1e-9, atol=1e-12)
    assert np.allclose(lts, lr, rtol=1e-9)
    assert np.all(np.isnan(lls))


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("N", [2, 3, 5])
def test_force_vjp_few_particles_self_pair_adds_nothing(dev, form, N):
    """With unequal masses the self pair's bracket m_k lam_k - m_k lam_k must be
    exactly 0 (both products rounded before the difference); a fused form
    leaves the rounding error of one product, which r^-3 = eps^-3 turns into
    an error that dominates sums over few particles."""
    x, m = inputs.random_cloud(N, 70 + N, scale=0.5)
    lam = np.random.default_rng(N).standard_normal((1, 3, N))
    xt, mt, lt = to_dev(x, dev), to_dev(m, dev), to_dev(lam, dev)
    ref = oracle.force_vjp(x, m, lam[0], 0.01)
    colatus.set_option(colatus.OPT_PAIR_FORM, form)
    try:
        for prec, tol in (("fp64", 1e-12), ("mixed_twosum", 1e-6), ("fp32", 1e-6)):
            got = colatus.force_vjp(xt, mt, lt, 0.01, 1.0, precision=prec).cpu().numpy()
            assert _rel(got[0], ref) <= tol, prec
    finally:
        colatus.set_option(colatus.OPT_PAIR_FORM, -1)


@pytest.mark.parametrize("prec", ["fp64", "mixed_twosum"])
def test_adjoint_of_a_batch_equals_each_box_alone(dev, prec):
    """Boxes of a batch do not interact: the batched adjoint's gradients of
    each box equal the adjoint of that box run alone (the same work items per
    box), and a cotangent on one box moves no other box's gradient."""
    sizes = [300, 1000, 77]
    xs, vs, ms, epss = [], [], [], []
    for k, n in enumerate(sizes):
        x, m = inputs.random_cloud(n, 400 + k, scale=0.6)
        xs.append(x)
        ms.append(m)
        vs.append(0.1 * np.random.default_rng(k).standard_normal((3, n)))
        epss.append(0.01 * (k + 1))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X, V, M = np.concatenate(xs, axis=1), np.concatenate(vs, axis=1), np.concatenate(ms)
    N = X.shape[1]
    rng = np.random.default_rng(9)
    lx = rng.standard_normal((2, 3, N))
    lv = rng.standard_normal((2, 3, N))
    lx[1, :, off[1]:] = 0.0  # second cotangent on box 0 only
    lv[1, :, off[1]:] = 0.0
    gx, gv = colatus.adjoint(to_dev(X, dev), to_dev(V, dev), to_dev(M, dev), 0.0, 1.0, LCDM,
                             0.3, 0.8, 9, to_dev(lx, dev), to_dev(lv, dev), checkpoint_every=4,
                             precision=prec, batch=(off, epss))
    gx, gv = gx.cpu().numpy(), gv.cpu().numpy()
    for k in range(len(sizes)):
        sl = slice(off[k], off[k + 1])
        bx, bv = colatus.adjoint(to_dev(xs[k], dev), to_dev(vs[k], dev), to_dev(ms[k], dev),
                                 epss[k], 1.0, LCDM, 0.3, 0.8, 9,
                                 to_dev(np.ascontiguousarray(lx[:, :, sl]), dev),
                                 to_dev(np.ascontiguousarray(lv[:, :, sl]), dev),
                                 checkpoint_every=4, precision=prec)
        assert _rel(gx[:, :, sl], bx.cpu().numpy()) <= 1e-13, k
        assert _rel(gv[:, :, sl], bv.cpu().numpy()) <= 1e-13, k
    assert np.all(gx[1, :, off[1]:] == 0.0) and np.all(gv[1, :, off[1]:] == 0.0)
