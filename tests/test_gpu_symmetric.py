"""GPU parity of the symmetric pair loop (pair-loop form 2) against the FP64 oracle.

Form 2 evaluates each unordered pair once and applies it to both particles
(the pair term of Eq. (1) is antisymmetric); boxes are cut into parts of
R x threads particles and every particle receives one partial sum per part.
Checked here for every supported shape: lattice and random clouds with
unequal masses and ragged sizes (missing targets and sources in the last
part), the potential, softening zero (coincident pairs masked), ragged
batches, the persistent grid, and the 32^3 LCDM workload on sampled targets.
Tolerances: the per-particle relative bars of the ordered loop (median 1e-6,
max 1e-4) on the lattice and the 32^3 workload; on random clouds the
conditioned error |a - a_ref| / sum_j |term_j| <= 5e-6.  Every partial sum
here is one FP32 sum of at most 256 terms (a target's from one part, a
source's reaction from one part), or, in the forward loop's 2x2 groups
(4 targets per lane, 64 threads), the FP32 sum of two such sums, whose
conditioned error is at most about (257 + 10) u = 1.6e-5 (u = 2^-24, 10 u
for the pair term itself); the largest value observed is 3.7e-6.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import rel_err_per_particle, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(4, 64), (8, 64), (4, 128)]


def _term_scale(x, m, eps):
    d = x[:, None, :] - x[:, :, None]
    s = (d ** 2).sum(axis=0) + eps * eps
    with np.errstate(divide="ignore"):  # eps = 0: the diagonal, cleared below
        w = m[None, :] * s ** -1.5
    np.fill_diagonal(w, 0.0)
    return (w * np.sqrt((d ** 2).sum(axis=0))).sum(axis=1)


def _gpu(x, m, eps, dev, prec, a=1.0, with_phi=False, batch=None):
    out = colatus.forces(to_dev(x, dev), to_dev(m, dev), eps, a=a, precision=prec,
                         with_phi=with_phi, batch=batch)
    torch.cuda.synchronize()
    if with_phi:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


@pytest.fixture
def form2():
    colatus.set_option(colatus.OPT_PAIR_FORM, 2)
    yield
    for k in (colatus.OPT_TILE_R, colatus.OPT_TILE_TPB):
        colatus.set_option(k, 0)
    colatus.set_option(colatus.OPT_PERSISTENT, 0)
    colatus.set_option(colatus.OPT_PAIR_FORM, -1)


def _shape(R, tpb):
    colatus.set_option(colatus.OPT_TILE_R, R)
    colatus.set_option(colatus.OPT_TILE_TPB, tpb)


@pytest.mark.parametrize("R,tpb", SHAPES)
def test_lattice_with_potential(dev, form2, R, tpb):
    _shape(R, tpb)
    cfg = colatus.tile_config(4096, "mixed_twosum")
    assert cfg == (R, tpb, -(-4096 // (R * tpb)), 2)
    w = inputs.eds_lattice(16)
    ref = oracle.forces(w.x, w.m, w.eps, a=0.1)
    pref = oracle.potential(w.x, w.m, w.eps)
    for prec, med, mx in (("mixed_twosum", 1e-6, 1e-4), ("mixed_f64acc", 1e-6, 1e-4),
                          ("fp32", 1e-5, 1e-3)):
        got, phi = _gpu(w.x, w.m, w.eps, dev, prec, a=0.1, with_phi=True)
        e = rel_err_per_particle(got, ref)
        ep = np.abs(phi - pref) / np.abs(pref)
        print(f"R={R} tpb={tpb} {prec}: force median {np.median(e):.2e} max {e.max():.2e}; "
              f"potential median {np.median(ep):.2e} max {ep.max():.2e}", flush=True)
        assert np.median(e) <= med and e.max() <= mx
        pm, px = (1e-6, 1e-5) if prec != "fp32" else (1e-5, 1e-4)
        assert np.median(ep) <= pm and ep.max() <= px


@pytest.mark.parametrize("R,tpb", SHAPES)
@pytest.mark.parametrize("N", [1, 2, 3, 63, 64, 65, 255, 257, 511, 513, 1000, 1537])
def test_ragged_unequal_masses(dev, form2, R, tpb, N):
    """Parts with missing targets/sources; unequal masses take the general loop."""
    _shape(R, tpb)
    x, m = inputs.random_cloud(N, 100 + N, scale=0.5, mass_spread=True)
    eps = 0.01
    got, phi = _gpu(x, m, eps, dev, "mixed_twosum", with_phi=True)
    if N == 1:
        assert np.all(got == 0.0)
        return
    ref = oracle.forces(x, m, eps)
    err = np.max(np.linalg.norm(got - ref, axis=0) / _term_scale(x, m, eps))
    pref = oracle.potential(x, m, eps)
    ep = np.max(np.abs(phi - pref) / np.abs(pref))
    print(f"R={R} tpb={tpb} N={N}: conditioned force error {err:.2e}, potential {ep:.2e}")
    assert err <= 5e-6 and ep <= 1e-5


def test_equal_and_unequal_masses_agree(dev, form2):
    """The equal-mass loop (mass factored out) and the general loop agree."""
    x, m = inputs.random_cloud(1300, 5, scale=0.5, mass_spread=False)
    assert np.all(m == m[0])
    eps = 0.02
    ref = oracle.forces(x, m, eps)
    got_eq = _gpu(x, m, eps, dev, "mixed_twosum")
    m2 = m.copy()
    m2[0] *= 1.0 + 2.0 ** -40  # not equal: the general loop runs
    got_ne = _gpu(x, m2, eps, dev, "mixed_twosum")
    sc = _term_scale(x, m, eps)
    assert np.max(np.linalg.norm(got_eq - ref, axis=0) / sc) <= 5e-6
    assert np.max(np.linalg.norm(got_ne - ref, axis=0) / sc) <= 5e-6


@pytest.mark.parametrize("R,tpb", SHAPES)
def test_softening_zero_masks_coincident_pairs(dev, form2, R, tpb):
    _shape(R, tpb)
    x, m = inputs.random_cloud(700, 7, scale=0.5)
    got = _gpu(x, m, 0.0, dev, "mixed_twosum")
    assert np.all(np.isfinite(got))
    err = np.max(np.linalg.norm(got - oracle.forces(x, m, 0.0), axis=0) / _term_scale(x, m, 0.0))
    assert err <= 1e-5


def test_batch_and_persistent_grid(dev, form2):
    sizes = [1, 40, 513, 2, 1030, 300]
    xs, ms, epss = [], [], []
    for i, n in enumerate(sizes):
        x, m = inputs.random_cloud(n, 60 + i, scale=0.5, mass_spread=bool(i % 2))
        xs.append(x + 0.1 * i)
        ms.append(m)
        epss.append(0.01 * (i + 1))
    x = np.concatenate(xs, axis=1)
    m = np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)])
    runs = {}
    for pers in (0, 1):
        colatus.set_option(colatus.OPT_PERSISTENT, pers)
        runs[pers] = _gpu(x, m, 0.0, dev, "mixed_twosum", a=0.5, with_phi=True,
                          batch=(off, np.array(epss)))
    # same items, same arithmetic: bitwise equal whatever the grid
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    got, phi = runs[0]
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        if sizes[b] == 1:
            assert np.all(got[:, sl] == 0.0)
            continue
        ref = oracle.forces(xs[b], ms[b], epss[b], a=0.5)
        scale = _term_scale(xs[b], ms[b], epss[b]) / 0.5 ** 3
        assert np.max(np.linalg.norm(got[:, sl] - ref, axis=0) / scale) <= 5e-6
        pref = oracle.potential(xs[b], ms[b], epss[b])
        assert np.max(np.abs(phi[sl] - pref) / np.abs(pref)) <= 1e-5
    # a box computed inside the batch equals the box computed alone
    alone = _gpu(xs[4], ms[4], epss[4], dev, "mixed_twosum", a=0.5)
    assert np.array_equal(alone, got[:, off[4]:off[5]])


def test_lcdm_32cubed_sampled(dev, form2):
    w = inputs.lcdm_grf(32)
    t = np.arange(0, w.N, 37)
    ref = oracle.forces_targets(w.x, w.m, t, w.eps, a=w.a_begin)
    a1 = _gpu(w.x, w.m, w.eps, dev, "mixed_twosum", a=w.a_begin)
    a2 = _gpu(w.x, w.m, w.eps, dev, "mixed_twosum", a=w.a_begin)
    assert np.array_equal(a1, a2)
    e = rel_err_per_particle(a1[:, t], ref)
    print(f"form 2 32^3: median {np.median(e):.3e} max {e.max():.3e}")
    assert np.median(e) <= 1e-6 and e.max() <= 1e-4


# ---- symmetric adjoint sweep (form 2, one cotangent per launch) -------------

def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("N,C,spread,eps", [(700, 1, True, 0.02), (700, 3, True, 0.02),
                                            (1000, 2, False, 0.02), (257, 1, True, 0.0),
                                            (65, 5, False, 0.01), (2, 1, True, 0.01)])
def test_force_vjp_symmetric_matches_oracle(dev, form2, N, C, spread, eps):
    """Transpose-Jacobian sweep M(d)(m_k lam_j - m_j lam_k), each unordered pair
    once: per cotangent against the oracle's VJP (relative 2-norm <= 1e-5, the
    ordered mixed loop's bar); ragged parts, unequal and equal masses,
    softening zero, more cotangents than the heuristic would send here."""
    x, m = inputs.random_cloud(N, 300 + N, scale=0.5, mass_spread=spread)
    G = 1.3
    lam = np.random.default_rng(C).standard_normal((C, 3, N))
    xt, mt, lt = to_dev(x, dev), to_dev(m, dev), to_dev(lam, dev)
    # Without softening the closest pairs' r^-5 terms dominate the sum, and
    # the FP32 separation of such a pair (coordinates rounded relative to a
    # part centre up to 0.5 away; the closest pair at N = 257 is 0.004 apart)
    # carries a relative error up to u |x - c| / r = 8e-6, amplified about
    # five times in M(d).
    tol = 1e-5 if eps > 0 else 5e-5
    for prec in ("mixed_twosum", "mixed_f64acc", "fp32"):
        got = colatus.force_vjp(xt, mt, lt, eps, G, precision=prec).cpu().numpy()
        assert np.all(np.isfinite(got))
        for c in range(C):
            ref = oracle.force_vjp(x, m, lam[c], eps, G=G)
            e = _rel(got[c], ref)
            print(f"N={N} C={C} {prec} cot {c}: {e:.2e}", flush=True)
            assert e <= tol


@pytest.mark.parametrize("spread", [False, True])
def test_force_vjp_symmetric_scales_exactly_with_the_cotangent(dev, form2, spread):
    """The sweep is linear in the cotangent and every operation on it is a
    product or sum with cotangent-free factors, so scaling lam by 2^80 or
    2^-60 scales the FP32 result exactly (no rounding changes, no overflow).
    On a ragged box (parts of 256, 256, 188: chunks with padding lanes) this
    also shows that no padding position (|d| ~ 1e18) meets an unscaled
    cotangent: d.u would overflow FP32 at |u| ~ 1e20 and the sum turn NaN."""
    N = 700
    x, m = inputs.random_cloud(N, 41, scale=0.5, mass_spread=spread)
    lam = np.random.default_rng(42).standard_normal((1, 3, N))
    xt, mt = to_dev(x, dev), to_dev(m, dev)
    for prec in ("mixed_twosum", "fp32"):
        base = colatus.force_vjp(xt, mt, to_dev(lam, dev), 0.02, 1.3, precision=prec)
        base = base.cpu().numpy()
        assert np.all(np.isfinite(base))
        for k in (80, -60):
            got = colatus.force_vjp(xt, mt, to_dev(lam * 2.0 ** k, dev), 0.02, 1.3,
                                    precision=prec).cpu().numpy()
            assert np.array_equal(got, base * 2.0 ** k), (prec, k)


def test_force_vjp_symmetric_is_the_default_for_few_cotangents(dev):
    """Boxes large enough to fill the GPU with symmetric items (about 11 000
    particles and more) take the symmetric adjoint loop by default, smaller
    ones the ordered loop; both give the oracle's VJP."""
    N = 12000
    assert colatus.tile_config(N, "mixed_twosum", kind=1)[3] == 2
    assert colatus.tile_config(700, "mixed_twosum", kind=1) == (1, 256, 3, 0)
    x, m = inputs.random_cloud(N, 9, scale=0.5)
    lam = np.random.default_rng(1).standard_normal((1, 3, N))
    xt, mt, lt = to_dev(x, dev), to_dev(m, dev), to_dev(lam, dev)
    a = colatus.force_vjp(xt, mt, lt, 0.02, 1.0, precision="mixed_twosum").cpu().numpy()
    colatus.set_option(colatus.OPT_PAIR_FORM, 0)
    try:
        b = colatus.force_vjp(xt, mt, lt, 0.02, 1.0, precision="mixed_twosum").cpu().numpy()
    finally:
        colatus.set_option(colatus.OPT_PAIR_FORM, -1)
    ref = oracle.force_vjp(x, m, lam[0], 0.02)
    assert _rel(a[0], ref) <= 1e-5 and _rel(b[0], ref) <= 1e-5
    assert not np.array_equal(a, b)  # the two loops really differ


def test_adjoint_run_symmetric_close_to_fp64_gradient(dev, form2):
    w = inputs.lcdm_grf(8, seed=4, a_begin=0.2, n_steps=20)
    v0 = w.velocities(oracle.hubble(0.2, *w.cosmo.values()))
    tr = np.arange(0, w.N, 37)
    xN, vN = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, 0.2, 1.0, 20)
    lv = np.zeros((3, w.N))
    lv[:, tr] = 2 * vN[:, tr]
    lx = np.zeros((3, w.N))
    gx_r, gv_r, _, _ = oracle.adjoint(w.x, v0, w.m, w.eps, w.G, w.cosmo, 0.2, 1.0, 20, lx, lv)
    args = [to_dev(a, dev) for a in (w.x, v0, w.m)]
    gx, gv = colatus.adjoint(*args, w.eps, w.G, w.cosmo, 0.2, 1.0, 20, to_dev(lx, dev),
                             to_dev(lv, dev), checkpoint_every=6, precision="mixed_twosum")
    assert _rel(gx.cpu().numpy(), gx_r) <= 1e-3
    assert _rel(gv.cpu().numpy(), gv_r) <= 1e-3


# ---- FP64 pairs in the symmetric loops ----------------------------------------

@pytest.mark.parametrize("R,tpb", [(4, 64), (2, 128)])
def test_fp64_symmetric_forces(dev, form2, R, tpb):
    """FP64 symmetric loop at the FP64 parity bar: lattice (median and max
    1e-12, potential too), ragged random clouds with unequal masses (conditioned
    1e-14), softening zero."""
    _shape(R, tpb)
    assert colatus.tile_config(4096, "fp64") == (R, tpb, -(-4096 // (R * tpb)), 2)
    w = inputs.eds_lattice(16)
    got, phi = _gpu(w.x, w.m, w.eps, dev, "fp64", a=0.1, with_phi=True)
    e = rel_err_per_particle(got, oracle.forces(w.x, w.m, w.eps, a=0.1))
    pref = oracle.potential(w.x, w.m, w.eps)
    ep = np.abs(phi - pref) / np.abs(pref)
    print(f"fp64 R={R} tpb={tpb}: force max {e.max():.2e}, potential max {ep.max():.2e}")
    assert e.max() <= 1e-12 and ep.max() <= 1e-12
    for N in (2, 65, 257, 1000):
        x, m = inputs.random_cloud(N, 400 + N, scale=0.5)
        for eps in (0.01, 0.0):
            got = _gpu(x, m, eps, dev, "fp64")
            ref = oracle.forces(x, m, eps)
            err = np.max(np.linalg.norm(got - ref, axis=0) / _term_scale(x, m, eps))
            assert err <= 1e-14, (N, eps, err)


@pytest.mark.parametrize("N,C", [(700, 1), (65, 2), (2, 1)])
def test_fp64_symmetric_vjp(dev, form2, N, C):
    x, m = inputs.random_cloud(N, 500 + N, scale=0.5)
    lam = np.random.default_rng(C).standard_normal((C, 3, N))
    got = colatus.force_vjp(to_dev(x, dev), to_dev(m, dev), to_dev(lam, dev), 0.02, 1.3,
                            precision="fp64").cpu().numpy()
    for c in range(C):
        assert _rel(got[c], oracle.force_vjp(x, m, lam[c], 0.02, G=1.3)) <= 1e-12


@pytest.mark.parametrize("eps", [0.0, 1e-30])
def test_fp64_symmetric_pair_law_over_twelve_decades(dev, form2, eps):
    """FP64 pairs that need no potential take r^-3 from v_rsq_f64 with a
    first-order correction of its cube (relative error below 3e-14 for
    v_rsq_f64's 6e-8).  Two particles at +-r/2 (the separation exact in
    FP64), r from 1e-8 to 1e4: each acceleration is G m / r^2 along the pair
    to 5e-14; eps = 0 takes the coincident-pair mask, eps = 1e-30 does not."""
    G, mass = 1.3, 0.7
    for r in np.logspace(-8, 4, 49):
        x = np.zeros((3, 2))
        x[0] = [-r / 2, r / 2]
        x[1] = [0.25 * r, -0.25 * r]
        d = x[:, 1] - x[:, 0]
        rr = np.sqrt((d ** 2).sum())
        acc = colatus.forces(to_dev(x, dev), to_dev(np.full(2, mass), dev), eps, G=G,
                             precision="fp64").cpu().numpy()
        want = G * mass * d / rr ** 3
        e = max(np.abs(acc[:, 0] - want).max(), np.abs(acc[:, 1] + want).max())
        assert e <= 5e-14 * np.abs(want).max(), (r, e / np.abs(want).max())
