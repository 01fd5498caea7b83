"""GPU parity of the Eq. (10) deformation attractor against the FP64 oracle,
through the C ABI: forces and potential (ordered and symmetric pair loops,
batches), runs with diagnostics, the transpose Jacobian, and the adjoint
with the gradient with respect to the attractor's strength and position.
The attractor's own terms are FP64 in every precision; the bars are those of
the pair sum they join."""
import numpy as np
import pytest

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import rel_err_per_particle, to_dev

pytestmark = pytest.mark.gpu

ATT = (0.2, (0.3, 0.6, 0.45))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("form", [-1, 0])
def test_forces_and_potential(dev, form):
    w = inputs.eds_lattice(16)
    ref = oracle.forces(w.x, w.m, w.eps, a=0.1, attractor=ATT)
    pref = oracle.potential(w.x, w.m, w.eps, attractor=ATT)
    colatus.set_option(colatus.OPT_PAIR_FORM, form)
    try:
        for prec, med, mx in (("fp64", 1e-12, 1e-12), ("mixed_twosum", 1e-6, 1e-4)):
            acc, phi = colatus.forces(to_dev(w.x, dev), to_dev(w.m, dev), w.eps, a=0.1,
                                      precision=prec, with_phi=True, attractor=ATT)
            e = rel_err_per_particle(acc.cpu().numpy(), ref)
            ep = np.abs(phi.cpu().numpy() - pref) / np.abs(pref)
            print(f"form {form} {prec}: force max {e.max():.2e}, potential max {ep.max():.2e}")
            assert np.median(e) <= med and e.max() <= mx
            assert np.median(ep) <= med and ep.max() <= (1e-12 if prec == "fp64" else 1e-5)
    finally:
        colatus.set_option(colatus.OPT_PAIR_FORM, -1)
    # the attractor is really there: without it the forces differ
    acc0 = colatus.forces(to_dev(w.x, dev), to_dev(w.m, dev), w.eps, a=0.1, precision="fp64")
    assert rel_err_per_particle(acc0.cpu().numpy(), ref).max() > 1e-3


def test_batch_with_attractor(dev):
    sizes = [40, 513, 300]
    xs, ms, epss = [], [], []
    for i, n in enumerate(sizes):
        x, m = inputs.random_cloud(n, 80 + i, scale=0.5)
        xs.append(x + 0.1 * i)
        ms.append(m)
        epss.append(0.01 * (i + 1))
    x, m = np.concatenate(xs, axis=1), np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)])
    acc, phi = colatus.forces(to_dev(x, dev), to_dev(m, dev), 0.0, a=0.5, precision="fp64",
                              with_phi=True, batch=(off, np.array(epss)), attractor=ATT)
    acc, phi = acc.cpu().numpy(), phi.cpu().numpy()
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        ref = oracle.forces(xs[b], ms[b], epss[b], a=0.5, attractor=ATT)
        assert _rel(acc[:, sl], ref) <= 1e-13
        pref = oracle.potential(xs[b], ms[b], epss[b], attractor=ATT)
        assert np.max(np.abs(phi[sl] - pref) / np.abs(pref)) <= 1e-13


def test_run_with_attractor_matches_oracle(dev):
    w = inputs.eds_lattice(8, n_steps=12)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    # outside the box: a smooth pull (an attractor among the particles makes
    # close passes whose growth of rounding differences no bar at 1e-12 covers)
    att = (0.3, (1.5, 0.4, 0.55))
    xr, vr, dr = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 12,
                            diag=True, attractor=att)
    x, v = to_dev(w.x, dev), to_dev(v0, dev)
    d = colatus.run(x, v, to_dev(w.m, dev), w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 12,
                    precision="fp64", diag=True, attractor=att)
    assert np.max(np.abs(x.cpu().numpy() - xr)) <= 1e-12
    assert np.max(np.abs(v.cpu().numpy() - vr)) <= 1e-11 * np.abs(vr).max()
    for f in ("K", "U", "LI"):
        scale = np.abs(dr["U"]).max()
        assert np.max(np.abs(d[f] - dr[f])) <= 1e-11 * scale, f
    # mixed precision over the first three steps (later the collapse of the
    # open box amplifies any difference, whatever its source)
    x3, _ = oracle.run(w.x, v0, w.m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 12,
                       last_step=3, attractor=att)
    x, v = to_dev(w.x, dev), to_dev(v0, dev)
    colatus.run(x, v, to_dev(w.m, dev), w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 12,
                last_step=3, precision="mixed_twosum", attractor=att)
    assert np.max(np.abs(x.cpu().numpy() - x3)) <= 1e-6


def test_circular_orbit_static_limit(dev):
    S, r = 1.5, 0.8
    om = np.sqrt(S / r ** 3)
    x0 = np.array([[r], [0.0], [0.0]])
    v0 = np.array([[0.0], [r * om], [0.0]])
    T = 2 * np.pi / om
    static = {"H0": 0.0, "Om_R": 0.0, "Om_M": 0.0, "Om_K": 0.0, "Om_L": 0.0}
    m = np.array([1e-3])
    xr, vr = oracle.run(x0, v0, m, 0.0, 0.0, static, 1.0, T, 200, attractor=(S, (0, 0, 0)))
    x, v = to_dev(x0, dev), to_dev(v0, dev)
    colatus.run(x, v, to_dev(m, dev), 0.0, 0.0, static, 1.0, T, 200, precision="fp64",
                attractor=(S, (0.0, 0.0, 0.0)))
    assert np.max(np.abs(x.cpu().numpy() - xr)) <= 1e-13
    assert np.linalg.norm(x.cpu().numpy() - x0) < 2e-3  # back after one period


@pytest.mark.parametrize("C", [1, 5])
def test_force_vjp_with_attractor(dev, C):
    x, m = inputs.random_cloud(700, 8, scale=0.5)
    lam = np.random.default_rng(C).standard_normal((C, 3, 700))
    for prec, tol in (("fp64", 1e-12), ("mixed_twosum", 1e-5)):
        got = colatus.force_vjp(to_dev(x, dev), to_dev(m, dev), to_dev(lam, dev), 0.02, 1.3,
                                precision=prec, attractor=ATT).cpu().numpy()
        for c in range(C):
            ref = oracle.force_vjp(x, m, lam[c], 0.02, G=1.3, attractor=ATT)
            assert _rel(got[c], ref) <= tol, prec


def test_adjoint_with_attractor_gradients(dev):
    x0, m = inputs.random_cloud(96, 12, scale=0.5)
    v0 = 0.3 * np.random.default_rng(1).standard_normal((3, 96))
    eps, G, n = 0.03, 0.5, 12
    LCDM = inputs.LCDM
    att = (0.25, (0.05, -0.1, 0.2))
    rng = np.random.default_rng(2)
    lx = rng.standard_normal((2, 3, 96))
    lv = rng.standard_normal((2, 3, 96))
    gx_r, gv_r, xN_r, vN_r, ga_r = oracle.adjoint(x0, v0, m, eps, G, LCDM, 0.2, 1.0, n, lx, lv,
                                                  attractor=att)
    args = [to_dev(a, dev) for a in (x0, v0, m)]
    outs = []
    for K in (1, 5, 12, 0):
        gx, gv, xN, vN, ga = colatus.adjoint(*args, eps, G, LCDM, 0.2, 1.0, n, to_dev(lx, dev),
                                             to_dev(lv, dev), checkpoint_every=K,
                                             precision="fp64", return_state=True, attractor=att)
        outs.append((gx.cpu().numpy(), gv.cpu().numpy(), ga.cpu().numpy()))
        assert np.max(np.abs(xN.cpu().numpy() - xN_r)) <= 1e-12
    for gx, gv, ga in outs:
        assert _rel(gx, gx_r) <= 1e-10 and _rel(gv, gv_r) <= 1e-10
        assert np.max(np.abs(ga - ga_r) / np.abs(ga_r)) <= 1e-10, (ga, ga_r)
    for gx, gv, ga in outs[1:]:  # checkpoint recomputation is bitwise
        assert np.array_equal(gx, outs[0][0]) and np.array_equal(ga, outs[0][2])
    # mixed precision: the gradient of a nearby map
    gx, gv, ga = colatus.adjoint(*args, eps, G, LCDM, 0.2, 1.0, n, to_dev(lx, dev),
                                 to_dev(lv, dev), checkpoint_every=5, precision="mixed_twosum",
                                 attractor=att)
    assert _rel(gx.cpu().numpy(), gx_r) <= 1e-3
    assert np.max(np.abs(ga.cpu().numpy() - ga_r) / np.abs(ga_r)) <= 1e-3


def test_zero_strength_attractor_changes_nothing_but_gives_d_dS(dev):
    x0, m = inputs.random_cloud(64, 13, scale=0.5)
    v0 = 0.2 * np.random.default_rng(3).standard_normal((3, 64))
    lx = np.random.default_rng(4).standard_normal((3, 64))
    lv = np.zeros_like(lx)
    args = [to_dev(a, dev) for a in (x0, v0, m)]
    cos = inputs.LCDM
    g0 = colatus.adjoint(*args, 0.03, 0.5, cos, 0.2, 1.0, 8, to_dev(lx, dev), to_dev(lv, dev),
                         precision="fp64")
    att = (0.0, (0.2, 0.1, -0.3))
    g1 = colatus.adjoint(*args, 0.03, 0.5, cos, 0.2, 1.0, 8, to_dev(lx, dev), to_dev(lv, dev),
                         precision="fp64", attractor=att)
    assert np.array_equal(g0[0].cpu().numpy(), g1[0].cpu().numpy())
    assert np.array_equal(g0[1].cpu().numpy(), g1[1].cpu().numpy())
    ga_r = oracle.adjoint(x0, v0, m, 0.03, 0.5, cos, 0.2, 1.0, 8, lx, lv, attractor=att)[4]
    ga = g1[2].cpu().numpy()
    assert ga[0] == pytest.approx(ga_r[0], rel=1e-10)
    assert np.all(ga[1:] == 0.0)
