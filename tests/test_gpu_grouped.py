"""GPU checks of the grouped symmetric forward loop (COLATUS_OPT_PAIR_GROUP).

The forward symmetric loop runs 2x2 blocks of part pairs in one workgroup
of four waves and adds, in LDS, the two partial sums that share a target
part and the two that share a source part before writing them, so every
particle gets ceil(P/2) + 1 partial-sum slots instead of P.  The grouped
and single-item forms evaluate the same pair terms in the same order; the
grouped sums differ by one rounding per combined slot (FP32 with FP32
pairs, FP64 with FP64 pairs).  The symmetric form is forced at every size
(COLATUS_OPT_PAIR_FORM = 2: boxes too small to fill the GPU take the
ordered loop by default).  Checked here:
  * both forms against each other and against the oracle, for box sizes
    with an odd and an even number of parts, ragged last parts, a lone
    part, unequal masses, the potential and softening zero;
  * ragged batches, and the persistent grid giving the same bits as the
    one-shot grid;
  * that no slot a reader adds is left from an earlier sweep: a call after
    a call on other positions gives the same bits as a repeated call;
  * a run of steps in both forms.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _term_scale(x, m, eps):
    d = x[:, None, :] - x[:, :, None]
    s = (d ** 2).sum(axis=0) + eps * eps
    with np.errstate(divide="ignore"):
        w = m[None, :] * s ** -1.5
    np.fill_diagonal(w, 0.0)
    return (w * np.sqrt((d ** 2).sum(axis=0))).sum(axis=1)


def _pot_scale(x, m, eps):
    d = x[:, None, :] - x[:, :, None]
    s = (d ** 2).sum(axis=0) + eps * eps
    with np.errstate(divide="ignore"):
        w = m[None, :] / np.sqrt(s)
    np.fill_diagonal(w, 0.0 if eps == 0.0 else m / eps)
    return w.sum(axis=1)


@pytest.fixture
def grouping():
    # the symmetric form at every size (small boxes take the ordered loop by
    # default)
    colatus.set_option(colatus.OPT_PAIR_FORM, 2)
    yield
    colatus.set_option(colatus.OPT_PAIR_GROUP, 1)
    colatus.set_option(colatus.OPT_PERSISTENT, 0)
    colatus.set_option(colatus.OPT_PAIR_FORM, -1)


def _forces(x, m, eps, dev, prec, group, with_phi=False, batch=None, a=1.0):
    colatus.set_option(colatus.OPT_PAIR_GROUP, group)
    out = colatus.forces(to_dev(x, dev), to_dev(m, dev), eps, a=a, precision=prec,
                         with_phi=with_phi, batch=batch)
    torch.cuda.synchronize()
    if with_phi:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy(), None


# FP64: the two forms differ by the rounding of a few FP64 additions;
# FP32 forms: by one FP32 rounding of each combined partial sum
PAIR_BAR = {"fp64": 1e-14, "mixed_twosum": 1e-6, "mixed_f64acc": 1e-6, "fp32": 2e-6}
ORACLE_BAR = {"fp64": 1e-13, "mixed_twosum": 5e-6, "mixed_f64acc": 5e-6, "fp32": 2e-5}


@pytest.mark.parametrize("N", [1, 2, 200, 256, 257, 700, 1025, 1300, 2091])
@pytest.mark.parametrize("prec", ["fp64", "mixed_twosum", "mixed_f64acc", "fp32"])
def test_grouped_matches_single_items_and_oracle(dev, grouping, N, prec):
    x, m = inputs.random_cloud(N, 900 + N, scale=0.5, mass_spread=bool(N % 2))
    eps = 0.01
    g, gp = _forces(x, m, eps, dev, prec, 1, with_phi=True)
    s, sp = _forces(x, m, eps, dev, prec, 0, with_phi=True)
    if N == 1:
        assert np.all(g == 0.0) and np.all(s == 0.0)
        return
    sc, ps = _term_scale(x, m, eps), _pot_scale(x, m, eps)
    d = np.max(np.linalg.norm(g - s, axis=0) / sc)
    dp = np.max(np.abs(gp - sp) / ps)
    ref = oracle.forces(x, m, eps)
    pref = oracle.potential(x, m, eps)
    e = np.max(np.linalg.norm(g - ref, axis=0) / sc)
    ep = np.max(np.abs(gp - pref) / ps)
    print(f"N={N} {prec}: grouped vs single {d:.2e} (potential {dp:.2e}); grouped vs "
          f"oracle {e:.2e} (potential {ep:.2e})", flush=True)
    assert d <= PAIR_BAR[prec] and dp <= PAIR_BAR[prec]
    assert e <= ORACLE_BAR[prec] and ep <= ORACLE_BAR[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed_twosum"])
def test_grouped_softening_zero(dev, grouping, prec):
    x, m = inputs.random_cloud(1100, 31, scale=0.5)
    x[:, 7] = x[:, 900]  # a coincident pair across parts
    x[:, 8] = x[:, 9]    # and one inside a part
    g, _ = _forces(x, m, 0.0, dev, prec, 1)
    s, _ = _forces(x, m, 0.0, dev, prec, 0)
    assert np.all(np.isfinite(g))
    # the coincident pairs add nothing (the oracle's sum is undefined there):
    # those particles are checked against the single-item form only
    pairs = [7, 900, 8, 9]
    keep = np.ones(x.shape[1], bool)
    keep[pairs] = False
    with np.errstate(invalid="ignore"):
        sc = _term_scale(x, m, 0.0)
        ref = oracle.forces(x, m, 0.0)
    d = np.max(np.linalg.norm(g - s, axis=0)[keep] / sc[keep])
    e = np.max(np.linalg.norm(g - ref, axis=0)[keep] / sc[keep])
    dc = np.max(np.linalg.norm(g - s, axis=0)[pairs] / np.linalg.norm(s, axis=0)[pairs])
    print(f"{prec} eps=0: grouped vs single {d:.2e} (coincident {dc:.2e}), vs oracle {e:.2e}",
          flush=True)
    assert d <= PAIR_BAR[prec] and e <= (1e-13 if prec == "fp64" else 1e-5)
    assert dc <= 100 * PAIR_BAR[prec]


def test_grouped_batch_persistent_and_alone(dev, grouping):
    sizes = [1, 255, 256, 257, 600, 1500, 3000, 2]
    xs, ms, epss = [], [], []
    for i, n in enumerate(sizes):
        x, m = inputs.random_cloud(n, 70 + i, scale=0.5, mass_spread=bool(i % 2))
        xs.append(x + 0.1 * i)
        ms.append(m)
        epss.append(0.01 * (i + 1))
    x = np.concatenate(xs, axis=1)
    m = np.concatenate(ms)
    off = np.concatenate([[0], np.cumsum(sizes)])
    batch = (off, np.array(epss))
    runs = {}
    for pers in (0, 1):
        colatus.set_option(colatus.OPT_PERSISTENT, pers)
        runs[pers] = _forces(x, m, 0.0, dev, "mixed_twosum", 1, with_phi=True, batch=batch,
                             a=0.5)
    colatus.set_option(colatus.OPT_PERSISTENT, 0)
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    got, phi = runs[0]
    single, _ = _forces(x, m, 0.0, dev, "mixed_twosum", 0, with_phi=True, batch=batch, a=0.5)
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        if sizes[b] == 1:
            assert np.all(got[:, sl] == 0.0)
            continue
        sc = _term_scale(xs[b], ms[b], epss[b]) / 0.5 ** 3
        ref = oracle.forces(xs[b], ms[b], epss[b], a=0.5)
        assert np.max(np.linalg.norm(got[:, sl] - ref, axis=0) / sc) <= 5e-6
        assert np.max(np.linalg.norm(got[:, sl] - single[:, sl], axis=0) / sc) <= 1e-6
        pref = oracle.potential(xs[b], ms[b], epss[b])
        assert np.max(np.abs(phi[sl] - pref) / _pot_scale(xs[b], ms[b], epss[b])) <= 5e-6
    alone, _ = _forces(xs[6], ms[6], epss[6], dev, "mixed_twosum", 1, a=0.5)
    assert np.array_equal(alone, got[:, off[6]:off[7]])


@pytest.mark.parametrize("N", [257, 513, 1025, 32768])
@pytest.mark.parametrize("prec", ["fp64", "mixed_twosum"])
def test_grouped_writes_every_slot_it_reads(dev, grouping, N, prec):
    """A slot left from an earlier sweep would change the sum: the result of
    a call after a call on other positions equals that of a repeated call."""
    colatus.set_option(colatus.OPT_PAIR_GROUP, 1)
    xa, m = inputs.random_cloud(N, 5, scale=0.5)
    xb, _ = inputs.random_cloud(N, 6, scale=0.5)
    mt = to_dev(m, dev)
    colatus.forces(to_dev(xb, dev), mt, 0.01, precision=prec)
    b1 = colatus.forces(to_dev(xb, dev), mt, 0.01, precision=prec).cpu().numpy()
    colatus.forces(to_dev(xa, dev), mt, 0.01, precision=prec)
    b2 = colatus.forces(to_dev(xb, dev), mt, 0.01, precision=prec).cpu().numpy()
    assert np.array_equal(b1, b2)


def test_grouped_run_close_to_single_items(dev, grouping):
    """Ten mixed steps at 16^3: the two forms differ by one rounding per
    combined slot, which the run carries like any FP32 rounding: they stay
    closer to each other than the single-item run is to the FP64 run."""
    w = inputs.lcdm_grf(16)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    out = {}
    for group, prec in ((1, "mixed_twosum"), (0, "mixed_twosum"), (0, "fp64")):
        colatus.set_option(colatus.OPT_PAIR_GROUP, group)
        xt, vt = to_dev(w.x, dev), to_dev(v0, dev)
        colatus.run(xt, vt, to_dev(w.m, dev), w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 30,
                    last_step=10, precision=prec)
        out[(group, prec)] = (xt.cpu().numpy(), vt.cpu().numpy())
    g, s, d = out[(1, "mixed_twosum")], out[(0, "mixed_twosum")], out[(0, "fp64")]
    dv_scale = np.abs(d[1] - v0).max()
    dx_gs, dx_sd = np.abs(g[0] - s[0]).max(), np.abs(s[0] - d[0]).max()
    dv_gs, dv_sd = np.abs(g[1] - s[1]).max() / dv_scale, np.abs(s[1] - d[1]).max() / dv_scale
    print(f"10 steps at 16^3: grouped vs single |dx| {dx_gs:.2e}, |dv| {dv_gs:.2e}; single vs "
          f"FP64 |dx| {dx_sd:.2e}, |dv| {dv_sd:.2e} (|dv| / max|v - v0|)", flush=True)
    assert dx_gs <= dx_sd and dv_gs <= dv_sd
