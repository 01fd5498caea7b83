"""Every kernel family run twice on the same input gives the same bits:
forward sweeps (symmetric and ordered, with the potential), runs with
diagnostics (graph and eager launches, both schemes, a batch, the external
terms and tracks), the transpose Jacobian and the adjoint (symmetric and
ordered loops), and the velocity spectrum.  Every partial sum has one
writer and every reduction a fixed order, so a race or an order that
depends on scheduling would show here."""
import numpy as np
import pytest

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _twice(fn):
    a, b = fn(), fn()
    flat_a = a if isinstance(a, (list, tuple)) else [a]
    flat_b = b if isinstance(b, (list, tuple)) else [b]
    for u, v in zip(flat_a, flat_b):
        if isinstance(u, dict):
            for k in u:
                assert np.array_equal(u[k], v[k]), k
        else:
            assert np.array_equal(np.asarray(u), np.asarray(v))


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("form", [-1, 0])
@pytest.mark.parametrize("prec", ["fp64", "mixed_twosum", "mixed_f64acc", "fp32"])
def test_forces_with_potential(dev, form, prec):
    w = inputs.lcdm_grf(16, seed=21)
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    colatus.set_option(colatus.OPT_PAIR_FORM, form)
    try:
        _twice(lambda: [_np(t) for t in colatus.forces(x, m, w.eps, precision=prec,
                                                       with_phi=True)])
    finally:
        colatus.set_option(colatus.OPT_PAIR_FORM, -1)


@pytest.mark.parametrize("graph", [1, 0])
@pytest.mark.parametrize("scheme", ["kdk", "he"])
def test_runs_with_diagnostics_tracks_and_external_terms(dev, graph, scheme):
    w = inputs.eds_lattice(8, n_steps=12)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    bg = (colatus.background_coefficient(w.cosmo), (0.5, 0.5, 0.5))

    def go():
        x, v = to_dev(w.x, dev), to_dev(v0, dev)
        d, tr = colatus.run(x, v, to_dev(w.m, dev), w.eps, w.G, w.cosmo, w.a_begin, w.a_end,
                            12, diag=True, scheme=scheme, attractor=(0.1, (0.5, 0.5, 0.5)),
                            background=bg, tracers=[0, 17, 300])
        return [_np(x), _np(v), d, _np(tr)]

    prev = colatus.get_option(colatus.OPT_GRAPH)
    colatus.set_option(colatus.OPT_GRAPH, graph)
    try:
        _twice(go)
    finally:
        colatus.set_option(colatus.OPT_GRAPH, prev)


def test_ensemble_run(dev):
    e = inputs.ragged_ensemble(12, 64, 1500)
    ve = e.velocities(oracle.hubble(e.a_begin, *e.cosmo.values()))

    def go():
        x, v = to_dev(e.x, dev), to_dev(ve, dev)
        d = colatus.run(x, v, to_dev(e.m, dev), 0.0, e.G, e.cosmo, e.a_begin, e.a_end, 10,
                        diag=True, batch=(e.box_offsets, e.box_eps))
        return [_np(x), _np(v)] + d

    _twice(go)


@pytest.mark.parametrize("C", [1, 5])
def test_vjp_and_adjoint(dev, C):
    x0, m = inputs.random_cloud(300, 41, scale=0.5)
    v0 = 0.2 * np.random.default_rng(42).standard_normal((3, 300))
    rng = np.random.default_rng(43)
    lx, lv = rng.standard_normal((C, 3, 300)), rng.standard_normal((C, 3, 300))
    args = [to_dev(a, dev) for a in (x0, v0, m)]
    for prec in ("fp64", "mixed_twosum"):
        _twice(lambda: _np(colatus.force_vjp(args[0], args[2], to_dev(lx, dev), 0.02, 0.7,
                                             precision=prec)))
        _twice(lambda: [_np(t) for t in colatus.adjoint(
            *args, 0.02, 0.7, inputs.LCDM, 0.2, 1.0, 10, to_dev(lx, dev), to_dev(lv, dev),
            checkpoint_every=3, precision=prec, attractor=(0.2, (0.1, 0.0, 0.0)))])


def test_spectrum(dev):
    tr = np.random.default_rng(44).standard_normal((1001, 2, 3, 64))
    t = to_dev(tr, dev)
    _twice(lambda: _np(colatus.velocity_spectrum(t, remove_mean=True)))
