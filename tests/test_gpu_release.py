"""colatus_release frees every workspace: the calls made after it rebuild
their scratch and give the same bits as before it, and the caller's current
device is left as it was."""
import numpy as np
import pytest
import torch

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _all_kinds(dev):
    """One call of each kind that owns scratch: forces with the potential, a
    tracked run with diagnostics, the spectrum of its track, an adjoint."""
    w = inputs.eds_lattice(8, n_steps=10)
    v0 = w.velocities(oracle.hubble(w.a_begin, *w.cosmo.values()))
    x, m = to_dev(w.x, dev), to_dev(w.m, dev)
    acc, phi = colatus.forces(x, m, w.eps, precision="mixed_twosum", with_phi=True)
    xr, vr = to_dev(w.x, dev), to_dev(v0, dev)
    d, tr = colatus.run(xr, vr, m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 10, diag=True,
                        tracers=[1, 60, 400])
    spec = colatus.velocity_spectrum(tr, remove_mean=True)
    rng = np.random.default_rng(7)
    lx, lv = rng.standard_normal((1, 3, w.N)), rng.standard_normal((1, 3, w.N))
    gx, gv = colatus.adjoint(x, to_dev(v0, dev), m, w.eps, w.G, w.cosmo, w.a_begin, w.a_end, 10,
                             to_dev(lx, dev), to_dev(lv, dev), checkpoint_every=4,
                             precision="mixed_twosum")
    out = [t.cpu().numpy() for t in (acc, phi, xr, vr, tr, spec, gx, gv)]
    return out + [d[k] for k in sorted(d)]


def test_release_then_reuse(dev):
    before = _all_kinds(dev)
    current = torch.cuda.current_device()
    colatus.release()
    assert torch.cuda.current_device() == current
    after = _all_kinds(dev)
    assert len(before) == len(after)
    for u, v in zip(before, after):
        assert np.array_equal(u, v)
    colatus.release()  # twice in a row is harmless
    again = _all_kinds(dev)
    for u, v in zip(before, again):
        assert np.array_equal(u, v)
