"""The allocation-free pair sum (colatus_forces_noalloc) against colatus_forces,
both called through the C ABI on the same device buffers.

Two calls in a row, the second with a smaller input (the scratch array keeps
the first call's contents), in every precision, with and without the
potential: the outputs must be bitwise equal to colatus_forces with the
symmetric pair loop (COLATUS_OPT_PAIR_FORM = 2: same kernels, same slots,
same fixed-order slot sum), and agree with colatus_forces at its default
tile shape (the ordered loop for the smaller case, whose symmetric items
would not fill the GPU) to the precision's tolerance.  The oversize case is
rejected on the host.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1208_3444_amd import colatus, inputs
from conftest import rel_err_per_particle, to_dev

pytestmark = pytest.mark.gpu

PRECISIONS = ("fp64", "mixed_twosum", "mixed_f64acc", "fp32")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _call(name, x, m, eps, G, a, prec, with_phi):
    L = colatus.lib()
    N = m.shape[0]
    acc = torch.full_like(x, float("nan"))
    phi = torch.full_like(m, float("nan")) if with_phi else None
    stream = ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    fn = getattr(L, name)
    if name == "colatus_forces":
        rc = fn(_ptr(x), _ptr(m), N, eps, G, a, colatus.PRECISIONS[prec], _ptr(acc), _ptr(phi),
                None, None, None, stream)
    else:
        rc = fn(_ptr(x), _ptr(m), N, eps, G, a, colatus.PRECISIONS[prec], _ptr(acc), _ptr(phi),
                None, None, stream)
    assert rc == 0, (name, rc)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), (phi.cpu().numpy() if with_phi else None)


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("with_phi", [False, True])
def test_noalloc_equals_forces_two_calls(dev, prec, with_phi):
    # a ragged 12000-particle cloud (47 parts, the last one partial), then a
    # 2900-particle lattice: the second call reuses the scratch with fewer
    # parts, items and blocks
    x1, m1 = inputs.random_cloud(12000, 31, scale=1.0)
    w2 = inputs.eds_lattice(16)
    cases = [(x1, m1, 0.004, 1.0, 0.7), (w2.x[:, :2900], w2.m[:2900], w2.eps, 1.0, 0.1)]
    for k, (x, m, eps, G, a) in enumerate(cases):
        xt, mt = to_dev(x, dev), to_dev(m, dev)
        colatus.set_option(colatus.OPT_PAIR_FORM, 2)
        try:
            ref_acc, ref_phi = _call("colatus_forces", xt, mt, eps, G, a, prec, with_phi)
        finally:
            colatus.set_option(colatus.OPT_PAIR_FORM, -1)
        got_acc, got_phi = _call("colatus_forces_noalloc", xt, mt, eps, G, a, prec, with_phi)
        dft_acc, _ = _call("colatus_forces", xt, mt, eps, G, a, prec, False)
        e_dft = rel_err_per_particle(got_acc, dft_acc)
        print(f"call {k} N={m.shape[0]} {prec} phi={with_phi}: max |diff| "
              f"{np.max(np.abs(got_acc - ref_acc)):.3e}; against the default tile shape "
              f"max relative {e_dft.max():.3e}", flush=True)
        assert np.array_equal(got_acc, ref_acc), (k, prec)
        if with_phi:
            assert np.array_equal(got_phi, ref_phi), (k, prec)
        assert e_dft.max() <= (1e-12 if prec == "fp64" else 1e-4), (k, prec)
    # and the last call against the oracle, to the precision's tolerance
    ref = oracle.forces(cases[1][0], cases[1][1], cases[1][2], a=0.1)
    e = rel_err_per_particle(got_acc, ref)
    bound = 1e-12 if prec == "fp64" else 1e-4
    assert e.max() <= bound, (prec, e.max())


def test_noalloc_rejects_oversize_on_host(dev):
    N = 16385
    x = torch.zeros((3, N), dtype=torch.float64, device=dev)
    m = torch.ones(N, dtype=torch.float64, device=dev)
    acc = torch.zeros_like(x)
    L = colatus.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = L.colatus_forces_noalloc(_ptr(x), _ptr(m), N, 0.01, 1.0, 1.0, 0, _ptr(acc), None,
                                  None, None, stream)
    assert rc == -7
    assert L.colatus_strerror(rc).decode().startswith("problem too large")
    assert torch.count_nonzero(acc).item() == 0
