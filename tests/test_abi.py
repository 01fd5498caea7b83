"""The C ABI on the host: every declared symbol is exported, and argument
checks reject bad input before any HIP call (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1208_3444_amd import colatus

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "colatus.h")

EINVAL, EFRIEDMANN, ENODEV = -1, -2, -3
FAKE = ctypes.c_void_p(4096)  # never dereferenced: checks fail first

LCDM = (math.sqrt(8 * math.pi / 0.9), 0.0, 0.3, 0.0, 0.7)


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(colatus_[a-z0-9_]+)\s*\(", text)))


def _declared_arity():
    """Number of parameters of every prototype in the header."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(colatus_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", text):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_every_declared_symbol_is_exported():
    L = colatus.lib()
    names = _declared()
    assert "colatus_forces" in names and "colatus_adjoint" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(colatus.SIGNATURES), "binding signatures out of sync with header"
    arity = _declared_arity()
    assert set(arity) == set(names)
    for n, (_, args) in colatus.SIGNATURES.items():
        assert len(args) == arity[n], (n, len(args), arity[n])


def test_strerror_and_version():
    L = colatus.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.colatus_strerror(code)
    assert L.colatus_strerror(-99) == b"unknown error code"
    assert L.colatus_version() == 10400


def test_forces_rejects_bad_arguments():
    L = colatus.lib()
    f = L.colatus_forces
    ok = dict(x=FAKE, m=FAKE, N=16, eps=0.01, G=1.0, a=1.0, prec=0, acc=FAKE, phi=None)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["x"], a["m"], a["N"], a["eps"], a["G"], a["a"], a["prec"], a["acc"],
                 a["phi"], None, a.get("att"), a.get("bg"), None)

    assert call(N=0) == EINVAL
    assert call(N=(1 << 28) + 1) == EINVAL
    assert call(eps=-1e-3) == EINVAL
    assert call(eps=float("nan")) == EINVAL
    assert call(G=float("inf")) == EINVAL
    assert call(a=0.0) == EINVAL
    assert call(a=-1.0) == EINVAL
    assert call(prec=4) == EINVAL
    assert call(x=None) == EINVAL
    assert call(acc=None) == EINVAL
    # the Eq. (10) attractor must be finite
    for bad in ((float("nan"), (0.0, 0.0, 0.0)), (1.0, (0.0, float("inf"), 0.0))):
        pa, keep = colatus._attractor(bad)
        assert call(att=pa) == EINVAL
    # so must the Eq. (6) background term
    for bad in ((float("inf"), (0.5, 0.5, 0.5)), (1.0, (0.5, float("nan"), 0.5))):
        pb, keep = colatus._background(bad)
        assert call(bg=pb) == EINVAL


def test_batch_descriptor_checks():
    L = colatus.lib()
    import numpy as np
    off = np.array([0, 10, 10, 30], dtype=np.int64)  # empty box
    eps = np.array([0.1, 0.1, 0.1])
    b = colatus._Batch(3, off.ctypes.data, eps.ctypes.data)
    rc = L.colatus_forces(FAKE, FAKE, 30, 0.0, 1.0, 1.0, 1, FAKE, None, ctypes.byref(b), None,
                          None, None)
    assert rc == EINVAL
    off2 = np.array([0, 10, 25], dtype=np.int64)  # does not end at N
    b2 = colatus._Batch(2, off2.ctypes.data, eps.ctypes.data)
    assert L.colatus_forces(FAKE, FAKE, 30, 0.0, 1.0, 1.0, 1, FAKE, None, ctypes.byref(b2),
                            None, None, None) == EINVAL
    eps3 = np.array([0.1, -0.1])
    off3 = np.array([0, 10, 30], dtype=np.int64)
    b3 = colatus._Batch(2, off3.ctypes.data, eps3.ctypes.data)
    assert L.colatus_forces(FAKE, FAKE, 30, 0.0, 1.0, 1.0, 1, FAKE, None, ctypes.byref(b3),
                            None, None, None) == EINVAL



def test_binding_batch_lengths():
    """The binding checks the batch arrays' lengths before they reach the
    library, which reads B + 1 offsets and B softenings."""
    off, keep = colatus._batch(([0, 10, 30], [0.1, 0.2]))
    assert off.n_boxes == 2 and keep[0].size == 3
    for bad in (([0, 30], [0.1, 0.2]), ([0, 10, 20, 30], [0.1, 0.2]), ([0], [])):
        with pytest.raises(ValueError, match="offsets"):
            colatus._batch(bad)

def _run(**kw):
    L = colatus.lib()
    a = dict(x=FAKE, v=FAKE, m=FAKE, N=8, eps=0.01, G=1.0, cos=LCDM, a0=0.1, a1=1.0,
             n=10, first=0, last=10, prec=1)
    a.update(kw)
    return L.colatus_run(a["x"], a["v"], a["m"], a["N"], a["eps"], a["G"], *a["cos"],
                         a["a0"], a["a1"], a["n"], a["first"], a["last"], a["prec"], None, None,
                         a.get("att"), a.get("bg"), a.get("trk"), None)


def test_run_rejects_bad_arguments():
    assert _run(n=0, last=0) == EINVAL
    assert _run(first=-1) == EINVAL
    assert _run(first=5, last=5) == EINVAL
    assert _run(last=11) == EINVAL
    assert _run(a0=0.0) == EINVAL
    assert _run(a1=-1.0) == EINVAL
    assert _run(a1=0.1) == EINVAL  # zero span with H0 > 0
    assert _run(cos=(-1.0, 0, 1, 0, 0)) == EINVAL
    assert _run(cos=(1.0, 0, float("nan"), 0, 0)) == EINVAL
    assert _run(v=None) == EINVAL
    assert _run(prec=7) == EINVAL
    pa, keep = colatus._attractor((0.5, (0.0, float("nan"), 0.0)))
    assert _run(att=pa) == EINVAL


def _tracks(idx, n=None, out=FAKE):
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    t = colatus._Tracks(len(idx) if n is None else n,
                        idx.ctypes.data if len(idx) else None, out)
    return ctypes.byref(t), (t, idx)


def test_run_rejects_bad_tracks():
    L = colatus.lib()
    bad = [
        _tracks([], n=0),                 # no tracers
        _tracks([1, 2], n=70000),         # above the limit
        _tracks([8]),                     # out of range (N = 8)
        _tracks([-1, 2]),                 # negative
        _tracks([2, 5, 2]),               # repeated
        _tracks([1, 2], out=None),        # no output
    ]
    for pt, keep in bad:
        assert _run(trk=pt) == EINVAL
        args = dict(x=FAKE, v=FAKE, m=FAKE)
        rc = L.colatus_run_he(args["x"], args["v"], args["m"], 8, 0.01, 1.0, *LCDM, 0.1, 1.0,
                              10, 0, 10, 1, None, None, None, None, pt, None)
        assert rc == EINVAL
    t = colatus._Tracks(2, None, FAKE)  # NULL index list
    assert _run(trk=ctypes.byref(t)) == EINVAL
    pb, keep = colatus._background((0.5, (0.0, 0.0, float("inf"))))
    assert _run(bg=pb) == EINVAL


def test_step_rejects_aliased_force_cache():
    L = colatus.lib()
    for g in (FAKE, ctypes.c_void_p(8192)):
        x, v = FAKE, ctypes.c_void_p(8192)
        rc = L.colatus_step(x, v, FAKE, 8, 0.01, 1.0, *LCDM, 0.2, 0.3, 1, g, None, None, None,
                            None)
        assert rc == EINVAL


def test_spectrum_rejects_bad_arguments():
    L = colatus.lib()
    assert L.colatus_velocity_spectrum(FAKE, 0, 4, 0, FAKE, None) == EINVAL
    assert L.colatus_velocity_spectrum(FAKE, (1 << 17) + 1, 4, 0, FAKE, None) == EINVAL
    assert L.colatus_velocity_spectrum(FAKE, 100, 0, 0, FAKE, None) == EINVAL
    assert L.colatus_velocity_spectrum(FAKE, 100, 65537, 0, FAKE, None) == EINVAL
    assert L.colatus_velocity_spectrum(None, 100, 4, 0, FAKE, None) == EINVAL
    assert L.colatus_velocity_spectrum(FAKE, 100, 4, 0, None, None) == EINVAL


def test_run_rejects_unphysical_friedmann_range():
    # closed matter universe: H^2 ~ a^-3 (1 - 2a) turns negative past a = 0.5
    assert _run(cos=(1.0, 0.0, 1.0, -2.0, 0.0), a0=0.3, a1=0.9) == EFRIEDMANN
    # a dip below zero strictly inside the range, positive at both ends:
    # f(a) = 1 - 3a + 2.5 a^2 ... via Om_R + Om_M a + Om_K a^2 with a minimum < 0
    assert _run(cos=(1.0, 1.0, -3.0, 2.2, 0.0), a0=0.2, a1=1.2) == EFRIEDMANN


def test_adjoint_rejects_bad_arguments():
    L = colatus.lib()

    def call(**kw):
        a = dict(N=8, K=5, C=1, batch=None, prec=1, ga=None, att=None)
        a.update(kw)
        return L.colatus_adjoint(FAKE, FAKE, FAKE, a["N"], 0.01, 1.0, *LCDM, 0.2, 1.0, 10,
                                 a["K"], a["C"], FAKE, FAKE, FAKE, FAKE, None, None, a["ga"],
                                 a["prec"], a["batch"], a["att"], a.get("bg"), None)

    assert call(K=-2) == EINVAL
    assert call(C=0) == EINVAL
    assert call(C=5000) == EINVAL
    # a batch is read on the host: its offsets must end at N, its softenings
    # be non-negative
    off = np.array([0, 3, 7], dtype=np.int64)
    eps = np.array([0.01, 0.02])
    bad = colatus._Batch(2, off.ctypes.data, eps.ctypes.data)
    assert call(batch=ctypes.byref(bad)) == EINVAL
    eps_bad = np.array([0.01, -0.02])
    off_ok = np.array([0, 3, 8], dtype=np.int64)
    bad2 = colatus._Batch(2, off_ok.ctypes.data, eps_bad.ctypes.data)
    assert call(batch=ctypes.byref(bad2)) == EINVAL
    empty = colatus._Batch(0, off_ok.ctypes.data, eps.ctypes.data)
    assert call(batch=ctypes.byref(empty)) == EINVAL
    # attractor gradients need an attractor
    assert call(ga=FAKE) == EINVAL
    pa, keep = colatus._attractor((float("inf"), (0.0, 0.0, 0.0)))
    assert call(att=pa) == EINVAL


def test_hubble_host():
    L = colatus.lib()
    out = ctypes.c_double()
    assert L.colatus_hubble(0.5, 2.0, 0.0, 1.0, 0.0, 0.0, ctypes.byref(out)) == 0
    assert abs(out.value - 2.0 * 0.5 ** -1.5) < 1e-15 * out.value
    assert L.colatus_hubble(0.9, 1.0, 0.0, 1.0, -2.0, 0.0, ctypes.byref(out)) == EFRIEDMANN
    assert L.colatus_hubble(0.0, 1.0, 0.0, 1.0, 0.0, 0.0, ctypes.byref(out)) == EINVAL


def test_options_and_tile_config():
    L = colatus.lib()
    v = ctypes.c_int64()
    assert L.colatus_get_option(1, ctypes.byref(v)) == 0 and v.value == 0  # graphs off
    assert L.colatus_get_option(8, ctypes.byref(v)) == 0 and v.value == -1
    assert L.colatus_set_option(8, 3) == EINVAL
    assert L.colatus_set_option(4, 3) == EINVAL
    assert L.colatus_set_option(5, 32) == EINVAL
    assert L.colatus_set_option(99, 0) == EINVAL
    # roctx ranges: off by default, any nonzero value turns them on
    assert L.colatus_get_option(9, ctypes.byref(v)) == 0 and v.value == 0
    assert L.colatus_set_option(9, 5) == 0
    assert L.colatus_get_option(9, ctypes.byref(v)) == 0 and v.value == 1
    assert L.colatus_set_option(9, 0) == 0
    # 2x2 groups of part pairs: on by default, 0 or 1 only
    assert L.colatus_get_option(10, ctypes.byref(v)) == 0 and v.value == 1
    assert L.colatus_set_option(10, 2) == EINVAL
    assert L.colatus_set_option(10, 0) == 0
    assert L.colatus_get_option(10, ctypes.byref(v)) == 0 and v.value == 0
    assert L.colatus_set_option(10, 1) == 0
    # forward sweeps and the few-cotangent adjoint: symmetric form, parts of
    # 4 x 64 particles
    assert colatus.tile_config(32768, "mixed") == (4, 64, 128, 2)
    # boxes too small to fill the GPU with symmetric items (fewer than 1024
    # waves): the ordered loop, one target per lane, one source tile per slice
    assert colatus.tile_config(1000, "fp32") == (1, 128, 8, 0)
    assert colatus.tile_config(4096, "fp64") == (1, 128, 32, 0)
    assert colatus.tile_config(8000, "mixed") == (1, 256, 32, 0)
    assert colatus.tile_config(13824, "mixed") == (4, 64, 54, 2)
    assert colatus.tile_config(4096, "mixed", kind=1) == (1, 256, 16, 0)
    assert colatus.tile_config(13824, "mixed", kind=1) == (4, 64, 54, 2)
    assert colatus.tile_config(32768, "fp64") == (4, 64, 128, 2)
    assert colatus.tile_config(32768, "mixed", kind=1) == (4, 64, 128, 2)
    assert colatus.tile_config(262144, "mixed") == (4, 64, 1024, 2)
    # beyond 2^18 particles in a box: ordered form
    assert colatus.tile_config(300000, "mixed")[3] == 0
    assert colatus.tile_config(300000, "fp64")[0:2] == (2, 256)
    assert colatus.tile_config(300000, "fp64", kind=1)[3] == 0
    colatus.set_option(colatus.OPT_TILE_SLICES, 3)
    colatus.set_option(colatus.OPT_PAIR_FORM, 1)
    try:
        assert colatus.tile_config(32768, "mixed")[2:] == (3, 1)
        assert colatus.tile_config(32768, "fp64")[3] == 0  # no form 1 for FP64 pairs
        assert colatus.tile_config(32768, "mixed", kind=1)[3] == 0  # nor for the adjoint
        colatus.set_option(colatus.OPT_PAIR_FORM, 2)
        # form 2 derives its slots from the part size; TILE_SLICES does not apply
        assert colatus.tile_config(200000, "mixed") == (4, 64, 782, 2)
        colatus.set_option(colatus.OPT_TILE_R, 8)
        assert colatus.tile_config(4096, "mixed") == (8, 64, 8, 2)
    finally:
        colatus.set_option(colatus.OPT_TILE_SLICES, 0)
        colatus.set_option(colatus.OPT_TILE_R, 0)
        colatus.set_option(colatus.OPT_PAIR_FORM, -1)


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_valid_call_without_device_is_enodev():
    assert _run() == ENODEV
    L = colatus.lib()
    assert L.colatus_forces(FAKE, FAKE, 16, 0.01, 1.0, 1.0, 0, FAKE, None, None, None,
                            None, None) == ENODEV


def test_forces_noalloc_rejects_bad_arguments_on_host():
    """The allocation-free pair sum checks its arguments before any HIP call;
    N beyond its fixed scratch is COLATUS_ESCRATCH."""
    L = colatus.lib()
    f = L.colatus_forces_noalloc

    def call(N=16, eps=0.01, G=1.0, a=1.0, prec=0, x=FAKE, m=FAKE, acc=FAKE):
        return f(x, m, N, eps, G, a, prec, acc, None, None, None, None)

    assert call(N=16385) == -7
    assert call(N=(1 << 28)) == -7
    assert b"too large" in L.colatus_strerror(-7)
    assert call(N=0) == EINVAL
    assert call(eps=-1.0) == EINVAL
    assert call(eps=float("nan")) == EINVAL
    assert call(a=0.0) == EINVAL
    assert call(G=float("inf")) == EINVAL
    assert call(prec=4) == EINVAL
    assert call(x=None) == EINVAL
    assert call(acc=None) == EINVAL


def test_ftle_and_cosmic_time_reject_bad_arguments_on_host():
    L = colatus.lib()
    tr = np.array([0, 3, 7], dtype=np.int64)

    def call(N=8, T=3, idx=tr, K=5, lam=FAKE, prec=1, n_steps=10):
        return L.colatus_ftle(FAKE, FAKE, FAKE, N, 0.01, 1.0, *LCDM, 0.2, 1.0, n_steps, K, T,
                              idx.ctypes.data_as(ctypes.c_void_p) if idx is not None else None,
                              lam, None, None, prec, None, None, None, None)

    assert call(T=0) == EINVAL
    assert call(T=1366) == EINVAL
    assert call(idx=None) == EINVAL
    assert call(idx=np.array([0, 8, 1], dtype=np.int64)) == EINVAL
    assert call(idx=np.array([-1, 2, 1], dtype=np.int64)) == EINVAL
    assert call(lam=None) == EINVAL
    assert call(K=-3) == EINVAL
    assert call(n_steps=0) == EINVAL
    assert call(prec=7) == EINVAL
    t = ctypes.c_double()
    assert L.colatus_cosmic_time(0.2, 1.0, 0, *LCDM, ctypes.byref(t), None) == EINVAL
    assert L.colatus_cosmic_time(0.2, 1.0, 10, *LCDM, None, None) == EINVAL
    assert L.colatus_cosmic_time(-0.2, 1.0, 10, *LCDM, ctypes.byref(t), None) == EINVAL
    assert L.colatus_cosmic_time(0.3, 0.9, 10, 1.0, 0.0, 1.0, -2.0, 0.0, ctypes.byref(t),
                                 None) == EFRIEDMANN


def test_periodic_entry_points_reject_bad_arguments_on_host():
    L = colatus.lib()
    f = L.colatus_forces_periodic

    def forces(N=16, eps=0.01, a=1.0, box=1.0, prec=0, x=FAKE):
        return f(x, FAKE, N, eps, 1.0, a, box, prec, FAKE, None, None)

    assert forces(box=0.0) == EINVAL
    assert forces(box=-1.0) == EINVAL
    assert forces(box=float("inf")) == EINVAL
    assert forces(N=0) == EINVAL
    assert forces(N=262145) == EINVAL
    assert forces(eps=-0.1) == EINVAL
    assert forces(a=0.0) == EINVAL
    assert forces(prec=9) == EINVAL
    assert forces(x=None) == EINVAL
    r = L.colatus_run_periodic

    def run(box=1.0, first=0, last=4, n=4, cos=LCDM, a0=0.2, a1=1.0):
        return r(FAKE, FAKE, FAKE, 16, 0.01, 1.0, *cos, box, a0, a1, n, first, last, 1, None, None)

    assert run(box=0.0) == EINVAL
    assert run(first=3, last=3) == EINVAL
    assert run(last=5) == EINVAL
    assert run(cos=(1.0, 0.0, 1.0, -2.0, 0.0), a0=0.3, a1=0.9) == EFRIEDMANN
