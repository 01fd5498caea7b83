"""Python binding of libcolatus (argument marshalling only).

Every computation happens in the HIP library behind the C ABI declared in
``include/colatus.h``; this module checks tensor placement, dtype and shape,
passes device pointers and the current HIP stream, and turns negative return
codes into exceptions.  There is no CPU fallback: if ``libcolatus.so`` has not
been built, every call raises.

Tensors are torch float64 on a HIP device, contiguous, positions and
velocities shaped (3, N) (structure of arrays), masses (N,).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcolatus.so")

FP64 = 0
MIXED_TWOSUM = 1
MIXED_F64ACC = 2
FP32 = 3
PRECISIONS = {"fp64": FP64, "mixed_twosum": MIXED_TWOSUM, "mixed": MIXED_TWOSUM,
              "mixed_f64acc": MIXED_F64ACC, "fp32": FP32}

OPT_GRAPH = 1
OPT_TIMER = 2
OPT_AUTOTUNE = 3
OPT_TILE_R = 4
OPT_TILE_TPB = 5
OPT_TILE_SLICES = 6
OPT_PERSISTENT = 7
OPT_PAIR_FORM = 8
OPT_ROCTX = 9
OPT_PAIR_GROUP = 10

ERRORS = {0: "OK", -1: "EINVAL", -2: "EFRIEDMANN", -3: "ENODEV", -4: "ENOMEM", -5: "EHIP",
          -6: "ENONFINITE", -7: "ESCRATCH"}

# Every symbol include/colatus.h declares, with its ctypes signature.
_d, _i64, _i32, _i, _p = (ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                          ctypes.c_void_p)
SIGNATURES = {
    "colatus_forces": (_i, [_p, _p, _i64, _d, _d, _d, _i, _p, _p, _p, _p, _p, _p]),
    "colatus_step": (_i, [_p, _p, _p, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i, _p, _p,
                          _p, _p, _p]),
    "colatus_run": (_i, [_p, _p, _p, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i64, _i64,
                         _i64, _i, _p, _p, _p, _p, _p, _p]),
    "colatus_run_he": (_i, [_p, _p, _p, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i64, _i64,
                            _i64, _i, _p, _p, _p, _p, _p, _p]),
    "colatus_velocity_spectrum": (_i, [_p, _i64, _i32, _i, _p, _p]),
    "colatus_adjoint": (_i, [_p, _p, _p, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i64, _i64,
                             _i32, _p, _p, _p, _p, _p, _p, _p, _i, _p, _p, _p, _p]),
    "colatus_forces_noalloc": (_i, [_p, _p, _i64, _d, _d, _d, _i, _p, _p, _p, _p, _p]),
    "colatus_ftle": (_i, [_p, _p, _p, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i64, _i64,
                          _i32, _p, _p, _p, _p, _i, _p, _p, _p, _p]),
    "colatus_cosmic_time": (_i, [_d, _d, _i64, _d, _d, _d, _d, _d, ctypes.POINTER(_d), _p]),
    "colatus_forces_periodic": (_i, [_p, _p, _i64, _d, _d, _d, _d, _i, _p, _p, _p]),
    "colatus_run_periodic": (_i, [_p, _p, _p, _i64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _d,
                                  _i64, _i64, _i64, _i, _p, _p]),
    "colatus_force_vjp": (_i, [_p, _p, _i64, _d, _d, _i32, _p, _p, _i, _p, _p, _p]),
    "colatus_hubble": (_i, [_d, _d, _d, _d, _d, _d, ctypes.POINTER(_d)]),
    "colatus_strerror": (ctypes.c_char_p, [_i]),
    "colatus_set_option": (_i, [_i, _i64]),
    "colatus_get_option": (_i, [_i, ctypes.POINTER(_i64)]),
    "colatus_timer_read": (_i, [_i, ctypes.POINTER(_d), ctypes.POINTER(_i64), _i]),
    "colatus_tile_config": (_i, [_i64, _i, _i, ctypes.POINTER(_i32)]),
    "colatus_release": (_i, []),
    "colatus_version": (_i, []),
}


class ColatusError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        msg = _lib_or_none().colatus_strerror(code).decode() if _lib_or_none() else ""
        super().__init__(f"{fn} failed: {ERRORS.get(code, code)} ({msg})")


class _Batch(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int32), ("box_offsets", ctypes.c_void_p),
                ("eps", ctypes.c_void_p)]


class _Attractor(ctypes.Structure):
    _fields_ = [("strength", _d), ("x", _d * 3)]


def _attractor(att):
    """att = (S, (x, y, z)) -> pointer to a colatus_attractor, or None."""
    if att is None:
        return None, None
    S, xp = att
    xp = [float(v) for v in xp]
    if len(xp) != 3:
        raise ValueError("attractor position must have 3 components")
    a = _Attractor(float(S), (_d * 3)(*xp))
    return ctypes.byref(a), a


class _Background(ctypes.Structure):
    _fields_ = [("coefficient", _d), ("centre", _d * 3)]


def _background(bg):
    """bg = (b, (cx, cy, cz)) -> pointer to a colatus_background, or None."""
    if bg is None:
        return None, None
    b, c = bg
    c = [float(v) for v in c]
    if len(c) != 3:
        raise ValueError("background centre must have 3 components")
    o = _Background(float(b), (_d * 3)(*c))
    return ctypes.byref(o), o


def background_coefficient(cosmo):
    """b = Om_M H0^2 / 2: the Eq. (6) background coefficient consistent with
    the expansion of Eq. (2) (comoving mean matter density 3 Om_M H0^2 / (8 pi G))."""
    return 0.5 * float(cosmo["Om_M"]) * float(cosmo["H0"]) ** 2


class _Tracks(ctypes.Structure):
    _fields_ = [("n_tracers", ctypes.c_int32), ("index", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


def _tracks(tracers, rows, like):
    """tracers (sequence of particle indices) -> (pointer to a colatus_tracks,
    objects to keep alive, the device track tensor (rows, 2, 3, T))."""
    if tracers is None:
        return None, None, None
    import numpy as np
    idx = np.ascontiguousarray(np.asarray(tracers, dtype=np.int64).reshape(-1))
    track = torch.empty((rows, 2, 3, idx.size), dtype=torch.float64, device=like.device)
    t = _Tracks(int(idx.size), idx.ctypes.data_as(ctypes.c_void_p),
                ctypes.c_void_p(track.data_ptr()))
    return ctypes.byref(t), (t, idx), track


class Diag(ctypes.Structure):
    _fields_ = [("a", _d), ("t", _d), ("K", _d), ("U", _d), ("LI", _d), ("P", _d * 3),
                ("L", _d * 3), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


_LIB = None


def _lib_or_none():
    return _LIB


def lib():
    """The loaded libcolatus (ctypes.CDLL); raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libcolatus.so not found at {LIB_PATH}: build it with "
            "`python -m paper_1208_3444_amd.build` (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(fn, rc):
    if rc != 0:
        raise ColatusError(fn, rc)


def _prec(p):
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _dev(t, name, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a HIP device (got {t.device})")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    current = torch.cuda.current_device()
    if t.device.index is not None and t.device.index != current:
        raise ValueError(f"{name} is on {t.device}, but the library runs on the current "
                         f"HIP device (cuda:{current})")
    return ctypes.c_void_p(t.data_ptr())


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _batch(batch):
    """batch = (box_offsets (B+1,) int64 array-like, eps (B,) array-like) or None."""
    if batch is None:
        return None, None
    import numpy as np
    off = np.ascontiguousarray(np.asarray(batch[0], dtype=np.int64).reshape(-1))
    eps = np.ascontiguousarray(np.asarray(batch[1], dtype=np.float64).reshape(-1))
    if eps.size < 1 or off.size != eps.size + 1:
        # the library reads n_boxes + 1 offsets and n_boxes softenings
        raise ValueError(f"batch needs B + 1 box offsets for B softenings (got {off.size} "
                         f"offsets, {eps.size} softenings)")
    b = _Batch(int(eps.size), off.ctypes.data, eps.ctypes.data)
    return b, (off, eps)


def forces(x, m, eps, G=1.0, a=1.0, precision="mixed_twosum", with_phi=False, batch=None,
           attractor=None, background=None):
    """a^-3 G sum_{j != k} m_j (x_j - x_k) / (|x_j - x_k|^2 + eps^2)^{3/2}  (Eq. (1)).

    Returns acc (3, N), and phi (N,) (-G sum m_j / r) if with_phi.
    attractor: None or (S, (x, y, z)), the Eq. (10) deformation term.
    background: None or (b, (cx, cy, cz)), the Eq. (6) background term
    b (x - c) (b = background_coefficient(cosmo) for consistency with Eq. (2)).
    """
    N = m.shape[0]
    px, pm = _dev(x, "x", (3, N)), _dev(m, "m", (N,))
    acc = torch.empty_like(x)
    phi = torch.empty_like(m) if with_phi else None
    b, keep = _batch(batch)
    pa, keep_a = _attractor(attractor)
    pb, keep_b = _background(background)
    rc = lib().colatus_forces(px, pm, N, float(eps) if batch is None else 0.0, float(G),
                              float(a), _prec(precision), ctypes.c_void_p(acc.data_ptr()),
                              ctypes.c_void_p(phi.data_ptr()) if with_phi else None,
                              ctypes.byref(b) if b is not None else None, pa, pb, _stream(x))
    del keep, keep_a, keep_b
    _check("colatus_forces", rc)
    return (acc, phi) if with_phi else acc


def forces_periodic(x, m, eps, box, G=1.0, a=1.0, precision="mixed_twosum", with_phi=False):
    """The periodic comoving field (Ewald summation, box side `box`, mean
    density removed, nearest image Plummer-softened), times a^-3: acc (3, N),
    and phi (N,) if with_phi (colatus_forces_periodic)."""
    N = m.shape[0]
    px, pm = _dev(x, "x", (3, N)), _dev(m, "m", (N,))
    acc = torch.empty_like(x)
    phi = torch.empty_like(m) if with_phi else None
    rc = lib().colatus_forces_periodic(px, pm, N, float(eps), float(G), float(a), float(box),
                                       _prec(precision), ctypes.c_void_p(acc.data_ptr()),
                                       ctypes.c_void_p(phi.data_ptr()) if with_phi else None,
                                       _stream(x))
    _check("colatus_forces_periodic", rc)
    return (acc, phi) if with_phi else acc


def run_periodic(x, v, m, eps, G, cosmo, box, a_begin, a_end, n_steps, first_step=0,
                 last_step=None, precision="mixed_twosum", diag=False):
    """Kick-drift-kick steps with the periodic field, positions wrapped into
    [0, box) after each drift, in place (colatus_run_periodic).  Returns the
    diagnostics dict if diag, else None."""
    if last_step is None:
        last_step = n_steps
    N = m.shape[0]
    px, pv, pm = _dev(x, "x", (3, N)), _dev(v, "v", (3, N)), _dev(m, "m", (N,))
    nr = last_step - first_step + 1
    rows = (Diag * nr)() if diag else None
    rc = lib().colatus_run_periodic(px, pv, pm, N, float(eps), float(G), *_cosmo(cosmo),
                                    float(box), float(a_begin), float(a_end), int(n_steps),
                                    int(first_step), int(last_step), _prec(precision),
                                    ctypes.cast(rows, ctypes.c_void_p) if diag else None,
                                    _stream(x))
    _check("colatus_run_periodic", rc)
    return _diag_dict(rows) if diag else None


def _cosmo(c):
    return (float(c["H0"]), float(c["Om_R"]), float(c["Om_M"]), float(c["Om_K"]),
            float(c["Om_L"]))


def step(x, v, m, eps, G, cosmo, a, a_next, precision="mixed_twosum", batch=None,
         attractor=None, background=None, g_cache=None):
    """One kick-drift-kick step from a to a_next, in place on x and v.

    g_cache: None, or a (3, N) tensor holding g at the current positions
    (forces(..., a=1.0) or the previous step's); it is used for the opening
    kick and overwritten with g at the new positions (one force evaluation
    per step instead of two)."""
    N = m.shape[0]
    px, pv, pm = _dev(x, "x", (3, N)), _dev(v, "v", (3, N)), _dev(m, "m", (N,))
    b, keep = _batch(batch)
    pa, keep_a = _attractor(attractor)
    pb, keep_b = _background(background)
    pg = _dev(g_cache, "g_cache", (3, N)) if g_cache is not None else None
    rc = lib().colatus_step(px, pv, pm, N, float(eps) if batch is None else 0.0, float(G),
                            *_cosmo(cosmo), float(a), float(a_next), _prec(precision), pg,
                            ctypes.byref(b) if b is not None else None, pa, pb, _stream(x))
    del keep, keep_a, keep_b
    _check("colatus_step", rc)


DIAG_FIELDS = ("a", "t", "K", "U", "LI", "Px", "Py", "Pz", "Lx", "Ly", "Lz", "flags")


def _diag_dict(rows):
    import numpy as np
    out = {f: np.empty(len(rows)) for f in DIAG_FIELDS}
    for i, r in enumerate(rows):
        out["a"][i], out["t"][i], out["K"][i], out["U"][i], out["LI"][i] = r.a, r.t, r.K, r.U, r.LI
        out["Px"][i], out["Py"][i], out["Pz"][i] = r.P[0], r.P[1], r.P[2]
        out["Lx"][i], out["Ly"][i], out["Lz"][i] = r.L[0], r.L[1], r.L[2]
        out["flags"][i] = r.flags
    return out


def run(x, v, m, eps, G, cosmo, a_begin, a_end, n_steps, first_step=0, last_step=None,
        precision="mixed_twosum", diag=False, batch=None, attractor=None, scheme="kdk",
        tracers=None, background=None):
    """Kick-drift-kick steps [first_step, last_step) of the global ln-a grid, in place.

    Returns the diagnostics (dict of numpy arrays, one entry per grid point;
    with a batch, a list of such dicts, one per box) if diag, else None.
    attractor: None or (S, (x, y, z)), the Eq. (10) deformation term.
    background: None or (b, (cx, cy, cz)), the Eq. (6) background term.
    scheme: 'kdk' (the Eq. (9) operators, colatus_run) or 'he' (the paper's
    difference equations, Eqs. (3)-(5), colatus_run_he).
    tracers: None or particle indices; then the return value is the pair
    (diagnostics or None, track), track a device tensor (rows, 2, 3, T) of
    x and v = dx/dt of each tracer at every grid point of the call.
    """
    if last_step is None:
        last_step = n_steps
    N = m.shape[0]
    px, pv, pm = _dev(x, "x", (3, N)), _dev(v, "v", (3, N)), _dev(m, "m", (N,))
    b, keep = _batch(batch)
    pa, keep_a = _attractor(attractor)
    n_boxes = 1 if batch is None else len(keep[1])
    nr = last_step - first_step + 1
    rows = (Diag * (n_boxes * nr))() if diag else None
    if scheme not in ("kdk", "he"):
        raise ValueError("scheme must be 'kdk' (Eq. (9) operators) or 'he' (Eqs. (3)-(5))")
    pt, keep_t, track = _tracks(tracers, nr, x)
    pb, keep_b = _background(background)
    fn = lib().colatus_run if scheme == "kdk" else lib().colatus_run_he
    rc = fn(px, pv, pm, N, float(eps) if batch is None else 0.0, float(G),
            *_cosmo(cosmo), float(a_begin), float(a_end), int(n_steps),
            int(first_step), int(last_step), _prec(precision),
            ctypes.cast(rows, ctypes.c_void_p) if diag else None,
            ctypes.byref(b) if b is not None else None, pa, pb, pt, _stream(x))
    del keep, keep_a, keep_t, keep_b
    _check("colatus_run" if scheme == "kdk" else "colatus_run_he", rc)
    d = None
    if diag:
        per_box = [_diag_dict(rows[k * nr:(k + 1) * nr]) for k in range(n_boxes)]
        d = per_box[0] if batch is None else per_box
    return d if tracers is None else (d, track)


def velocity_spectrum(track, remove_mean=False):
    """Periodogram of each tracer's velocity over the rows of a track
    (rows, 2, 3, T) on the device: out[t, k] = (1/rows) sum_c |sum_n
    w_c[n] exp(-2 pi i k n / rows)|^2, k = 0..rows//2, w = v (less its mean
    over the rows if remove_mean).  Returns a (T, rows//2 + 1) tensor."""
    if track.dim() != 4 or track.shape[1] != 2 or track.shape[2] != 3:
        raise ValueError("track must be (rows, 2, 3, T)")
    M, T = track.shape[0], track.shape[3]
    pt = _dev(track, "track", tuple(track.shape))
    out = torch.empty((T, M // 2 + 1), dtype=torch.float64, device=track.device)
    rc = lib().colatus_velocity_spectrum(pt, M, T, 1 if remove_mean else 0,
                                         ctypes.c_void_p(out.data_ptr()), _stream(track))
    _check("colatus_velocity_spectrum", rc)
    return out


def force_vjp(x, m, lam, eps, G=1.0, precision="mixed_twosum", attractor=None,
              background=None):
    """J(x)^T lam for the comoving sum (pair sum, plus the Eq. (10) attractor
    and the Eq. (6) background term if given); lam (3, N) or (C, 3, N)."""
    N = m.shape[0]
    px, pm = _dev(x, "x", (3, N)), _dev(m, "m", (N,))
    C = 1 if lam.dim() == 2 else lam.shape[0]
    pl = _dev(lam, "lam", (3, N) if lam.dim() == 2 else (C, 3, N))
    out = torch.empty_like(lam)
    pa, keep_a = _attractor(attractor)
    pb, keep_b = _background(background)
    rc = lib().colatus_force_vjp(px, pm, N, float(eps), float(G), C, pl,
                                 ctypes.c_void_p(out.data_ptr()), _prec(precision), pa, pb,
                                 _stream(x))
    del keep_a, keep_b
    _check("colatus_force_vjp", rc)
    return out


def adjoint(x0, v0, m, eps, G, cosmo, a_begin, a_end, n_steps, lam_xN, lam_vN,
            checkpoint_every=-1, precision="mixed_twosum", return_state=False,
            attractor=None, background=None, batch=None):
    """Gradients of <lam_xN, x_N> + <lam_vN, v_N> with respect to (x_0, v_0).

    lam_xN, lam_vN: (3, N) or (C, 3, N).  Returns (grad_x0, grad_v0) shaped
    like the cotangents, plus (x_N, v_N) if return_state.  checkpoint_every:
    K >= 1 stores the state every K steps and recomputes the segments; 0 keeps
    every position (24 B per particle and step) and recomputes nothing.  With an attractor
    (S, (x, y, z)) (Eq. (10)) the run includes it and the gradient with
    respect to (S, x_psi) is appended: (4,) or (C, 4).  background: the
    Eq. (6) term (b, (cx, cy, cz)) of the run, or None.  batch: as in run().
    """
    N = m.shape[0]
    px, pv, pm = _dev(x0, "x0", (3, N)), _dev(v0, "v0", (3, N)), _dev(m, "m", (N,))
    b, keep = _batch(batch)
    C = 1 if lam_xN.dim() == 2 else lam_xN.shape[0]
    shp = (3, N) if lam_xN.dim() == 2 else (C, 3, N)
    plx, plv = _dev(lam_xN, "lam_xN", shp), _dev(lam_vN, "lam_vN", shp)
    gx, gv = torch.empty_like(lam_xN), torch.empty_like(lam_vN)
    xN = torch.empty_like(x0) if return_state else None
    vN = torch.empty_like(v0) if return_state else None
    pa, keep_a = _attractor(attractor)
    pb, keep_b = _background(background)
    ga = None
    if attractor is not None:
        ga = torch.empty((4,) if lam_xN.dim() == 2 else (C, 4), dtype=torch.float64,
                         device=x0.device)
    rc = lib().colatus_adjoint(
        px, pv, pm, N, float(eps) if batch is None else 0.0, float(G), *_cosmo(cosmo),
        float(a_begin), float(a_end),
        int(n_steps), int(checkpoint_every), C, plx, plv, ctypes.c_void_p(gx.data_ptr()),
        ctypes.c_void_p(gv.data_ptr()),
        ctypes.c_void_p(xN.data_ptr()) if return_state else None,
        ctypes.c_void_p(vN.data_ptr()) if return_state else None,
        ctypes.c_void_p(ga.data_ptr()) if ga is not None else None,
        _prec(precision), ctypes.byref(b) if b is not None else None, pa, pb, _stream(x0))
    del keep, keep_a, keep_b
    _check("colatus_adjoint", rc)
    out = (gx, gv) + ((xN, vN) if return_state else ())
    if ga is not None:
        out = out + (ga,)
    return out


class ColatusRun(torch.autograd.Function):
    """(x_0, v_0) -> (x_N, v_N) of a full run, differentiable by the discrete adjoint.

    ``ColatusRun.apply(x0, v0, m, params)`` with params a dict holding eps, G,
    cosmo, a_begin, a_end, n_steps and optionally checkpoint_every, precision,
    attractor (S, (x, y, z)) and background (b, (cx, cy, cz)).  The backward
    pass calls colatus_adjoint, which re-runs the forward with checkpoints and
    returns gradients for x0 and v0.
    """

    @staticmethod
    def forward(ctx, x0, v0, m, params):
        x = x0.detach().clone()
        v = v0.detach().clone()
        run(x, v, m, params["eps"], params["G"], params["cosmo"], params["a_begin"],
            params["a_end"], params["n_steps"], precision=params.get("precision", "mixed_twosum"),
            attractor=params.get("attractor"), background=params.get("background"))
        ctx.save_for_backward(x0.detach(), v0.detach(), m)
        ctx.params = params
        return x, v

    @staticmethod
    def backward(ctx, gx, gv):
        x0, v0, m = ctx.saved_tensors
        P = ctx.params
        gx = torch.zeros_like(x0) if gx is None else gx.contiguous()
        gv = torch.zeros_like(v0) if gv is None else gv.contiguous()
        res = adjoint(x0, v0, m, P["eps"], P["G"], P["cosmo"], P["a_begin"], P["a_end"],
                      P["n_steps"], gx, gv, checkpoint_every=P.get("checkpoint_every", -1),
                      precision=P.get("precision", "mixed_twosum"),
                      attractor=P.get("attractor"), background=P.get("background"))
        return res[0], res[1], None, None


def ftle(x0, v0, m, eps, G, cosmo, a_begin, a_end, n_steps, tracers, checkpoint_every=-1,
         precision="mixed_twosum", attractor=None, background=None, batch=None):
    """Finite-time Lyapunov exponents of tracer particles (colatus_ftle).

    The library reads the 3x3 block d x_t(a_end) / d x_t(a_begin) of each
    tracer off one adjoint pass (3 unit cotangents per tracer) and takes
    ln sigma_max over the elapsed cosmic time and over ln(a_end / a_begin).
    Returns device tensors (lambda per unit cosmic time (T,), lambda per unit
    ln a (T,), blocks (T, 3, 3)).
    """
    import numpy as np
    N = m.shape[0]
    px, pv, pm = _dev(x0, "x0", (3, N)), _dev(v0, "v0", (3, N)), _dev(m, "m", (N,))
    idx = np.ascontiguousarray(np.asarray(tracers, dtype=np.int64).reshape(-1))
    T = int(idx.size)
    lam_t = torch.empty(T, dtype=torch.float64, device=x0.device)
    lam_lna = torch.empty_like(lam_t)
    blocks = torch.empty((T, 3, 3), dtype=torch.float64, device=x0.device)
    b, keep = _batch(batch)
    pa, keep_a = _attractor(attractor)
    pb, keep_b = _background(background)
    rc = lib().colatus_ftle(
        px, pv, pm, N, float(eps) if batch is None else 0.0, float(G), *_cosmo(cosmo),
        float(a_begin), float(a_end), int(n_steps), int(checkpoint_every), T,
        idx.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(lam_t.data_ptr()),
        ctypes.c_void_p(lam_lna.data_ptr()), ctypes.c_void_p(blocks.data_ptr()),
        _prec(precision), ctypes.byref(b) if b is not None else None, pa, pb, _stream(x0))
    del keep, keep_a, keep_b, idx
    _check("colatus_ftle", rc)
    return lam_t, lam_lna, blocks


def cosmic_time(cosmo, a_begin, a_end, n_steps, device=None):
    """Cosmic time elapsed over the run's grid (colatus_cosmic_time): the sum
    of the steps' Friedmann time integrals, as the diagnostics' t reports."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = ctypes.c_double()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check("colatus_cosmic_time",
           lib().colatus_cosmic_time(float(a_begin), float(a_end), int(n_steps), *_cosmo(cosmo),
                                     ctypes.byref(out), stream))
    return out.value


def hubble(a, cosmo):
    """H(a) of Eq. (2), computed by the library on the host."""
    out = ctypes.c_double()
    _check("colatus_hubble", lib().colatus_hubble(float(a), *_cosmo(cosmo), ctypes.byref(out)))
    return out.value


def set_option(key, value):
    _check("colatus_set_option", lib().colatus_set_option(int(key), int(value)))


def get_option(key):
    out = ctypes.c_int64()
    _check("colatus_get_option", lib().colatus_get_option(int(key), ctypes.byref(out)))
    return out.value


def timer_read(kind=0, reset=True):
    """(total ms, launches) of the pair sweeps timed since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check("colatus_timer_read", lib().colatus_timer_read(int(kind), ctypes.byref(ms),
                                                          ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def tile_config(N, precision="mixed_twosum", kind=0):
    """(targets per lane, threads per block, source slices, pair-loop form)."""
    out = (ctypes.c_int32 * 4)()
    _check("colatus_tile_config", lib().colatus_tile_config(int(N), _prec(precision), int(kind),
                                                            out))
    return tuple(out)


def release():
    _check("colatus_release", lib().colatus_release())


def version():
    return lib().colatus_version()
