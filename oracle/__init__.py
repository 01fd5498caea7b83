"""FP64 CPU oracle for the COLATUS hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_1208_3444_amd``) and never imports it.

Every function is a thin numpy wrapper over ``colatus_oracle.c``; the
arithmetic, and the citation of the paper passage each function follows,
lives there:

* ``forces``           -- Eq. (1) pair sum, a^-3 G sum m_j (x_j - x_k) r^-3
                          (+ the Eq. (10) attractor when given)
* ``potential``        -- softened potential whose gradient is that sum
* ``force_vjp``        -- transpose Jacobian of the comoving pair sum
* ``attractor_field``, ``attractor_vjp`` -- the Eq. (10) deformation term
  alone: a fixed point of strength S = C psi at x_psi
* ``hubble``           -- Eq. (2)
* ``time_integral``    -- the cosmic-time, kick and drift integrals of Eq. (9)
* ``step_coefficients``-- the kick/drift/kick coefficients of one step
* ``run``              -- kick-drift-kick run built from Eq. (9), diagnostics
* ``run_he``           -- the paper's difference equations, Eqs. (3)-(5)
* ``he_coefficients``  -- (tau, a, H) of one step of ``run_he``
* ``adjoint``          -- discrete reverse mode of ``run``
* ``ftle``             -- finite-time Lyapunov exponent of tracer particles

Arrays are float64, positions and velocities structure-of-arrays ``(3, N)``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DIAG_FIELDS = ("a", "t", "K", "U", "LI", "Px", "Py", "Pz", "Lx", "Ly", "Lz")

_d = ctypes.c_double
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.restype = None
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_hubble.restype = _d
    lib.oracle_hubble.argtypes = [_d] * 6
    lib.oracle_time_integral.restype = _d
    lib.oracle_time_integral.argtypes = [ctypes.c_int] + [_d] * 7
    lib.oracle_step_coefficients.restype = None
    lib.oracle_step_coefficients.argtypes = [_d] * 7 + [_i64, _i64, _p]
    lib.oracle_forces.restype = None
    lib.oracle_forces.argtypes = [_p, _p, _i64, _d, _d, _d, _p]
    lib.oracle_forces_targets.restype = None
    lib.oracle_forces_targets.argtypes = [_p, _p, _i64, _p, _i64, _d, _d, _d, _p]
    lib.oracle_potential.restype = None
    lib.oracle_potential.argtypes = [_p, _p, _i64, _d, _d, _p]
    lib.oracle_force_vjp.restype = None
    lib.oracle_force_vjp.argtypes = [_p, _p, _i64, _d, _d, _p, _p]
    lib.oracle_attractor_add.restype = None
    lib.oracle_attractor_add.argtypes = [_p, _i64, _d, _d, _p, _p, _p]
    lib.oracle_attractor_vjp.restype = None
    lib.oracle_attractor_vjp.argtypes = [_p, _i64, _d, _d, _p, _p, _p]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run.argtypes = [_p, _p, _p, _i64, _d, _d] + [_d] * 5 + \
        [_d, _d, _i64, _i64, _i64, _p, _d, _p, _d, _p, _p, _i64, _p]
    lib.oracle_run_he.restype = ctypes.c_int
    lib.oracle_run_he.argtypes = [_p, _p, _p, _i64, _d, _d] + [_d] * 5 + \
        [_d, _d, _i64, _i64, _i64, _p, _d, _p, _d, _p, _p, _i64, _p]
    lib.oracle_background_add.restype = None
    lib.oracle_background_add.argtypes = [_p, _i64, _d, _p, _p, _p]
    lib.oracle_forces_periodic.restype = None
    lib.oracle_forces_periodic.argtypes = [_p, _p, _i64, _d, _d, _d, _d, _d, ctypes.c_int,
                                           ctypes.c_int, _p, _i64, _p, _p]
    lib.oracle_velocity_spectrum_bins.restype = None
    lib.oracle_velocity_spectrum_bins.argtypes = [_p, _i64, _i64, ctypes.c_int, _p, _i64, _p]
    lib.oracle_velocity_spectrum.restype = None
    lib.oracle_velocity_spectrum.argtypes = [_p, _i64, _i64, ctypes.c_int, _p]
    lib.oracle_he_coefficients.restype = None
    lib.oracle_he_coefficients.argtypes = [_d] * 7 + [_i64, _i64, _p]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_adjoint.argtypes = [_p, _p, _p, _i64, _d, _d] + [_d] * 5 + \
        [_d, _d, _i64, _i32, _p, _p, _p, _p, _p, _p, _d, _p, _d, _p, _p]
    _lib = lib
    return lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return a.ctypes.data_as(_p) if a is not None else None


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def hubble(a, H0, Om_R, Om_M, Om_K, Om_L):
    return _load().oracle_hubble(a, H0, Om_R, Om_M, Om_K, Om_L)


def time_integral(kind, a1, a2, H0, Om_R, Om_M, Om_K, Om_L):
    """kind: 'time' -> int da/(aH), 'kick' -> int da/(a^2 H), 'drift' -> int da/(a^3 H)."""
    k = {"time": 1, "kick": 2, "drift": 3}[kind]
    return _load().oracle_time_integral(k, a1, a2, H0, Om_R, Om_M, Om_K, Om_L)


def step_coefficients(cosmo, a_begin, a_end, n_steps, n):
    """(k1, d, k2, dt) of step n of the global grid."""
    out = np.zeros(4)
    _load().oracle_step_coefficients(
        cosmo["H0"], cosmo["Om_R"], cosmo["Om_M"], cosmo["Om_K"], cosmo["Om_L"],
        a_begin, a_end, n_steps, n, _ptr(out))
    return tuple(out)


def _att(attractor):
    """(S, xpsi array or None) from None or (S, (x, y, z))."""
    if attractor is None:
        return 0.0, None
    S, xp = attractor
    return float(S), np.ascontiguousarray(xp, dtype=np.float64).reshape(3)


def attractor_field(x, eps, attractor):
    """(f, phi_ext): the Eq. (10) term added to the comoving sum g and its
    potential, for attractor = (S, (x, y, z))."""
    x = _c(x)
    N = x.shape[1]
    S, xp = _att(attractor)
    f = np.zeros((3, N))
    phi = np.zeros(N)
    _load().oracle_attractor_add(_ptr(x), N, eps, S, _ptr(xp), _ptr(f), _ptr(phi))
    return f, phi


def _bg(background):
    """(b, centre array or None) from None or (b, (cx, cy, cz))."""
    if background is None:
        return 0.0, None
    b, c = background
    return float(b), np.ascontiguousarray(c, dtype=np.float64).reshape(3)


def background_coefficient(cosmo):
    """b = Om_M H0^2 / 2, the Eq. (6) background coefficient consistent with
    Eq. (2): (4 pi G / 3) times the comoving mean matter density."""
    return 0.5 * cosmo["Om_M"] * cosmo["H0"] ** 2


def background_field(x, background):
    """(f, phi_ext): the Eq. (6) background term b (x - c) added to the
    comoving sum g and its potential -b |x - c|^2 / 2."""
    x = _c(x)
    N = x.shape[1]
    b, c = _bg(background)
    f = np.zeros((3, N))
    phi = np.zeros(N)
    _load().oracle_background_add(_ptr(x), N, b, _ptr(c), _ptr(f), _ptr(phi))
    return f, phi


def attractor_vjp(x, lam, eps, attractor):
    x = _c(x)
    lam = _c(lam)
    N = x.shape[1]
    S, xp = _att(attractor)
    out = np.empty((3, N))
    _load().oracle_attractor_vjp(_ptr(x), N, eps, S, _ptr(xp), _ptr(lam), _ptr(out))
    return out


def forces(x, m, eps, G=1.0, a=1.0, attractor=None, background=None):
    x = _c(x)
    m = _c(m)
    N = m.shape[0]
    assert x.shape == (3, N)
    acc = np.empty((3, N))
    _load().oracle_forces(_ptr(x), _ptr(m), N, eps, G, a, _ptr(acc))
    if attractor is not None:
        acc += attractor_field(x, eps, attractor)[0] / a ** 3
    if background is not None:
        acc += background_field(x, background)[0] / a ** 3
    return acc


def forces_targets(x, m, targets, eps, G=1.0, a=1.0):
    x = _c(x)
    m = _c(m)
    N = m.shape[0]
    t = np.ascontiguousarray(targets, dtype=np.int64)
    acc = np.empty((3, t.shape[0]))
    _load().oracle_forces_targets(_ptr(x), _ptr(m), N, _ptr(t), t.shape[0],
                                  eps, G, a, _ptr(acc))
    return acc


def periodic_cutoffs(L, alpha=None):
    """Splitting parameter and cutoffs of the oracle's Ewald sums: alpha = 6/L
    by default; the real-space images around the nearest one (|n_i| <= 1:
    every omitted image lies 1.5 L away or more, erfc(1.5 alpha L) < 1e-35
    for alpha L >= 6), and the reciprocal vectors |n| <= n_kmax with
    exp(-pi^2 n^2 / (alpha L)^2) below 1e-18 beyond."""
    if alpha is None:
        alpha = 6.0 / L
    aL = alpha * L
    assert aL >= 4.0, "real-space images |n_i| <= 1 need alpha L >= 4"
    n_kmax = int(np.ceil(aL * np.sqrt(18.0 * np.log(10.0)) / np.pi))
    return alpha, 1, n_kmax


def forces_periodic(x, m, eps, L, G=1.0, a=1.0, with_phi=False, targets=None, alpha=None):
    """Periodic comoving field (Ewald summation in a box of side L, mean
    density removed, nearest image Plummer-softened): acc (3, N) or
    (3, n_targets), and phi if with_phi.  alpha: the Ewald splitting
    parameter (the result does not depend on it)."""
    x = _c(x)
    m = _c(m)
    N = m.shape[0]
    assert x.shape == (3, N)
    alpha, n_img, n_kmax = periodic_cutoffs(L, alpha)
    t = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = N if t is None else t.shape[0]
    acc = np.empty((3, nt))
    phi = np.empty(nt) if with_phi else None
    _load().oracle_forces_periodic(_ptr(x), _ptr(m), N, eps, G, a, L, alpha, n_img, n_kmax,
                                   _ptr(t), nt, _ptr(acc), _ptr(phi))
    return (acc, phi) if with_phi else acc


def run_periodic(x, v, m, eps, G, cosmo, L, a_begin, a_end, n_steps, first_step=0,
                 last_step=None):
    """Kick-drift-kick steps [first_step, last_step) of the run's grid (the
    same steps and coefficients as run()) with the periodic field, each
    drift followed by the wrap of every position into [0, L).  Written
    step by step in Python on top of the pinned periodic field and step
    coefficients.  Returns (x, v)."""
    if last_step is None:
        last_step = n_steps
    x = _c(x).copy()
    v = _c(v).copy()
    def grid_a(n):  # a_n = a_begin exp(n ln(a_end / a_begin) / n_steps), as run()
        if cosmo["H0"] == 0:
            return a_begin
        if n == n_steps:
            return a_end
        return a_begin * np.exp(n * (np.log(a_end / a_begin) / n_steps))

    a0 = grid_a(first_step)
    p = a0 * a0 * v
    g = forces_periodic(x, m, eps, L, G=G, a=1.0)
    for n in range(first_step, last_step):
        k1, d, k2, _ = step_coefficients(cosmo, a_begin, a_end, n_steps, n)
        p = p + k1 * g
        x = x + d * p
        x = x - L * np.floor(x / L)
        g = forces_periodic(x, m, eps, L, G=G, a=1.0)
        p = p + k2 * g
    a1 = grid_a(last_step)
    return x, p / (a1 * a1)


def potential(x, m, eps, G=1.0, attractor=None, background=None):
    x = _c(x)
    m = _c(m)
    N = m.shape[0]
    phi = np.empty(N)
    _load().oracle_potential(_ptr(x), _ptr(m), N, eps, G, _ptr(phi))
    if attractor is not None:
        phi += attractor_field(x, eps, attractor)[1]
    if background is not None:
        phi += background_field(x, background)[1]
    return phi


def force_vjp(x, m, lam, eps, G=1.0, attractor=None, background=None):
    x = _c(x)
    m = _c(m)
    lam = _c(lam)
    N = m.shape[0]
    out = np.empty((3, N))
    _load().oracle_force_vjp(_ptr(x), _ptr(m), N, eps, G, _ptr(lam), _ptr(out))
    if attractor is not None:
        out += attractor_vjp(x, lam, eps, attractor)
    if background is not None:
        out += _bg(background)[0] * lam
    return out


def _run(fn, name, x, v, m, eps, G, cosmo, a_begin, a_end, n_steps, first_step, last_step,
         diag, attractor, tracers, background):
    if last_step is None:
        last_step = n_steps
    x = _c(x).copy()
    v = _c(v).copy()
    m = _c(m)
    N = m.shape[0]
    S, xp = _att(attractor)
    bb, bc = _bg(background)
    nr = last_step - first_step + 1
    rows = np.zeros((nr, len(DIAG_FIELDS))) if diag else None
    trk = track = None
    if tracers is not None:
        trk = np.ascontiguousarray(tracers, dtype=np.int64)
        if trk.ndim != 1 or trk.size == 0 or trk.min() < 0 or trk.max() >= N:
            raise ValueError(f"{name}: tracers must be indices in [0, N)")
        track = np.zeros((nr, 2, 3, trk.size))
    rc = fn(_ptr(x), _ptr(v), _ptr(m), N, eps, G, cosmo["H0"], cosmo["Om_R"],
            cosmo["Om_M"], cosmo["Om_K"], cosmo["Om_L"], a_begin, a_end, n_steps,
            first_step, last_step, _ptr(rows), S, _ptr(xp), bb, _ptr(bc),
            trk.ctypes.data_as(_p) if trk is not None else None,
            0 if trk is None else trk.size, _ptr(track))
    if rc != 0:
        raise ValueError(f"{name}: invalid arguments")
    out = [x, v]
    if diag:
        out.append({f: rows[:, i].copy() for i, f in enumerate(DIAG_FIELDS)})
    if tracers is not None:
        out.append(track)
    return tuple(out)


def run(x, v, m, eps, G, cosmo, a_begin, a_end, n_steps, first_step=0,
        last_step=None, diag=False, attractor=None, tracers=None, background=None):
    """Kick-drift-kick run over steps first_step..last_step-1 of the grid.

    Returns (x, v) at a_{last_step}, then the diagnostics rows (dict of
    arrays) if diag is true, then the tracer track (rows, 2, 3, T) -- x and
    v = dx/dt of particles ``tracers`` at every grid point -- if tracers is
    given.  attractor: None or (S, (x, y, z)), the Eq. (10) term; background:
    None or (b, (cx, cy, cz)), the Eq. (6) term.
    """
    return _run(_load().oracle_run, "oracle_run", x, v, m, eps, G, cosmo, a_begin, a_end,
                n_steps, first_step, last_step, diag, attractor, tracers, background)


def run_he(x, v, m, eps, G, cosmo, a_begin, a_end, n_steps, first_step=0,
           last_step=None, diag=False, attractor=None, tracers=None, background=None):
    """Steps of the paper's difference equations (Eqs. (3)-(5)) on the same
    grid as ``run``; returns as ``run``."""
    return _run(_load().oracle_run_he, "oracle_run_he", x, v, m, eps, G, cosmo, a_begin,
                a_end, n_steps, first_step, last_step, diag, attractor, tracers, background)


def velocity_spectrum_bins(track, bins, remove_mean=False):
    """``velocity_spectrum`` at the given bins only: (T, len(bins))."""
    track = _c(track)
    M, two, three, T = track.shape
    assert two == 2 and three == 3
    b = np.ascontiguousarray(bins, dtype=np.int64)
    out = np.zeros((T, b.size))
    _load().oracle_velocity_spectrum_bins(_ptr(track), M, T, 1 if remove_mean else 0,
                                          b.ctypes.data_as(_p), b.size, _ptr(out))
    return out


def velocity_spectrum(track, remove_mean=False):
    """Periodogram of each tracer's velocity over the rows of a track
    (rows, 2, 3, T): E[t, k] = (1/M) sum_c |sum_n w_c[n] e^{-2 pi i k n/M}|^2,
    k = 0..M/2, w = v (less its mean if remove_mean).  Returns (T, M//2 + 1)."""
    track = _c(track)
    M, two, three, T = track.shape
    assert two == 2 and three == 3
    out = np.zeros((T, M // 2 + 1))
    _load().oracle_velocity_spectrum(_ptr(track), M, T, 1 if remove_mean else 0, _ptr(out))
    return out


def he_coefficients(cosmo, a_begin, a_end, n_steps, n):
    """(tau, a_half, H_half) of step n of ``run_he``."""
    out = np.zeros(3)
    _load().oracle_he_coefficients(
        cosmo["H0"], cosmo["Om_R"], cosmo["Om_M"], cosmo["Om_K"], cosmo["Om_L"],
        a_begin, a_end, n_steps, n, _ptr(out))
    return tuple(out)


def adjoint(x0, v0, m, eps, G, cosmo, a_begin, a_end, n_steps, lam_xN, lam_vN,
            attractor=None, background=None):
    """Gradients of <lam_xN, x_N> + <lam_vN, v_N> with respect to (x0, v0).

    lam_xN, lam_vN: (C, 3, N) or (3, N).  Returns (grad_x0, grad_v0, xN, vN)
    with the gradients shaped like the cotangents; with an attractor
    (S, (x, y, z)) also grad_att, (C, 4) (or (4,)): d/dS, d/dx_psi.
    """
    x0 = _c(x0)
    v0 = _c(v0)
    m = _c(m)
    N = m.shape[0]
    lx = _c(lam_xN)
    lv = _c(lam_vN)
    squeeze = lx.ndim == 2
    lx = lx.reshape(-1, 3, N)
    lv = lv.reshape(-1, 3, N)
    C = lx.shape[0]
    gx = np.empty_like(lx)
    gv = np.empty_like(lv)
    xN = np.empty((3, N))
    vN = np.empty((3, N))
    S, xp = _att(attractor)
    bb, bc = _bg(background)
    ga = np.zeros((C, 4)) if attractor is not None else None
    rc = _load().oracle_adjoint(
        _ptr(x0), _ptr(v0), _ptr(m), N, eps, G, cosmo["H0"], cosmo["Om_R"],
        cosmo["Om_M"], cosmo["Om_K"], cosmo["Om_L"], a_begin, a_end, n_steps,
        C, _ptr(lx), _ptr(lv), _ptr(gx), _ptr(gv), _ptr(xN), _ptr(vN), S, _ptr(xp),
        bb, _ptr(bc), _ptr(ga))
    if rc != 0:
        raise ValueError("oracle_adjoint: invalid arguments")
    if squeeze:
        gx, gv = gx[0], gv[0]
        ga = ga[0] if ga is not None else None
    if attractor is not None:
        return gx, gv, xN, vN, ga
    return gx, gv, xN, vN


def ftle(x0, v0, m, eps, G, cosmo, a_begin, a_end, n_steps, tracers):
    """Finite-time Lyapunov exponent of each tracer particle.

    The 3x3 block Phi_t = d x_t(a_end) / d x_t(a_begin) of the flow map is
    read off three reverse sweeps seeded with the unit vectors on x_t(a_end);
    lambda_t = ln sigma_max(Phi_t) / (t(a_end) - t(a_begin)), with the
    cosmic time from the Friedmann integral (or the elapsed time in the
    static limit).  Returns (lambda per unit cosmic time, lambda per unit
    ln a, the blocks Phi).
    """
    m = _c(m)
    N = m.shape[0]
    tracers = np.asarray(tracers, dtype=np.int64)
    T = tracers.shape[0]
    lam_x = np.zeros((3 * T, 3, N))
    for ti, t in enumerate(tracers):
        for i in range(3):
            lam_x[3 * ti + i, i, t] = 1.0
    lam_v = np.zeros_like(lam_x)
    gx, _, _, _ = adjoint(x0, v0, m, eps, G, cosmo, a_begin, a_end, n_steps,
                          lam_x, lam_v)
    phi = np.empty((T, 3, 3))
    for ti, t in enumerate(tracers):
        for i in range(3):
            phi[ti, i, :] = gx[3 * ti + i, :, t]
    smax = np.linalg.svd(phi, compute_uv=False)[:, 0]
    if cosmo["H0"] == 0.0:
        span_t = a_end
        span_lna = float("nan")
    else:
        span_t = time_integral("time", a_begin, a_end, cosmo["H0"], cosmo["Om_R"],
                               cosmo["Om_M"], cosmo["Om_K"], cosmo["Om_L"])
        span_lna = np.log(a_end / a_begin)
    lam = np.log(smax)
    return lam / span_t, lam / span_lna, phi
