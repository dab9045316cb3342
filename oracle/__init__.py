"""CPU FP64 reference for the geodesic ray tracer (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It shares no code with the HIP
implementation in ``paper_2310_15183_amd``; see ``oracle.c`` for the
arithmetic and the passages of the paper each step follows.

Flags: 0 timeout (step limit reached), 1 escape (r > escape_factor * r0),
2 horizon (|dt/dtau| > horizon_norm), 3 invalid (non-finite state).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Flags chosen so that no product is fused behind the source's back and libm is
# used exactly as written.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
          "-std=c11", "-Wall", "-Wextra"]

FLAG_TIMEOUT, FLAG_ESCAPE, FLAG_HORIZON, FLAG_INVALID = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, plain C11)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_trace_frame.restype = i64
        lib.oracle_trace_frame.argtypes = [d, d, d, d, d, d, d, i, i, d, d, d, d, i,
                                           vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, i, i, vp]
        lib.oracle_trace_rays.restype = i64
        lib.oracle_trace_rays.argtypes = [d, d, d, d, d, d, d, i, vp, i64,
                                          vp, vp, vp, vp, vp, vp, vp, vp, i]
        lib.oracle_camera.restype = None
        lib.oracle_camera.argtypes = [d, d, d, d, d, d, d, i, i, vp, i64, vp]
        lib.oracle_inverse_metric.restype = None
        lib.oracle_inverse_metric.argtypes = [d, d, d, d, d, vp]
        lib.oracle_set_trig_mode.restype = None
        lib.oracle_set_trig_mode.argtypes = [i]
        lib.oracle_sincos.restype = None
        lib.oracle_sincos.argtypes = [vp, i64, vp]
        lib.oracle_recip_newton.restype = None
        lib.oracle_recip_newton.argtypes = [vp, vp, i64, vp]
        lib.oracle_rhs.restype = None
        lib.oracle_rhs.argtypes = [d, d, d, d, d, d, d, d, d, d, vp, vp]
        lib.oracle_trace_frame_mn.restype = i64
        lib.oracle_trace_frame_mn.argtypes = lib.oracle_trace_frame.argtypes
        lib.oracle_inverse_metric_mn.restype = None
        lib.oracle_inverse_metric_mn.argtypes = [d, d, d, d, d, vp]
        lib.oracle_rhs_mn.restype = None
        lib.oracle_rhs_mn.argtypes = [d, d, d, d, d, d, d, d, d, d, vp, vp]
        lib.oracle_exp.restype = None
        lib.oracle_exp.argtypes = [vp, i64, vp]
        lib.oracle_redshift.restype = None
        lib.oracle_redshift.argtypes = [d, d, d, d, d, d, vp, vp, vp, vp, vp, i64, vp]
        lib.oracle_redshift_mn.restype = None
        lib.oracle_redshift_mn.argtypes = lib.oracle_redshift.argtypes
        lib.oracle_disk_orbit.restype = i
        lib.oracle_disk_orbit.argtypes = [i, d, d, d, d, d, d, vp]
        lib.oracle_shade.restype = None
        lib.oracle_shade.argtypes = [i, d, d, vp, vp, vp, vp, i64, vp]
        lib.oracle_mn_consts.restype = None
        lib.oracle_mn_consts.argtypes = [d, d, d, vp]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


@dataclass
class Result:
    t: np.ndarray
    r: np.ndarray
    theta: np.ndarray
    phi: np.ndarray
    pr: np.ndarray
    ptheta: np.ndarray
    flag: np.ndarray
    steps: np.ndarray
    p0: np.ndarray | None = None   # (n, 4) initial covector, frame mode only


def _disk(disk):
    return None if disk is None else np.ascontiguousarray(disk, dtype=np.float64)


def _alloc(n):
    return [np.empty(n, np.float64) for _ in range(6)] + [np.empty(n, np.int8),
                                                          np.empty(n, np.int32)]


def trace_frame(M, a, Q, r0, theta0, phi0, fov, width, height, dt=0.01, eps=1e-8,
                horizon_norm=1e4, escape_factor=1.5, max_steps=20000, pixels=None,
                threads=None, want_p0=False, method=0, disk=None) -> Result:
    """Trace the camera rays of a width x height frame (or the listed pixels);
    method 0 is RK4, 1 explicit Euler; disk = (r_in, r_out, half_angle) adds
    the solid equatorial ring (flag 4 on hitting it)."""
    lib = _load()
    if pixels is not None:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n = int(pixels.size)
    else:
        n = int(width) * int(height)
    t, r, th, ph, pr, pth, flag, steps = _alloc(n)
    p0 = np.empty((n, 4), np.float64) if want_p0 else None
    lib.oracle_trace_frame(M, a, Q, r0, theta0, phi0, fov, int(width), int(height), dt, eps,
                           horizon_norm, escape_factor, int(max_steps), _ptr(pixels), n,
                           _ptr(t), _ptr(r), _ptr(th), _ptr(ph), _ptr(pr), _ptr(pth), _ptr(p0),
                           _ptr(flag), _ptr(steps), int(threads or default_threads()),
                           int(method), _ptr(_disk(disk)))
    return Result(t, r, th, ph, pr, pth, flag, steps, p0)


def trace_rays(M, a, Q, init, dt=0.01, eps=1e-8, horizon_norm=1e4, escape_factor=1.5,
               max_steps=20000, threads=None) -> Result:
    """Trace rays from explicit initial states, init[k] = (t, r, th, ph, p_t, p_r, p_th, p_ph)."""
    lib = _load()
    init = np.ascontiguousarray(init, dtype=np.float64).reshape(-1, 8)
    n = init.shape[0]
    t, r, th, ph, pr, pth, flag, steps = _alloc(n)
    lib.oracle_trace_rays(M, a, Q, dt, eps, horizon_norm, escape_factor, int(max_steps),
                          _ptr(init), n, _ptr(t), _ptr(r), _ptr(th), _ptr(ph), _ptr(pr),
                          _ptr(pth), _ptr(flag), _ptr(steps), int(threads or default_threads()))
    return Result(t, r, th, ph, pr, pth, flag, steps)


def camera(M, a, Q, r0, theta0, phi0, fov, width, height, pixels=None) -> np.ndarray:
    """Initial states (n, 8) = (q^mu, p_mu) of the camera rays."""
    lib = _load()
    if pixels is not None:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n = int(pixels.size)
    else:
        n = int(width) * int(height)
    out = np.empty((n, 8), np.float64)
    lib.oracle_camera(M, a, Q, r0, theta0, phi0, fov, int(width), int(height), _ptr(pixels),
                      n, _ptr(out))
    return out


def inverse_metric(M, a, Q, r, theta) -> np.ndarray:
    """(g^tt, g^tphi, g^rr, g^thth, g^phph) at (r, theta)."""
    lib = _load()
    g = np.empty(5, np.float64)
    lib.oracle_inverse_metric(M, a, Q, float(r), float(theta), _ptr(g))
    return g


def rhs(M, a, Q, r, theta, p, eps=1e-8):
    """Hamilton right-hand side at (r, theta, p): (qdot[4], (pdot_r, pdot_theta))."""
    lib = _load()
    qd = np.empty(4, np.float64)
    pd = np.empty(2, np.float64)
    lib.oracle_rhs(M, a, Q, eps, float(r), float(theta), float(p[0]), float(p[1]),
                   float(p[2]), float(p[3]), _ptr(qd), _ptr(pd))
    return qd, pd


def set_trig_mode(mode: int) -> None:
    """0: sin/cos from their series definition (default); 1: the C library."""
    _load().oracle_set_trig_mode(int(mode))


def recip_newton(x, y0) -> np.ndarray:
    """The oracle's Newton-refined reciprocal of x from y0 (an exact 1/x0 of a
    nearby x0), elementwise."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y0 = np.ascontiguousarray(y0, dtype=np.float64).ravel()
    out = np.empty_like(x)
    _load().oracle_recip_newton(_ptr(x), _ptr(y0), x.size, _ptr(out))
    return out


def sincos(x) -> tuple[np.ndarray, np.ndarray]:
    """The oracle's sin/cos definition applied elementwise."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    sc = np.empty((x.size, 2), np.float64)
    _load().oracle_sincos(_ptr(x), x.size, _ptr(sc))
    return sc[:, 0], sc[:, 1]


# ---------------------------------------------------------------- Manko-Novikov
def trace_frame_mn(M, S, q, r0, theta0, phi0, fov, width, height, dt=0.01, eps=1e-8,
                   horizon_norm=1e4, escape_factor=1.5, max_steps=20000, pixels=None,
                   threads=None, want_p0=False, method=0, disk=None) -> Result:
    """trace_frame for the Manko-Novikov spacetime (mass M, spin S, quadrupole
    deviation q; paper Sec. 2.2.3)."""
    lib = _load()
    if pixels is not None:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        n = int(pixels.size)
    else:
        n = int(width) * int(height)
    t, r, th, ph, pr, pth, flag, steps = _alloc(n)
    p0 = np.empty((n, 4), np.float64) if want_p0 else None
    lib.oracle_trace_frame_mn(M, S, q, r0, theta0, phi0, fov, int(width), int(height), dt, eps,
                              horizon_norm, escape_factor, int(max_steps), _ptr(pixels), n,
                              _ptr(t), _ptr(r), _ptr(th), _ptr(ph), _ptr(pr), _ptr(pth),
                              _ptr(p0), _ptr(flag), _ptr(steps), int(threads or default_threads()),
                              int(method), _ptr(_disk(disk)))
    return Result(t, r, th, ph, pr, pth, flag, steps, p0)


def inverse_metric_mn(M, S, q, r, theta) -> np.ndarray:
    """Manko-Novikov (g^tt, g^tphi, g^rr, g^thth, g^phph) at (r, theta)."""
    lib = _load()
    g = np.empty(5, np.float64)
    lib.oracle_inverse_metric_mn(M, S, q, float(r), float(theta), _ptr(g))
    return g


def rhs_mn(M, S, q, r, theta, p, eps=1e-8):
    """Manko-Novikov Hamilton right-hand side: (qdot[4], (pdot_r, pdot_theta))."""
    lib = _load()
    qd = np.empty(4, np.float64)
    pd = np.empty(2, np.float64)
    lib.oracle_rhs_mn(M, S, q, eps, float(r), float(theta), float(p[0]), float(p[1]),
                      float(p[2]), float(p[3]), _ptr(qd), _ptr(pd))
    return qd, pd


def mn_consts(M, S, q) -> tuple[float, float, float]:
    """(alpha, k, beta) of the Manko-Novikov spacetime (M, S, q)."""
    out = np.empty(3, np.float64)
    _load().oracle_mn_consts(M, S, q, _ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


def exp_def(x) -> np.ndarray:
    """The oracle's exp definition applied elementwise."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.empty_like(x)
    _load().oracle_exp(_ptr(x), x.size, _ptr(out))
    return out


def shade(mode, t, theta, phi, flag, t_max=1.0, band=0.0) -> np.ndarray:
    """Colours (uint32, bytes R, G, B, A) of traced rays: mode 0 the listing's
    background bands, mode 1 the exit-time map (see oracle.c)."""
    flag = np.ascontiguousarray(flag, dtype=np.int8)
    n = flag.size
    conv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
    t, theta, phi = conv(t), conv(theta), conv(phi)
    out = np.empty(n, np.uint32)
    _load().oracle_shade(int(mode), float(t_max), float(band), _ptr(t), _ptr(theta), _ptr(phi),
                         _ptr(flag), n, _ptr(out))
    return out


# ------------------------------------------------------------------ ring redshift
def redshift(M, a, Q, r0, theta0, r, theta, pt, pph, flag, eps=1e-8, mn=False) -> np.ndarray:
    """z = lambda_O / lambda_S of rays that ended on the ring (flag 4; NaN for
    the others); (M, a, Q) are (M, S, q) with mn=True.  See oracle.c."""
    conv = lambda x: np.ascontiguousarray(x, dtype=np.float64)   # noqa: E731
    r, theta, pt, pph = conv(r), conv(theta), conv(pt), conv(pph)
    flag = np.ascontiguousarray(flag, dtype=np.int8)
    z = np.empty(flag.size)
    fn = _load().oracle_redshift_mn if mn else _load().oracle_redshift
    fn(M, a, Q, eps, r0, theta0, _ptr(r), _ptr(theta), _ptr(pt), _ptr(pph), _ptr(flag),
       flag.size, _ptr(z))
    return z


def disk_orbit(M, a, Q, r, theta=math.pi / 2, eps=1e-8, mn=False):
    """(S^t, S^phi, dphi/dt) of the ring's orbit at (r, theta), or None."""
    out = np.empty(3)
    ok = _load().oracle_disk_orbit(1 if mn else 0, M, a, Q, eps, float(r), float(theta),
                                   _ptr(out))
    return tuple(out) if ok else None
