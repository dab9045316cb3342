"""Python binding of libgrtrace (MI355X geodesic ray tracer).

Argument marshalling only: every step of the tracing runs in the HIP kernels
of ``libgrtrace.so``; PyTorch supplies device memory and streams.  The
functions carry the names of the C entry points declared in
``include/grtrace.h``; see that header for the meaning of every field.

Importing this package loads the built library and raises ImportError if it
is missing (build it with ``python paper_2310_15183_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrtrace.so")

GR_OK, GR_EINVAL, GR_ENOMEM, GR_EDEVICE, GR_EUNSUPPORTED = 0, -1, -2, -3, -4
GR_FLAG_TIMEOUT, GR_FLAG_ESCAPE, GR_FLAG_HORIZON, GR_FLAG_INVALID, GR_FLAG_DISK = 0, 1, 2, 3, 4
GR_FP64, GR_MIXED = 0, 1
GR_RK4, GR_EULER, GR_RK4_TIME = 0, 1, 2
GR_SHADE_BANDS, GR_SHADE_TIME, GR_SHADE_TEXTURE = 0, 1, 2
GR_F64, GR_F32 = 0, 1
GR_NOALLOC_MAX_INSTANCES = 512


class gr_metric(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("a", ctypes.c_double), ("Q", ctypes.c_double)]


class gr_metric_mn(ctypes.Structure):
    _fields_ = [("M", ctypes.c_double), ("S", ctypes.c_double), ("q", ctypes.c_double)]


class gr_shade(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("t_max", ctypes.c_double), ("band", ctypes.c_double),
                ("texture", ctypes.c_void_p), ("tex_width", ctypes.c_int32),
                ("tex_height", ctypes.c_int32)]


class gr_camera(ctypes.Structure):
    _fields_ = [("r0", ctypes.c_double), ("theta0", ctypes.c_double),
                ("phi0", ctypes.c_double), ("fov", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class gr_integrator(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("fd_eps", ctypes.c_double),
                ("horizon_norm", ctypes.c_double), ("escape_factor", ctypes.c_double),
                ("max_steps", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("method", ctypes.c_int32), ("disk_r_in", ctypes.c_double),
                ("disk_r_out", ctypes.c_double), ("disk_half_angle", ctypes.c_double)]


class gr_output(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("r", ctypes.c_void_p), ("theta", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("p_t", ctypes.c_void_p), ("p_r", ctypes.c_void_p),
                ("p_theta", ctypes.c_void_p), ("p_phi", ctypes.c_void_p),
                ("flag", ctypes.c_void_p), ("steps", ctypes.c_void_p),
                ("dtype", ctypes.c_int32)]


class gr_instance(ctypes.Structure):
    _fields_ = [("metric", gr_metric), ("camera", gr_camera), ("out", gr_output),
                ("pixels", ctypes.c_void_p), ("n_pixels", ctypes.c_int64)]


class gr_fallback(ctypes.Structure):
    _fields_ = [("logit_min", ctypes.c_float), ("edge_px", ctypes.c_int32),
                ("max_gain", ctypes.c_float), ("min_impact", ctypes.c_float)]


class gr_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("order", ctypes.c_int32)]


def _load():
    # Load torch's HIP runtime first: libgrtrace.so then binds to the same
    # libamdhip64.so.7 (one runtime per process, so torch's device pointers and
    # streams are valid in the library).  Loading the library first would pull
    # in a second runtime that does not share torch's device state.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_2310_15183_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "gr_trace_init": (ctypes.c_int, [P(vp), ctypes.c_int, P(gr_integrator)]),
        "gr_trace_frame": (ctypes.c_int, [vp, P(gr_metric), P(gr_camera), P(gr_output), vp]),
        "gr_trace_frame_mn": (ctypes.c_int, [vp, P(gr_metric_mn), P(gr_camera), P(gr_output),
                                             vp]),
        "gr_trace_batch": (ctypes.c_int, [vp, P(gr_instance), ctypes.c_int32, vp]),
        "gr_trace_batch_noalloc": (ctypes.c_int, [vp, P(gr_instance), ctypes.c_int32, vp]),
        "gr_shade_frame": (ctypes.c_int, [P(gr_shade), P(gr_output), ctypes.c_int64, vp, vp]),
        "gr_redshift": (ctypes.c_int, [vp, P(gr_metric), P(gr_camera), P(gr_output),
                                       ctypes.c_int64, vp, vp]),
        "gr_redshift_mn": (ctypes.c_int, [vp, P(gr_metric_mn), P(gr_camera), P(gr_output),
                                          ctypes.c_int64, vp, vp]),
        "gr_trace_set_integrator": (ctypes.c_int, [vp, P(gr_integrator)]),
        "gr_trace_set_launch": (ctypes.c_int, [vp, P(gr_launch)]),
        "gr_trace_get_launch": (ctypes.c_int, [vp, P(gr_launch)]),
        "gr_trace_autotune": (ctypes.c_int, [vp, P(gr_instance), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_char_p, P(gr_launch), vp]),
        "gr_trace_destroy": (ctypes.c_int, [vp]),
        "gr_trace_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "gr_trace_last_device_error": (ctypes.c_char_p, []),
        "gr_horizon_radius": (ctypes.c_double, [P(gr_metric)]),
        "gr_check_division": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int64, vp]),
        "gr_trace_validate": (ctypes.c_int, [P(gr_metric), P(gr_camera), P(gr_integrator),
                                             P(gr_output)]),
        "gr_mlp_num_params": (ctypes.c_int64, []),
        "gr_mlp_create": (ctypes.c_int, [P(vp), ctypes.c_int, ctypes.c_int64]),
        "gr_mlp_destroy": (ctypes.c_int, [vp]),
        "gr_mlp_init": (ctypes.c_int, [vp, ctypes.c_uint64]),
        "gr_mlp_set_params": (ctypes.c_int, [vp, vp]),
        "gr_mlp_get_params": (ctypes.c_int, [vp, vp]),
        "gr_mlp_forward": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp, vp]),
        "gr_mlp_loss_grad": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, vp,
                                            vp, vp]),
        "gr_mlp_adam_step": (ctypes.c_int, [vp, vp, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, vp]),
        "gr_mlp_steps": (ctypes.c_int64, [vp]),
        "gr_surrogate_inputs": (ctypes.c_int, [vp, P(gr_instance), ctypes.c_int32, vp, vp, vp]),
        "gr_surrogate_targets": (ctypes.c_int, [vp, P(gr_instance), ctypes.c_int32, vp, vp, vp]),
        "gr_surrogate_frame": (ctypes.c_int, [vp, vp, P(gr_metric), P(gr_camera),
                                              P(gr_fallback), vp, vp, vp, P(ctypes.c_int64),
                                              vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ["gr_trace_init", "gr_trace_frame", "gr_trace_frame_mn", "gr_trace_batch",
            "gr_trace_batch_noalloc", "gr_check_division",
            "gr_shade_frame", "gr_redshift", "gr_redshift_mn",
            "gr_trace_set_integrator",
            "gr_trace_set_launch", "gr_trace_get_launch", "gr_trace_autotune", "gr_trace_destroy",
            "gr_trace_strerror", "gr_trace_last_device_error", "gr_horizon_radius",
            "gr_trace_validate", "gr_mlp_num_params", "gr_mlp_create", "gr_mlp_destroy",
            "gr_mlp_init", "gr_mlp_set_params", "gr_mlp_get_params", "gr_mlp_forward",
            "gr_mlp_loss_grad", "gr_mlp_adam_step", "gr_mlp_steps", "gr_surrogate_inputs",
            "gr_surrogate_targets", "gr_surrogate_frame"]


class GrError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.gr_trace_strerror(code).decode()
        if code == GR_EDEVICE:
            msg += ": " + _lib.gr_trace_last_device_error().decode()
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


def _check(code: int, where: str) -> None:
    if code != GR_OK:
        raise GrError(code, where)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C entry points
def gr_trace_init(device: int = 0, integrator: gr_integrator | None = None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    integ = integrator if integrator is not None else make_integrator()
    _check(_lib.gr_trace_init(ctypes.byref(ctx), int(device), ctypes.byref(integ)),
           "gr_trace_init")
    return ctx


def gr_trace_frame(ctx, metric: gr_metric, camera: gr_camera, out: gr_output, stream=None):
    _check(_lib.gr_trace_frame(ctx, ctypes.byref(metric), ctypes.byref(camera),
                               ctypes.byref(out), _stream_handle(stream)), "gr_trace_frame")


def gr_trace_frame_mn(ctx, metric: gr_metric_mn, camera: gr_camera, out: gr_output,
                      stream=None):
    _check(_lib.gr_trace_frame_mn(ctx, ctypes.byref(metric), ctypes.byref(camera),
                                  ctypes.byref(out), _stream_handle(stream)),
           "gr_trace_frame_mn")


def shade_texture(texture) -> gr_shade:
    """GR_SHADE_TEXTURE settings for a (height, width) device tensor of
    32-bit texels (bytes R, G, B, A); the tensor must outlive the call."""
    assert texture.dim() == 2 and texture.element_size() == 4 and texture.is_contiguous()
    return gr_shade(GR_SHADE_TEXTURE, 0.0, 0.0, texture.data_ptr(), texture.shape[1],
                    texture.shape[0])


def gr_shade_frame(shade: gr_shade, out: gr_output, n: int, rgba, stream=None):
    """Colour n traced rays into rgba (a device tensor of n int32/uint32)."""
    _check(_lib.gr_shade_frame(ctypes.byref(shade), ctypes.byref(out), int(n),
                               ctypes.c_void_p(rgba.data_ptr()), _stream_handle(stream)),
           "gr_shade_frame")


def gr_redshift(ctx, metric, camera: gr_camera, out: gr_output, n: int, z, stream=None):
    """Ring redshift of n traced rays into z (a device tensor of out's dtype);
    metric is a gr_metric or a gr_metric_mn."""
    fn = _lib.gr_redshift_mn if isinstance(metric, gr_metric_mn) else _lib.gr_redshift
    _check(fn(ctx, ctypes.byref(metric), ctypes.byref(camera), ctypes.byref(out), int(n),
              ctypes.c_void_p(z.data_ptr()), _stream_handle(stream)), "gr_redshift")


def gr_trace_batch(ctx, instances, stream=None):
    arr = (gr_instance * len(instances))(*instances)
    _check(_lib.gr_trace_batch(ctx, arr, len(instances), _stream_handle(stream)),
           "gr_trace_batch")


def gr_trace_batch_noalloc(ctx, instances, stream=None):
    arr = (gr_instance * len(instances))(*instances)
    _check(_lib.gr_trace_batch_noalloc(ctx, arr, len(instances), _stream_handle(stream)),
           "gr_trace_batch_noalloc")


def gr_trace_set_integrator(ctx, integrator: gr_integrator):
    _check(_lib.gr_trace_set_integrator(ctx, ctypes.byref(integrator)),
           "gr_trace_set_integrator")


def gr_trace_set_launch(ctx, launch: gr_launch | None):
    _check(_lib.gr_trace_set_launch(ctx, ctypes.byref(launch) if launch is not None else None),
           "gr_trace_set_launch")


def gr_trace_get_launch(ctx) -> gr_launch:
    out = gr_launch()
    _check(_lib.gr_trace_get_launch(ctx, ctypes.byref(out)), "gr_trace_get_launch")
    return out


def gr_trace_autotune(ctx, instances, trial_steps=0, cache_path=None, stream=None) -> gr_launch:
    arr = (gr_instance * len(instances))(*instances)
    best = gr_launch()
    path = cache_path.encode() if cache_path else None
    _check(_lib.gr_trace_autotune(ctx, arr, len(instances), int(trial_steps), path,
                                  ctypes.byref(best), _stream_handle(stream)),
           "gr_trace_autotune")
    return best


def gr_trace_destroy(ctx):
    _check(_lib.gr_trace_destroy(ctx), "gr_trace_destroy")


def gr_trace_strerror(code: int) -> str:
    return _lib.gr_trace_strerror(int(code)).decode()


def gr_check_division(a, x, stream=None):
    """(a / x, 1 / x) of two float64 device tensors of equal length, formed
    as the binary64 step forms its divisions."""
    import torch
    assert a.dtype == x.dtype == torch.float64 and a.numel() == x.numel()
    a, x = a.contiguous(), x.contiguous()
    q, r = torch.empty_like(a), torch.empty_like(x)
    _check(_lib.gr_check_division(_p(a), _p(x), _p(q), _p(r), a.numel(),
                                  _stream_handle(stream)), "gr_check_division")
    return q, r


def gr_trace_last_device_error() -> str:
    return _lib.gr_trace_last_device_error().decode()


def gr_trace_validate(metric: gr_metric, camera: gr_camera, integrator: gr_integrator | None,
                      out: gr_output) -> int:
    """Host-side argument validation only (no device needed); returns the code."""
    return _lib.gr_trace_validate(ctypes.byref(metric), ctypes.byref(camera),
                                  ctypes.byref(integrator) if integrator is not None else None,
                                  ctypes.byref(out))


def gr_horizon_radius(metric: gr_metric) -> float:
    return _lib.gr_horizon_radius(ctypes.byref(metric))


# ---------------------------------------------------------------- marshalling helpers
def make_integrator(dt=0.01, fd_eps=1e-8, horizon_norm=1e4, escape_factor=1.5,
                    max_steps=20000, precision=GR_FP64, method=None,
                    disk=None) -> gr_integrator:
    """disk = (r_in, r_out, half_angle) adds the solid equatorial ring."""
    d = (0.0, 0.0, 0.0) if disk is None else tuple(float(v) for v in disk)
    return gr_integrator(dt, fd_eps, horizon_norm, escape_factor, int(max_steps),
                         int(precision), GR_RK4 if method is None else int(method), *d)


FIELDS = ("t", "r", "theta", "phi", "p_t", "p_r", "p_theta", "p_phi")


@dataclass
class Outputs:
    """Torch device tensors backing a gr_output (kept alive with it)."""
    tensors: dict = field(default_factory=dict)
    struct: gr_output = None

    def __getitem__(self, k):
        return self.tensors[k]


def alloc_outputs(n: int, dtype=GR_F64, fields=("t", "r", "theta", "phi"), steps=True,
                  device="cuda") -> Outputs:
    """Allocate per-ray output tensors on the device and the gr_output that
    points at them.  flag is int8 (pre-filled with -1), steps int32 (-1)."""
    import torch
    fdt = torch.float64 if dtype == GR_F64 else torch.float32
    ten = {f: torch.empty(n, dtype=fdt, device=device) for f in fields}
    ten["flag"] = torch.full((n,), -1, dtype=torch.int8, device=device)
    if steps:
        ten["steps"] = torch.full((n,), -1, dtype=torch.int32, device=device)
    ptr = lambda k: ten[k].data_ptr() if k in ten else None  # noqa: E731
    st = gr_output(*(ptr(f) for f in FIELDS), ptr("flag"), ptr("steps"), int(dtype))
    return Outputs(ten, st)


# ---------------------------------------------------------------- surrogate network
def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def gr_mlp_num_params() -> int:
    return int(_lib.gr_mlp_num_params())


def gr_mlp_create(device: int = 0, max_batch: int = 65536):
    m = ctypes.c_void_p()
    _check(_lib.gr_mlp_create(ctypes.byref(m), int(device), int(max_batch)), "gr_mlp_create")
    return m


def gr_mlp_destroy(m):
    _check(_lib.gr_mlp_destroy(m), "gr_mlp_destroy")


def gr_mlp_init(m, seed: int):
    _check(_lib.gr_mlp_init(m, int(seed)), "gr_mlp_init")


def gr_mlp_set_params(m, host_params):
    import numpy as np
    arr = np.ascontiguousarray(host_params, dtype=np.float32)
    assert arr.size == gr_mlp_num_params()
    _check(_lib.gr_mlp_set_params(m, arr.ctypes.data_as(ctypes.c_void_p)), "gr_mlp_set_params")


def gr_mlp_get_params(m):
    import numpy as np
    arr = np.empty(gr_mlp_num_params(), np.float32)
    _check(_lib.gr_mlp_get_params(m, arr.ctypes.data_as(ctypes.c_void_p)), "gr_mlp_get_params")
    return arr


def gr_mlp_forward(m, x, y, stream=None):
    """x: (n, 7) float32 cuda tensor, y: (n, 4) float32 cuda tensor."""
    _check(_lib.gr_mlp_forward(m, _p(x), x.shape[0], _p(y), _stream_handle(stream)),
           "gr_mlp_forward")


def gr_mlp_loss_grad(m, x, target, grad, loss=None, rows=None, n=None, lam=100.0, delta=1e30,
                     stream=None, dmax=1e30):
    n = int(rows.shape[0] if rows is not None else x.shape[0]) if n is None else int(n)
    _check(_lib.gr_mlp_loss_grad(m, _p(x), _p(target), _p(rows), n, int(x.shape[0]),
                                 float(lam), float(delta), float(dmax), _p(loss), _p(grad),
                                 _stream_handle(stream)), "gr_mlp_loss_grad")


def gr_mlp_adam_step(m, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.gr_mlp_adam_step(m, _p(grad), float(lr), float(beta1), float(beta2),
                                 float(eps), _stream_handle(stream)), "gr_mlp_adam_step")


def gr_mlp_steps(m) -> int:
    return int(_lib.gr_mlp_steps(m))


def gr_surrogate_inputs(ctx, instances, x, u_flat, stream=None):
    arr = (gr_instance * len(instances))(*instances)
    _check(_lib.gr_surrogate_inputs(ctx, arr, len(instances), _p(x), _p(u_flat),
                                    _stream_handle(stream)), "gr_surrogate_inputs")


def gr_surrogate_targets(ctx, instances, u_flat, target, stream=None):
    arr = (gr_instance * len(instances))(*instances)
    _check(_lib.gr_surrogate_targets(ctx, arr, len(instances), _p(u_flat), _p(target),
                                     _stream_handle(stream)), "gr_surrogate_targets")


def gr_surrogate_frame(ctx, mlp, metric, camera, logit_min, edge_px, flag, direction, fallback,
                       stream=None, count=True, max_gain=0.0, min_impact=0.0) -> int:
    """Returns the number of fallback pixels; with count=False the call does not
    wait for the GPU and returns -1.  The rule's fields are the keywords of the
    same names (gr_fallback)."""
    nfb = ctypes.c_int64(-1)
    rule = gr_fallback(float(logit_min), int(edge_px), float(max_gain), float(min_impact))
    _check(_lib.gr_surrogate_frame(ctx, mlp, ctypes.byref(metric), ctypes.byref(camera),
                                   ctypes.byref(rule), _p(flag), _p(direction),
                                   _p(fallback), ctypes.byref(nfb) if count else None,
                                   _stream_handle(stream)),
           "gr_surrogate_frame")
    return int(nfb.value)
