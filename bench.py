"""Benchmark: geodesic rays/s on a 1000x1000 Kerr-Newman frame (one GPU).

One step = one complete trace of the frame: camera rays built in-kernel,
metric and forward differences, Hamilton right-hand side, RK4 with the
coordinate-time normaliser, termination and the per-ray stores.
Inputs are synthetic (an analytic camera grid); nothing is cached between
steps.  Prints one JSON line.

Workload (the paper-scale configuration): M=0.5, a=0.24, Q=0.3 (Boyer-
Lindquist), camera r0=20, theta0=80 deg, phi0=0, fov 75 deg, 1000x1000;
dt=0.005, fd_eps=1e-8, at most 50000 steps, horizon at |dt/dtau| > 1e4,
escape at r > 30.  Parameters are rounded to binary32 first (the camera and
black-hole inputs of this configuration are binary32); state is binary64;
end coordinates are stored as binary32 with an int8 flag.

The roofline object reports the tracing kernel against the MI355X FP64
vector peak: achieved = algorithmic work per launch (613 operations per
ray-step times the ray-steps of the launch, read from the kernel's own step
counts) divided by the launch's duration measured with HIP events on the
launch stream.  The 613 are the method's own operations, whatever the kernel
executes: 584 arithmetic flops (an fma counts 2) plus 21 divisions and 8
sin/cos pairs, each of those counted once.  The fraction that hardware
counters measure for executed binary64 flops (the kernel's own series sin/cos
and reciprocal refinements included) is reported beside it, read from the
committed counter summary when that was taken on the current kernel source.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "geodesic rays/s @1000² Kerr: FP64 vs mixed vs surrogate, ≤1e-4 rad err"
# Algorithmic operations of one binary64 step of the method: fma = 2 flops,
# add/sub/mul 1, and each division, square root, exp and sin/cos pair 1.
# RK4 on Kerr-Newman: 4 stages of (3 metric evaluations of 23 flops + 1
# division, 2 sin/cos, 2 reciprocals of sin^2, differences 20, contraction 26,
# dq/dtau 8) + stage arguments 24 + update 42 + the normaliser's division
# = 584 flops + 21 divisions + 8 sin/cos.
FLOPS_PER_RAY_STEP = 613
OP_COUNTING = ("fma = 2 flops, add/sub/mul 1; each division, square root, exp and sin/cos "
               "pair counts 1 (the method's operations, not the kernel's instructions)")
FP64_PEAK_TFLOPS = 78.6           # MI355X FP64 vector (256 CU x 128 flop/clk x 2.4 GHz)
BF16_PEAK_TFLOPS = 2500.0         # MI355X dense bfloat16 MFMA
STRICT_TURN = 0.05                # surrogate_strict: also re-trace where neighbours' directions
                                  # differ by more than 0.05 rad
MIN_IMPACT = 1.2                  # surrogate_strict: also re-trace escaping rays with b < 1.2 b_c
KERNEL_SOURCES = ["paper_2310_15183_amd/csrc/trace_fp64.hip",
                  "paper_2310_15183_amd/csrc/step_fp64.h",
                  "paper_2310_15183_amd/csrc/grmath.h",
                  "paper_2310_15183_amd/csrc/internal.h"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "trace_fp64_kn1000_traffic.md")


def f32(x):
    import numpy as np
    return float(np.float32(x))


def workload():
    deg = math.pi / 180.0
    return dict(M=f32(0.5), a=f32(0.24), Q=f32(0.3), r0=f32(20.0), theta0=f32(80 * deg),
                phi0=0.0, fov=f32(75 * deg), W=1000, H=1000, dt=0.005, fd_eps=1e-8,
                horizon_norm=1e4, escape_factor=1.5, max_steps=50000)


def kernel_hash() -> str:
    """Hash of the tracing kernel's sources and of the hipcc options it is
    built with (the options change the code too), the same wherever the
    repository is checked out."""
    import importlib.util
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    spec = importlib.util.spec_from_file_location(
        "_grtrace_build_opts", os.path.join(ROOT, "paper_2310_15183_amd", "build.py"))
    opts = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(opts)
    # include directories name this checkout's location, not an option of the code
    flags = [f for f in opts.FLAGS + opts.EXTRA.get("trace_fp64.hip", []) if not f.startswith("-I")]
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def recorded_traffic(units_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"HBM bytes per launch:\s*([0-9.eE+]+)", text)
    if not (m_hash and m_bytes) or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


COUNTER_PROFILE = os.path.join(ROOT, "profiles", "trace_fp64_kn1000_counters.md")


def recorded_executed():
    """Executed binary64 flops of the tracing kernel as the committed counter
    summary measured them (64 x SQ_INSTS_VALU_FLOPS_FP64 over the kernel
    time), if it was taken on the current kernel source (else None)."""
    if not os.path.exists(COUNTER_PROFILE):
        return None
    text = open(COUNTER_PROFILE).read()
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", text)
    m_frac = re.search(r"executed FP64 fraction of peak:\s*([0-9.]+)", text)
    m_step = re.search(r"executed flop per ray-step:\s*([0-9.]+)", text)
    if not (m_hash and m_frac and m_step) or m_hash.group(1) != kernel_hash():
        return None
    return {"frac": float(m_frac.group(1)), "flop_per_ray_step": float(m_step.group(1)),
            "source": os.path.relpath(COUNTER_PROFILE, ROOT)}


def host_cpu_model():
    """The host CPU's model name (Linux), else the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, stride, threads):
    """Time the CPU oracle on every stride-th pixel in both axes of the same
    frame; returns rays/s and the sample's mean steps."""
    import numpy as np

    import oracle
    ii = np.arange(stride // 2, w["W"], stride)
    jj = np.arange(stride // 2, w["H"], stride)
    pix = (jj[:, None] * w["W"] + ii[None, :]).ravel()
    t0 = time.perf_counter()
    res = oracle.trace_frame(w["M"], w["a"], w["Q"], w["r0"], w["theta0"], w["phi0"], w["fov"],
                             w["W"], w["H"], dt=w["dt"], eps=w["fd_eps"],
                             horizon_norm=w["horizon_norm"], escape_factor=w["escape_factor"],
                             max_steps=w["max_steps"], pixels=pix, threads=threads)
    dt = time.perf_counter() - t0
    return pix.size / dt, pix.size, float(res.steps.mean()), dt


def time_frames(g, ctx, metric, cam, out, steps, warmup, stream):
    """Run warmup untimed frames, then time `steps` frames; returns (wall
    seconds for the timed frames, mean launch seconds from HIP events)."""
    import torch
    for _ in range(warmup):
        g.gr_trace_frame(ctx, metric, cam, out.struct, stream)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        g.gr_trace_frame(ctx, metric, cam, out.struct, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, sum(s.elapsed_time(e) for s, e in zip(starts, ends)) / 1e3 / steps


def frames_in_flight(g, w, n_rays, ray_steps, nstreams=3, nframes=6):
    """Binary64 frames on several streams at once (one context each): the
    tail of one frame overlaps the next.  Frame throughput, not the
    single-frame figure."""
    import torch
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    ctxs = [g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                                 horizon_norm=w["horizon_norm"],
                                                 escape_factor=w["escape_factor"],
                                                 max_steps=w["max_steps"]))
            for _ in range(nstreams)]
    outs = [g.alloc_outputs(n_rays, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
            for _ in range(nstreams)]
    metric = g.gr_metric(w["M"], w["a"], w["Q"])
    cam = g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"])
    for j in range(nstreams):
        g.gr_trace_frame(ctxs[j], metric, cam, outs[j].struct, streams[j])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nframes):
        j = k % nstreams
        g.gr_trace_frame(ctxs[j], metric, cam, outs[j].struct, streams[j])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / nframes
    for c in ctxs:
        g.gr_trace_destroy(c)
    return {"streams": nstreams, "frames": nframes, "ms_per_frame": sec * 1e3,
            "rays_per_s": n_rays / sec,
            "frac": FLOPS_PER_RAY_STEP * ray_steps / sec / 1e12 / FP64_PEAK_TFLOPS}


def traced_frame(g, w, stream, precision):
    """Trace the frame once with every output in binary64 (host arrays)."""
    import torch
    ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                               horizon_norm=w["horizon_norm"],
                                               escape_factor=w["escape_factor"],
                                               max_steps=w["max_steps"], precision=precision))
    out = g.alloc_outputs(w["W"] * w["H"], dtype=g.GR_F64, fields=g.FIELDS)
    g.gr_trace_frame(ctx, g.gr_metric(w["M"], w["a"], w["Q"]),
                     g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"]),
                     out.struct, stream)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.tensors.items()}
    g.gr_trace_destroy(ctx)
    return res


def accuracy_pair(g, w, stream, ref):
    """Mixed-precision frame against the binary64 one: where the rays cross
    the escape sphere, and the flags."""
    from paper_2310_15183_amd.evaluate import mixed_errors
    got = traced_frame(g, w, stream, g.GR_MIXED)
    return mixed_errors(w["M"], w["a"], w["Q"], w["escape_factor"] * w["r0"], ref, got)


def mixed_variant(g, w, args, stream, fp64_rays_per_s, ref):
    """Mixed-precision form on the same frame: rays/s, speedup and accuracy
    against the binary64 frame ref."""
    n = w["W"] * w["H"]
    ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                               horizon_norm=w["horizon_norm"],
                                               escape_factor=w["escape_factor"],
                                               max_steps=w["max_steps"], precision=g.GR_MIXED))
    out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
    metric = g.gr_metric(w["M"], w["a"], w["Q"])
    cam = g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"])
    wall, launch_s = time_frames(g, ctx, metric, cam, out, args.steps, args.warmup, stream)
    g.gr_trace_destroy(ctx)
    err = accuracy_pair(g, w, stream, ref)
    rays_s = n * args.steps / wall
    return {"rays_per_s": rays_s, "ms_per_step": wall / args.steps * 1e3,
            "launch_ms": launch_s * 1e3, "speedup_vs_fp64": rays_s / fp64_rays_per_s,
            "angle_err_rad": {k: err[k] for k in ("median", "p99", "p999", "max")},
            "flag_mismatch_frac": err["flag_mismatch"],
            "gate": "p99.9 <= 1e-4 rad, <= 0.1% misclassified",
            "passes_gate": err["p999"] <= 1e-4 and err["flag_mismatch"] <= 1e-3}


def bench_mixed(args):
    """Near-extremal Kerr (M=0.5, a=0.49, r0=20, theta0=60 deg, fov 75 deg,
    dt=0.005, 50000 steps) at 1000x1000 and 2048x2048: binary64 vs mixed."""
    import torch

    import paper_2310_15183_amd as g
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    lines = []
    for side in (1000, 2048):
        w = dict(workload(), M=0.5, a=0.49, Q=0.0, r0=20.0, theta0=math.radians(60.0),
                 fov=math.radians(75.0), W=side, H=side)
        n = side * side
        ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                                   horizon_norm=w["horizon_norm"],
                                                   escape_factor=w["escape_factor"],
                                                   max_steps=w["max_steps"]))
        out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
        wall, launch_s = time_frames(g, ctx, g.gr_metric(w["M"], w["a"], w["Q"]),
                                     g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"],
                                                 side, side), out, args.steps, args.warmup,
                                     stream)
        g.gr_trace_destroy(ctx)
        fp64 = n * args.steps / wall
        mixed = mixed_variant(g, w, args, stream, fp64, traced_frame(g, w, stream, g.GR_FP64))
        lines.append({"workload": f"near-extremal kerr {side}x{side}", "fp64_rays_per_s": fp64,
                      "fp64_ms_per_step": wall / args.steps * 1e3, "mixed": mixed})
    print(json.dumps({"metric": "geodesic rays/s, near-extremal Kerr: FP64 vs mixed",
                      "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic", "results": lines}), flush=True)


def train_surrogate(g, args):
    """Label args.train_rays rays with the binary64 tracer over the batch
    parameter ranges, train the network on them with the library's kernels,
    and score it on 2e5 held-out rays."""
    import torch

    from paper_2310_15183_amd import surrogate as S
    data = S.training_set(args.train_rays, seed=11)
    net = g.gr_mlp_create(0, 8192)
    g.gr_mlp_init(net, 11)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = S.train(net, data, epochs=args.train_epochs, seed=11)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    held = S.training_set(200_000, seed=12)
    info = {"label_rays": int(data.x.shape[0]), "label_s": data.seconds,
            "label_ray_steps": data.ray_steps, "epochs": args.train_epochs, "batch": 8192,
            "train_s": train_s, "final_loss": hist[-1] if hist else None,
            "held_out": S.evaluate_network(net, held)}
    del data, held
    return net, info


def surrogate_variant(g, net, w, args, stream, fp64_rays_per_s, ref, logit_min=3.0, edge=2,
                      max_gain=None, min_impact=0.0):
    """Surrogate + RK4 fallback on the frame w: rays/s, speedup over the
    binary64 tracer on the same frame and integrator, the network-only frame
    time against the MFMA peak, and the errors against the binary64 frame."""
    import torch

    from paper_2310_15183_amd import surrogate as S
    n = w["W"] * w["H"]
    ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                               horizon_norm=w["horizon_norm"],
                                               escape_factor=w["escape_factor"],
                                               max_steps=w["max_steps"]))
    metric = g.gr_metric(w["M"], w["a"], w["Q"])
    cam = g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"])
    flag = torch.empty(n, dtype=torch.int8, device="cuda")
    direc = torch.empty(n, 3, device="cuda")
    fb = torch.empty(n, dtype=torch.int8, device="cuda")

    if max_gain is None:
        max_gain = args.max_gain

    def run(lmin, e, turn, imp, steps, warmup):
        nfb = 0
        for _ in range(warmup):
            nfb = g.gr_surrogate_frame(ctx, net, metric, cam, lmin, e, flag, direc, fb, stream,
                                       max_gain=turn, min_impact=imp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            nfb = g.gr_surrogate_frame(ctx, net, metric, cam, lmin, e, flag, direc, fb, stream,
                                       max_gain=turn, min_impact=imp)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, nfb

    net_s, _ = run(0.0, 0, 0.0, 0.0, args.steps, args.warmup)   # network only, no fallback
    net_flag, net_dir = flag.cpu().numpy(), direc.cpu().numpy()
    wall, nfb = run(logit_min, edge, max_gain, min_impact, args.steps, args.warmup)
    g.gr_trace_destroy(ctx)
    got_flag, got_dir, got_fb = flag.cpu().numpy(), direc.cpu().numpy(), fb.cpu().numpy()
    err = S.frame_errors(w["M"], w["a"], w["Q"], w["escape_factor"] * w["r0"], ref, got_flag,
                         got_dir)
    # the network's own error on the pixels the fallback re-traced (known at run time)
    online = S.online_errors(net_flag, net_dir, got_flag, got_dir, got_fb)

    # many frames in flight: one context and stream each, nothing waits for the
    # GPU between frames, so one frame's latency-bound retrace overlaps the next
    # frame's network
    nstreams, nframes = args.pipeline_streams, max(3, 3 * args.steps)
    if nstreams < 1:
        return _surrogate_result(n, wall, net_s, nfb, fp64_rays_per_s, None, err, online,
                                 logit_min, edge, max_gain, min_impact)
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    ctxs = [g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                                 horizon_norm=w["horizon_norm"],
                                                 escape_factor=w["escape_factor"],
                                                 max_steps=w["max_steps"]))
            for _ in range(nstreams)]
    bufs = [(torch.empty(n, dtype=torch.int8, device="cuda"), torch.empty(n, 3, device="cuda"),
             torch.empty(n, dtype=torch.int8, device="cuda")) for _ in range(nstreams)]
    torch.cuda.synchronize()
    for j in range(nstreams):
        g.gr_surrogate_frame(ctxs[j], net, metric, cam, logit_min, edge, *bufs[j], streams[j],
                             count=False, max_gain=max_gain, min_impact=min_impact)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nframes):
        j = k % nstreams
        g.gr_surrogate_frame(ctxs[j], net, metric, cam, logit_min, edge, *bufs[j], streams[j],
                             count=False, max_gain=max_gain, min_impact=min_impact)
    torch.cuda.synchronize()
    pipe_s = (time.perf_counter() - t0) / nframes
    for c in ctxs:
        g.gr_trace_destroy(c)
    del bufs
    return _surrogate_result(n, wall, net_s, nfb, fp64_rays_per_s, pipe_s, err, online,
                             logit_min, edge, max_gain, min_impact, nstreams, nframes)


def _surrogate_result(n, wall, net_s, nfb, fp64_rays_per_s, pipe_s, err, online, logit_min,
                      edge, max_gain, min_impact, nstreams=0, nframes=0):
    from paper_2310_15183_amd import surrogate as S
    rays_s = n / wall
    tflops = S.FLOPS_PER_RAY * n / net_s / 1e12
    pipelined = None
    if pipe_s:
        pipelined = {"streams": nstreams, "frames": nframes, "ms_per_frame": pipe_s * 1e3,
                     "rays_per_s": n / pipe_s, "speedup_vs_fp64": n / pipe_s / fp64_rays_per_s}
    return {"rays_per_s": rays_s, "ms_per_step": wall * 1e3,
            "speedup_vs_fp64": rays_s / fp64_rays_per_s,
            "pipelined": pipelined,
            "fallback": {"rule": f"|logit| < {logit_min}, a pixel within Chebyshev "
                                 f"distance {edge} of the other predicted class"
                                 + (f", predicted escape with b < {min_impact} b_c"
                                    if min_impact > 0 else "")
                                 + (f", or an escaping 8-neighbour's direction more than "
                                    f"{max_gain:.4g} pixel widths away" if max_gain > 0 else ""),
                         "pixels": int(nfb), "frac": nfb / n, "online": online},
            "network_only_ms": net_s * 1e3,
            "network_mfma": {"achieved": tflops, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": tflops / BF16_PEAK_TFLOPS,
                             "flops_per_ray": S.FLOPS_PER_RAY},
            **err,
            "gate": "p99.9 <= 1e-4 rad, <= 0.1% misclassified",
            "passes_gate": err["angle_err_rad"]["p999"] <= 1e-4
            and err["misclassified_frac"] <= 1e-3}


def bench_surrogate(args):
    """Surrogate + fallback on 4096x4096 frames (the network trained first):
    the Kerr-Newman point of the headline frame, near-extremal Kerr, and four
    seeded draws from the batch parameter ranges; dt=0.01, 20000 steps."""
    import torch

    import paper_2310_15183_amd as g
    from paper_2310_15183_amd.workloads import batch_instances
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    net, info = train_surrogate(g, args)
    print(json.dumps({"training": info}), flush=True)
    side = args.surrogate_side
    base = dict(workload(), dt=0.01, max_steps=20000, W=side, H=side, phi0=0.0)
    frames = [("kerr-newman a=0.24 Q=0.3 theta0=80deg", dict(base)),
              ("near-extremal kerr a=0.49 theta0=60deg",
               dict(base, a=0.49, Q=0.0, theta0=math.radians(60.0)))]
    for k, I in enumerate(batch_instances(4, seed=777)):
        frames.append((f"draw {k}: a={I.a:.3f} Q={I.Q:.3f} r0={I.r0:.1f} "
                       f"theta0={math.degrees(I.theta0):.1f}deg fov={math.degrees(I.fov):.1f}deg",
                       dict(base, M=I.M, a=I.a, Q=I.Q, r0=I.r0, theta0=I.theta0, fov=I.fov)))
    lines = []
    for name, w in frames[:args.surrogate_frames]:
        n = side * side
        ref = traced_frame(g, w, stream, g.GR_FP64)
        ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"], max_steps=w["max_steps"]))
        out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
        fp64_s, _ = time_frames(g, ctx, g.gr_metric(w["M"], w["a"], w["Q"]),
                                g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], side,
                                            side), out, 1, 0, stream)
        g.gr_trace_destroy(ctx)
        del out
        sur = surrogate_variant(g, net, w, args, stream, n / fp64_s, ref)
        strict = surrogate_variant(g, net, w, args, stream, n / fp64_s, ref,
                                   max_gain=STRICT_TURN / (w["fov"] / side),
                                   min_impact=MIN_IMPACT)
        line = {"workload": f"{name} {side}x{side}", "fp64_rays_per_s": n / fp64_s,
                "fp64_ms_per_step": fp64_s * 1e3, "surrogate": sur, "surrogate_strict": strict}
        print(json.dumps(line), flush=True)
        lines.append(line)
        del ref
    g.gr_mlp_destroy(net)
    print(json.dumps({"metric": "geodesic rays/s, surrogate + RK4 fallback vs binary64",
                      "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic", "training": info, "results": lines}), flush=True)


def copy_calibration(mib=256, reps=3):
    """A plain elementwise copy y = 1.0 * x over `mib` MiB of binary32: it
    reads and writes exactly mib MiB per launch, which fixes the scale of the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": reps}))


# One Manko-Novikov RK4 step, same counting: 4 stages of (3 metric
# evaluations of 112 operations with 4 exp, 1 square root and 6 divisions, 2
# sin/cos, 4 squares and displaced points, differences 20, contraction 26,
# dq/dtau 8) + stage arguments 24 + update 42 + the normaliser's division.
FLOPS_PER_RAY_STEP_MN = 1651


def mn_workload():
    """The appendix listing's spacetime and camera radius: Manko-Novikov with
    M=0.5, S=0.24 (a = 0.96 M), q=2, camera r0=8 on the equator, fov 75 deg,
    1000x1000; dt=0.005, at most 50000 steps (binary32 parameters)."""
    import numpy as np
    f = lambda x: float(np.float32(x))          # noqa: E731
    return dict(M=f(0.5), S=f(0.24), q=f(2.0), r0=f(8.0), theta0=f(math.pi / 2), phi0=0.0,
                fov=f(75 * math.pi / 180), W=1000, H=1000, dt=0.005, fd_eps=1e-8,
                horizon_norm=1e4, escape_factor=1.5, max_steps=50000)


def bench_mn(args):
    """Manko-Novikov frame (paper Sec. 2.2.3): binary64 rays/s, roofline,
    and the oracle on a sample of the same frame."""
    import numpy as np
    import torch

    import paper_2310_15183_amd as g
    w = mn_workload()
    torch.cuda.set_device(0)
    n = w["W"] * w["H"]
    ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                               horizon_norm=w["horizon_norm"],
                                               escape_factor=w["escape_factor"],
                                               max_steps=w["max_steps"]))
    metric = g.gr_metric_mn(w["M"], w["S"], w["q"])
    cam = g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"])
    out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        g.gr_trace_frame_mn(ctx, metric, cam, out.struct, stream)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        g.gr_trace_frame_mn(ctx, metric, cam, out.struct, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_s = sum(a.elapsed_time(b) for a, b in zip(starts, ends)) / 1e3 / args.steps
    steps = out["steps"].cpu().numpy().astype(np.int64)
    flags = out["flag"].cpu().numpy()
    ray_steps = int(steps.sum())
    g.gr_trace_destroy(ctx)
    achieved = FLOPS_PER_RAY_STEP_MN * ray_steps / launch_s / 1e12
    # frames in flight on three streams: one frame's tail of trapped rays
    # overlaps the next frame's bulk
    nstreams, nframes = 3, 6
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    ctxs = [g.gr_trace_init(0, g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"],
                                                 horizon_norm=w["horizon_norm"],
                                                 escape_factor=w["escape_factor"],
                                                 max_steps=w["max_steps"]))
            for _ in range(nstreams)]
    outs = [g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
            for _ in range(nstreams)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nframes):
        j = k % nstreams
        g.gr_trace_frame_mn(ctxs[j], metric, cam, outs[j].struct, streams[j])
    torch.cuda.synchronize()
    pipe_s = (time.perf_counter() - t0) / nframes
    for c in ctxs:
        g.gr_trace_destroy(c)
    del outs
    result = {
        "metric": "geodesic rays/s, Manko-Novikov 1000x1000 (binary64)",
        "value": n * args.steps / wall, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "manko-novikov 1000x1000 fp64: M=0.5 S=0.24 q=2 r0=8 "
                               "theta0=90deg fov=75deg dt=0.005 eps=1e-8 max_steps=50000 "
                               "(binary32 params, binary32 end coordinates + int8 flag)",
                   "rays_per_step": n, "ray_steps_per_step": ray_steps,
                   "mean_steps_per_ray": ray_steps / n,
                   "flags": {"timeout": int((flags == 0).sum()),
                             "escape": int((flags == 1).sum()),
                             "horizon": int((flags == 2).sum()),
                             "invalid": int((flags == 3).sum())}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "trace_mn", "flops_per_ray_step": FLOPS_PER_RAY_STEP_MN,
                     "launch_ms": launch_s * 1e3},
        "pipelined": {"streams": nstreams, "frames": nframes, "ms_per_frame": pipe_s * 1e3,
                      "rays_per_s": n / pipe_s,
                      "frac": FLOPS_PER_RAY_STEP_MN * ray_steps / pipe_s / 1e12
                      / FP64_PEAK_TFLOPS},
        "cpu_baseline": None,
    }
    if not args.skip_cpu_baseline:
        import oracle
        stride = 16
        ii = np.arange(stride // 2, w["W"], stride)
        pix = (ii[:, None] * w["W"] + ii[None, :]).ravel()
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        res = oracle.trace_frame_mn(w["M"], w["S"], w["q"], w["r0"], w["theta0"], w["phi0"],
                                    w["fov"], w["W"], w["H"], dt=w["dt"], eps=w["fd_eps"],
                                    horizon_norm=w["horizon_norm"],
                                    escape_factor=w["escape_factor"],
                                    max_steps=w["max_steps"], pixels=pix, threads=threads)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": pix.size / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}th pixel in both axes of the same frame ({pix.size} rays, "
                      f"mean {res.steps.mean():.0f} steps/ray vs {ray_steps / n:.0f} for the "
                      f"full frame), {dt:.1f} s"}
    print(json.dumps(result), flush=True)


FLOPS_PER_RAY_STEP_EULER = 149   # one Kerr-Newman stage (136), the normaliser (1), update (6 fma)


FLOPS_PER_RAY_STEP_RK4_TIME = 641   # RK4's 613 + per stage one division and 6 multiplies
# The same three methods on the Manko-Novikov metric: RK4 1651 (above), the
# coordinate-time RK4 1651 + 28, Euler one stage (396) + the normaliser + 12.
MN_OPS = {"rk4": 1651, "rk4_time": 1679, "euler": 409, "euler_dt/4": 409,
          "reference_rk4_dt/4": 1651}


def bench_euler(args):
    """The integrators of Sec. 3.1 (the comparison of "Resolution and
    Calculation Speed"): RK4 with h fixed from the first stage, RK4 with
    coordinate time as the parameter (each stage reparametrised) and
    explicit Euler at dt and dt/4, on two frames, each against a reference
    frame traced by RK4 at dt/4:
      - the 1000x1000 Kerr-Newman frame (dt = 0.005): rays/s and the
        end-direction error (escape-sphere crossing) of every frame;
      - the 1000x1000 Manko-Novikov frame of the listing's spacetime
        (M = 0.5, S = 0.24, q = 2, r0 = 8; dt = 0.005), whose shadow has a
        chaotic region: the fraction of pixels whose flag or whose sky-line
        colour (the figures' shading) differs from the reference, over the
        frame and over the chaotic region (escaped reference pixels whose end
        direction differs from an 8-neighbour's by more than 0.5 rad, and
        their neighbours)."""
    import numpy as np
    import torch

    import paper_2310_15183_amd as g
    from paper_2310_15183_amd.evaluate import mixed_errors
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    methods = [("rk4", g.GR_RK4, 1, FLOPS_PER_RAY_STEP),
               ("rk4_time", g.GR_RK4_TIME, 1, FLOPS_PER_RAY_STEP_RK4_TIME),
               ("euler", g.GR_EULER, 1, FLOPS_PER_RAY_STEP_EULER),
               ("euler_dt/4", g.GR_EULER, 4, FLOPS_PER_RAY_STEP_EULER),
               ("reference_rk4_dt/4", g.GR_RK4, 4, FLOPS_PER_RAY_STEP)]

    def run(w, mn, method, div, reps):
        n = w["W"] * w["H"]
        ctx = g.gr_trace_init(0, g.make_integrator(dt=w["dt"] / div, fd_eps=w["fd_eps"],
                                                   horizon_norm=w["horizon_norm"],
                                                   escape_factor=w["escape_factor"],
                                                   max_steps=w["max_steps"] * div,
                                                   method=method))
        cam = g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"])
        metric = g.gr_metric_mn(w["M"], w["S"], w["q"]) if mn else g.gr_metric(w["M"], w["a"],
                                                                                w["Q"])
        trace = g.gr_trace_frame_mn if mn else g.gr_trace_frame
        out = g.alloc_outputs(n, dtype=g.GR_F64, fields=g.FIELDS)
        trace(ctx, metric, cam, out.struct, stream)                     # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            trace(ctx, metric, cam, out.struct, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        rgba = torch.empty(n, dtype=torch.int32, device="cuda")
        g.gr_shade_frame(g.gr_shade(g.GR_SHADE_BANDS, 1.0, 0.0), out.struct, n, rgba, stream)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.tensors.items()}
        res["rgba"] = rgba.cpu().numpy()
        g.gr_trace_destroy(ctx)
        return sec, res

    report = {}
    for label, w, mn in [("kerr_newman_1000", workload(), False),
                         ("manko_novikov_1000", mn_workload(), True)]:
        n = w["W"] * w["H"]
        frames = {}
        for name, method, div, ops in methods:
            sec, res = run(w, mn, method, div, 1 if mn or div > 1 else max(args.steps, 1))
            frames[name] = (sec, res, div, ops)
        ref = frames["reference_rk4_dt/4"][1]
        lines = {}
        if mn:
            # the chaotic region: escaped reference pixels whose end direction
            # jumps by more than 0.5 rad to an 8-neighbour, grown by one pixel
            th = ref["theta"].reshape(w["H"], w["W"])
            ph = ref["phi"].reshape(w["H"], w["W"])
            v = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
            esc = (ref["flag"] == g.GR_FLAG_ESCAPE).reshape(w["H"], w["W"])
            jump = np.zeros_like(esc)
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    if dj == 0 and di == 0:
                        continue
                    sv = np.roll(np.roll(v, dj, 0), di, 1)
                    se = np.roll(np.roll(esc, dj, 0), di, 1)
                    jump |= esc & se & (np.linalg.norm(v - sv, axis=-1) > 0.5)
            region = jump.copy()
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    region |= np.roll(np.roll(jump, dj, 0), di, 1)
            region = region.ravel()
        for name, (sec, res, div, ops) in frames.items():
            ops = MN_OPS[name] if mn else ops
            steps = int(res["steps"].astype(np.int64).sum())
            line = {"dt": w["dt"] / div, "ms_per_frame": sec * 1e3, "rays_per_s": n / sec,
                    "ray_steps": steps,
                    "roofline_frac": ops * steps / sec / 1e12 / FP64_PEAK_TFLOPS,
                    "ops_per_ray_step": ops}
            if name != "reference_rk4_dt/4":
                line["flag_changed_frac"] = float((res["flag"] != ref["flag"]).mean())
                line["colour_changed_frac"] = float((res["rgba"] != ref["rgba"]).mean())
                if mn:
                    line["chaotic_region_pixels"] = int(region.sum())
                    line["chaotic_region_colour_changed_frac"] = float(
                        (res["rgba"][region] != ref["rgba"][region]).mean())
                else:
                    line["angle_err_vs_reference_rad"] = mixed_errors(
                        w["M"], w["a"], w["Q"], w["escape_factor"] * w["r0"], ref, res)
            lines[name] = line
        report[label] = lines
    print(json.dumps({"metric": "integrators of Sec. 3.1: rays/s and agreement with RK4 at dt/4",
                      "unit": "rays/s", "n_gpus": 1, "data": "synthetic", "dtype": "f64",
                      "workload": "1000x1000 Kerr-Newman (dt=0.005) and Manko-Novikov "
                                  "(listing spacetime, dt=0.005) frames",
                      "results": report}), flush=True)


HBM_PEAK_GBS = 8000.0            # MI355X HBM3E


def bench_shade(args):
    """Shading kernels (the sky's three lines, the exit-time map, the
    bilinearly filtered sky texture) on a traced 4096x4096 Kerr-Newman frame
    (binary32 end coordinates): time per frame, pixels/s and algorithmic
    bytes against the HBM peak.  The texture is a seeded synthetic 4096x2048
    equirectangular sky (32 MiB); its bytes count once per frame."""
    import numpy as np
    import torch

    import paper_2310_15183_amd as g
    w = workload()
    side = 4096
    n = side * side
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"), steps=False)
    g.gr_trace_frame(ctx, g.gr_metric(w["M"], w["a"], w["Q"]),
                     g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], side, side),
                     out.struct, stream)
    torch.cuda.synchronize()
    g.gr_trace_destroy(ctx)
    rgba = torch.empty(n, dtype=torch.int32, device="cuda")
    from paper_2310_15183_amd.workloads import sky_texture
    tex_w, tex_h = 4096, 2048
    tex = torch.from_numpy(sky_texture(tex_w, tex_h).view(np.int32)).cuda()
    reps = max(args.steps, 10)
    results = {}
    # bytes per pixel: binary32 inputs the mode reads + int8 flag + 32-bit colour
    # (+ the texture once per frame)
    for name, sh, bpp, extra in [
            ("bands", g.gr_shade(g.GR_SHADE_BANDS, 1.0, 0.0), 4 + 4 + 1 + 4, 0),
            ("exit_time", g.gr_shade(g.GR_SHADE_TIME, 80.0, 5.0), 4 + 1 + 4, 0),
            ("texture", g.shade_texture(tex), 4 + 4 + 1 + 4, 4 * tex_w * tex_h)]:
        for _ in range(max(args.warmup, 2)):
            g.gr_shade_frame(sh, out.struct, n, rgba, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            g.gr_shade_frame(sh, out.struct, n, rgba, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        gbs = (bpp * n + extra) / sec / 1e9
        colours = np.unique(rgba.cpu().numpy()).size
        results[name] = {"ms_per_frame": sec * 1e3, "pixels_per_s": n / sec,
                         "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                      "bytes_per_pixel": bpp, "bytes_per_frame_extra": extra},
                         "distinct_colours": int(colours)}
    print(json.dumps({"metric": "shaded pixels/s, 4096^2 traced Kerr-Newman frame",
                      "unit": "pixels/s", "n_gpus": 1, "data": "synthetic", "dtype": "f64",
                      "workload": "kerr-newman 4096x4096 (dt=0.01, 20000 steps), binary32 "
                                  "end coordinates", "results": results}), flush=True)


def bench_disk(args):
    """Kerr (M=0.5, a=0.98 M) with a solid ring (r in [2, 5], |theta - pi/2| <=
    0.02) seen from r0=20, theta0=80 deg, fov 50 deg, 1000x1000, dt=0.005,
    50000 steps: the tracer with and without the ring, and the redshift of
    the ring's light (paper Sec. 3.3.3)."""
    import numpy as np
    import torch

    import paper_2310_15183_amd as g
    n = 1000 * 1000
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    metric = g.gr_metric(0.5, 0.49, 0.0)
    cam = g.gr_camera(20.0, math.radians(80.0), 0.0, math.radians(50.0), 1000, 1000)
    fields = ("t", "r", "theta", "phi", "p_t", "p_phi")
    res = {}
    for name, disk in [("no_ring", None), ("ring", (2.0, 5.0, 0.02))]:
        ctx = g.gr_trace_init(0, g.make_integrator(dt=0.005, max_steps=50000, disk=disk))
        out = g.alloc_outputs(n, dtype=g.GR_F32, fields=fields)
        wall, launch_s = time_frames(g, ctx, metric, cam, out, args.steps, args.warmup, stream)
        steps = int(out["steps"].cpu().numpy().astype(np.int64).sum())
        flags = out["flag"].cpu().numpy()
        achieved = FLOPS_PER_RAY_STEP * steps / launch_s / 1e12
        res[name] = {"ms_per_step": wall / args.steps * 1e3, "rays_per_s": n * args.steps / wall,
                     "ray_steps": steps, "ring_frac": float((flags == 4).mean()),
                     "roofline": {"bound": "alu", "achieved": achieved,
                                  "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": achieved / FP64_PEAK_TFLOPS,
                                  "flops_per_ray_step": FLOPS_PER_RAY_STEP}}
        if disk:
            z = torch.empty(n, dtype=torch.float32, device="cuda")
            for _ in range(2):
                g.gr_redshift(ctx, metric, cam, out.struct, n, z, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record(stream)
            for _ in range(reps):
                g.gr_redshift(ctx, metric, cam, out.struct, n, z, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / 1e3 / reps
            zz = z.cpu().numpy()
            ok = np.isfinite(zz)
            bpr = 4 * 4 + 1 + 4              # r, theta, p_t, p_phi (binary32), flag, z
            gbs = bpr * n / sec / 1e9
            res["redshift"] = {"ms": sec * 1e3, "rays_per_s": n / sec,
                               "z_min": float(zz[ok].min()), "z_max": float(zz[ok].max()),
                               "z_median": float(np.median(zz[ok])),
                               "roofline": {"bound": "hbm", "achieved": gbs,
                                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                            "frac": gbs / HBM_PEAK_GBS, "bytes_per_ray": bpr}}
        g.gr_trace_destroy(ctx)
    print(json.dumps({"metric": "geodesic rays/s with a solid ring, 1000^2 Kerr a=0.98M",
                      "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic", "dtype": "f64", "results": res}), flush=True)


def bench_batch(args):
    """All 256 seeded instances (uneven sizes, spins, charges, cameras) traced
    in one persistent launch per step, with the autotuned launch shape."""
    import numpy as np
    import torch

    import paper_2310_15183_amd as g
    from paper_2310_15183_amd.workloads import batch_instances

    torch.cuda.set_device(0)
    insts = batch_instances(256)
    ctx = g.gr_trace_init(0, g.make_integrator(dt=0.01, max_steps=20000))
    outs, structs = [], []
    for I in insts:
        o = g.alloc_outputs(I.width * I.height, dtype=g.GR_F32,
                            fields=("t", "r", "theta", "phi"))
        outs.append(o)
        structs.append(g.gr_instance(g.gr_metric(I.M, I.a, I.Q),
                                     g.gr_camera(I.r0, I.theta0, I.phi0, I.fov, I.width,
                                                 I.height), o.struct, None, -1))
    stream = torch.cuda.current_stream()
    best = g.gr_trace_autotune(ctx, structs, trial_steps=1000, stream=stream)
    for _ in range(args.warmup):
        g.gr_trace_batch(ctx, structs, stream)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        g.gr_trace_batch(ctx, structs, stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_s = sum(s.elapsed_time(e) for s, e in zip(starts, ends)) / 1e3 / args.steps
    n = sum(I.width * I.height for I in insts)
    ray_steps = int(sum(o["steps"].to(torch.int64).sum().item() for o in outs))
    g.gr_trace_destroy(ctx)
    achieved = FLOPS_PER_RAY_STEP * ray_steps / launch_s / 1e12
    print(json.dumps({
        "metric": "geodesic rays/s, 256-instance uneven batch in one launch",
        "value": n * args.steps / wall, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batch of 256 seeded Kerr-Newman instances (a~U[0,0.49], "
                               "Q~U[0,0.95 sqrt(M^2-a^2)], r0~U[10,50], theta0~U[5,90]deg, "
                               "side in {128,256,384,512}, fov~U[30,90]deg), dt=0.01, "
                               "max_steps=20000",
                   "rays_per_step": n, "ray_steps_per_step": ray_steps,
                   "launch": {"block": best.block, "waves_per_simd": best.waves_per_simd,
                              "order": best.order}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "trace_fp64_batch", "flops_per_ray_step": FLOPS_PER_RAY_STEP,
                     "launch_ms": launch_s * 1e3},
        "cpu_baseline": None,
    }), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-stride", type=int, default=5,
                    help="oracle sample: every n-th pixel in both axes")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (HBM counter scale)")
    ap.add_argument("--workload", choices=["frame", "batch", "mixed", "surrogate", "mn",
                                           "euler", "shade", "disk"],
                    default="frame",
                    help="frame: the 1000x1000 Kerr-Newman frame (default, the headline "
                         "line); batch: the 256-instance uneven batch in one launch; mixed: "
                         "near-extremal Kerr at 1000^2 and 2048^2, binary64 vs mixed; "
                         "surrogate: 4096^2 frames, surrogate + fallback vs binary64; "
                         "mn: the 1000x1000 Manko-Novikov frame; euler: RK4 vs explicit "
                         "Euler on the headline frame; shade: the shading kernels on a "
                         "4096^2 frame; disk: Kerr with a solid ring and its redshift")
    ap.add_argument("--train-rays", type=int, default=10_000_000,
                    help="surrogate: labelled rays to train on")
    ap.add_argument("--train-epochs", type=int, default=12)
    ap.add_argument("--surrogate-side", type=int, default=4096)
    ap.add_argument("--pipeline-streams", type=int, default=3,
                    help="surrogate: frames in flight for the pipelined figure (0: skip it)")
    ap.add_argument("--max-gain", type=float, default=0.0,
                    help="surrogate: also re-trace pixels whose predicted direction differs "
                         "from an escaping neighbour's by more than this many pixel widths "
                         "(0: off)")
    ap.add_argument("--surrogate-frames", type=int, default=6,
                    help="surrogate: how many of its frames to run (in order)")
    ap.add_argument("--skip-variants", action="store_true",
                    help="frame workload: time only the binary64 path")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the tracer has no multi-GPU path "
              "(rays are independent, so a frame would shard by pixel blocks with no "
              "exchange between GPUs).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "mixed":
        bench_mixed(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    if args.workload == "mn":
        bench_mn(args)
        return
    if args.workload == "euler":
        bench_euler(args)
        return
    if args.workload == "shade":
        bench_shade(args)
        return
    if args.workload == "disk":
        bench_disk(args)
        return

    import numpy as np
    import torch

    import paper_2310_15183_amd as g

    w = workload()
    torch.cuda.set_device(0)
    n = w["W"] * w["H"]
    integ = g.make_integrator(dt=w["dt"], fd_eps=w["fd_eps"], horizon_norm=w["horizon_norm"],
                              escape_factor=w["escape_factor"], max_steps=w["max_steps"])
    ctx = g.gr_trace_init(0, integ)
    metric = g.gr_metric(w["M"], w["a"], w["Q"])
    cam = g.gr_camera(w["r0"], w["theta0"], w["phi0"], w["fov"], w["W"], w["H"])
    out = g.alloc_outputs(n, dtype=g.GR_F32, fields=("t", "r", "theta", "phi"))
    stream = torch.cuda.current_stream()

    wall, launch_s = time_frames(g, ctx, metric, cam, out, args.steps, args.warmup, stream)

    steps = out["steps"].cpu().numpy().astype(np.int64)
    flags = out["flag"].cpu().numpy()
    ray_steps = int(steps.sum())
    g.gr_trace_destroy(ctx)

    achieved = FLOPS_PER_RAY_STEP * ray_steps / launch_s / 1e12
    traffic = recorded_traffic(ray_steps)
    result = {
        "metric": METRIC,
        "value": n * args.steps / wall,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "kerr-newman 1000x1000 fp64: M=0.5 a=0.24 Q=0.3 r0=20 theta0=80deg "
                        "fov=75deg dt=0.005 eps=1e-8 max_steps=50000 (binary32 params, "
                        "binary32 end coordinates + int8 flag)",
            "rays_per_step": n,
            "ray_steps_per_step": ray_steps,
            "mean_steps_per_ray": ray_steps / n,
            "flags": {"timeout": int((flags == 0).sum()), "escape": int((flags == 1).sum()),
                      "horizon": int((flags == 2).sum()), "invalid": int((flags == 3).sum())},
            "ray_steps_per_s": ray_steps * args.steps / wall,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "trace_fp64",
            "flops_per_ray_step": FLOPS_PER_RAY_STEP,
            "counting": OP_COUNTING,
            "launch_ms": launch_s * 1e3,
            "executed_by_counters": recorded_executed(),
        },
        "cpu_baseline": None,
        "variants": {},
    }
    if not args.skip_variants:
        ref = traced_frame(g, w, stream, g.GR_FP64)
        result["variants"]["fp64_in_flight"] = frames_in_flight(g, w, n, ray_steps)
        result["variants"]["mixed"] = mixed_variant(g, w, args, stream, result["value"], ref)
        net, info = train_surrogate(g, args)
        sur = surrogate_variant(g, net, w, args, stream, result["value"], ref)
        strict = surrogate_variant(g, net, w, args, stream, result["value"], ref,
                                   max_gain=STRICT_TURN / (w["fov"] / w["W"]),
                                   min_impact=MIN_IMPACT)
        g.gr_mlp_destroy(net)
        sur["training"] = info
        result["variants"]["surrogate"] = sur
        result["variants"]["surrogate_strict"] = strict
        del ref
    if not args.skip_cpu_baseline:
        import oracle
        threads = min(16, oracle.default_threads())
        rays_s, nsample, mean_steps, secs = cpu_baseline(w, args.cpu_stride, threads)
        stride1 = 4 * args.cpu_stride
        rays_s1, nsample1, _, secs1 = cpu_baseline(w, stride1, 1)
        result["cpu_baseline"] = {
            "value": rays_s, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"every {args.cpu_stride}th pixel in both axes of the same frame "
                      f"({nsample} rays, mean {mean_steps:.0f} steps/ray vs "
                      f"{ray_steps / n:.0f} for the full frame), {secs:.1f} s",
            "single_thread": {"value": rays_s1, "unit": "rays/s",
                              "sample": f"every {stride1}th pixel in both axes "
                                        f"({nsample1} rays), {secs1:.1f} s"},
            "host": {"cpu": host_cpu_model(), "nproc": os.cpu_count(),
                     "compiled": "gcc " + " ".join(oracle.CFLAGS)},
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
