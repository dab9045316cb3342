// Internal interface between the C-ABI host code and the kernel translation
// units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grmath.h"
#include "grtrace.h"

namespace gr {

// Per-ray outputs; any float pointer may be null.
struct OutPtrs {
    void* t;
    void* r;
    void* th;
    void* ph;
    void* pt;
    void* pr;
    void* pth;
    void* pph;
    int8_t* flag;
    int32_t* steps;
};

struct Integrator {
    double dt, eps, inv_eps, hnorm, esc_factor;
    double sin_eps, cos_eps;   // sincos_def(eps): angle addition for theta + eps
    double scale;              // -0.5 * (1/eps): p-dot = scale * sum of differences
    double disk_r_in, disk_r_out, disk_dth;   // the ring (used by kernels built with it)
    int32_t max_steps;
};

// Everything one frame launch needs, passed by value as the kernel argument
// (uniform values live in scalar registers).
struct FrameArgs {
    Hole hole;
    Camera cam;
    Integrator in;
    double r_esc;           // esc_factor * r0
    int64_t nray;           // rays to trace
    const int32_t* pixels;  // null: ray k is pixel k
    const int32_t* order;   // null: the queue hands out ray k as its k-th id; else
                            // id -> ray k = order[id] (a permutation of 0..nray-1);
                            // persistent tracers only
    OutPtrs out;
};

// Per-instance constants of the surrogate's features and baseline (host-made).
struct SurConst {
    float feat[5];          // a/M, |Q|/M, theta0, r0/(50 M), fov (M = 1 for flat space)
    double st, ct, sp, cp;  // sin/cos of theta0 and phi0
    double r0, R, u0, u1;   // camera radius, escape radius, 1/r0, 1/R
    double M, Q2;
    double bscale;          // b = bscale sin(alpha): r0 / sqrt(f(r0)) of the charged hole
    double inv_bc;          // 1 / critical impact parameter (0 for flat space)
    double uph;             // 1 / photon-sphere radius (0 for flat space)
};

// One instance of a batch (device table entry).
struct BatchInstance {
    Hole hole;
    Camera cam;
    double r_esc;
    const int32_t* pixels;  // null: ray k is pixel k
    OutPtrs out;
    int32_t f32;
    SurConst sur;
};

struct BatchArgs {
    Integrator in;
    const BatchInstance* inst;  // device table, ninst entries
    const int64_t* firsts;      // device prefix offsets, ninst + 1 entries (firsts[0] = 0)
    const int64_t* wfirsts;     // one ray per lane: prefix offsets of the instances' waves
                                // (8x8 tiles of a frame, 64 entries of a pixel list)
    int32_t ninst;
    int64_t total;              // rays on the host's side (launch shape; an upper bound when
                                // firsts[ninst] is produced on the device); the kernel reads
                                // the number of rays from firsts[ninst]
};

struct LaunchShape {
    int block;           // threads per workgroup
    int grid;            // workgroups
    int refill;          // persistent lanes pull rays from the queue
};

// Queue order of a frame: the permutation of its pixels sorted by
// |b - b_c|, the distance of each camera ray's impact parameter
// b = sqrt(Carter Q + L_z^2)/E from b_c, so that the near-critical rays, the
// longest, are traced first.  keys/vals: 2 x npix each; temp: frame_order_temp
// bytes.  The sorted permutation is left in vals + npix.
hipError_t frame_order(const Hole& H, const Camera& C, double b_crit, int64_t npix, float* keys,
                       int32_t* vals, void* temp, size_t temp_bytes, hipStream_t s);
size_t frame_order_temp(int64_t npix);

// Fill the queue counter with zero (a kernel, so that it can sit in a
// captured graph).
hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t s);

// FP64 frame tracer.  f32_out selects binary32 outputs.
hipError_t launch_trace_fp64(const FrameArgs& A, bool f32_out, int method, bool disk,
                             const LaunchShape& L, unsigned long long* counter, hipStream_t s);

// Workgroups of `block` threads that fit on one CU for the FP64 tracer.
int occupancy_trace_fp64(int block, bool f32_out);

// Mixed-precision frame tracer (binary32 state and stages, binary64
// differences, binary64 steps inside 1.2 r_+ or near radial turning points).
hipError_t launch_trace_mixed(const FrameArgs& A, double r_plus, bool f32_out,
                              const LaunchShape& L, unsigned long long* counter,
                              hipStream_t s);
int occupancy_trace_mixed(int block, bool f32_out);

// Colours of n traced rays (mode 0 the sky's lines, 1 exit time, 2 the sky
// texture, tex_w x tex_h device words) from the output arrays o (binary32
// when f32).
hipError_t launch_shade(int mode, const OutPtrs& o, bool f32, int64_t n, double t_max,
                        double band, const uint32_t* texture, int tex_w, int tex_h,
                        uint32_t* rgba, hipStream_t s);

// Rays a one-ray-per-lane launch parks after `cap` steps (0: none) for a
// second launch to continue: structure-of-arrays state of up to `capacity`
// rays (y: t, r, theta, phi, p_r, p_theta, each `capacity` long), their step
// counts and pixels, and the number parked (zeroed by the launcher).  Rays
// beyond the capacity are finished by the first launch.
struct Parked {
    double* y;
    int32_t* steps;
    int64_t* pix;
    unsigned long long* count;
    int64_t capacity;
    int32_t cap;
};

// A Manko-Novikov frame, one ray per lane over 8x8 pixel tiles (L.refill
// must be 0), then (park.cap > 0) the parked rays in a persistent launch of
// shape L2; A.hole is not used.
hipError_t launch_trace_mn(const FrameArgs& A, const MnHole& K, bool f32_out, int method,
                           bool disk, const LaunchShape& L, const Parked& park,
                           const LaunchShape& L2, hipStream_t s);
int occupancy_trace_mn_resume(int block);

// Ring redshift of n rays (flag GR_FLAG_DISK; NaN otherwise) from the output
// arrays o, with the camera observer's frequency nu_o = sqrt(-1/g^tt(camera)).
// mn selects the Manko-Novikov metric K, else the Kerr-Newman hole H.
hipError_t launch_redshift(const Hole& H, const MnHole& K, bool mn, const Integrator& in,
                           double nu_o, const OutPtrs& o, bool f32, int64_t n, void* z,
                           hipStream_t s);

// All instances of a batch in one launch: persistent (L.refill), or one ray
// per lane over the waves of B.wfirsts.
hipError_t launch_trace_fp64_batch(const BatchArgs& B, const LaunchShape& L,
                                   unsigned long long* counter, hipStream_t s);
int occupancy_trace_fp64_batch(int block);

}  // namespace gr
