// FP64 geodesic tracer for gfx950: one lane per ray, state in registers.
//
// Each lane integrates Hamilton's equations for H = 1/2 g^{mu nu} p_mu p_nu
// (arXiv 2310.15183, Sec. 2.1 eq. hamGeodesic with the 1/2 of Appendix A)
// with RK4 (Sec. 3.1.2) in coordinate-time steps h = dt/|dt/dtau| fixed from
// the first stage (appendix listing), forward-difference metric derivatives
// (listing; Sec. 3.3.3), and the escape / horizon / step-limit exits of
// Sec. 3.3.2.  The camera ray of each pixel is built in-lane (Sec. 3.3.1).
//
// Lane management: in the persistent form every wave keeps its lanes busy by
// taking new rays from a global counter as old ones finish; the lanes that
// finished in a step are counted with one ballot, the wave's first such lane
// takes that many consecutive ray ids with one atomic, and each finished lane
// picks its id by its rank in the ballot mask.  Results are independent of
// which lane traces which ray.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "internal.h"

namespace gr {
namespace {

enum { RUNNING = -1 };

struct Deriv {
    double qt, qr, qh, qp;   // dq^mu/dtau
    double pr, ph;           // dp_r/dtau, dp_theta/dtau
};

// Right-hand side at one stage point: metric at (r, th), (r+eps, th),
// (r, th+eps); difference quotients times 1/eps; p-dot = -1/2 sum of the five
// independent terms in the order tt, tphi (weight 2 p_t p_phi), rr, thth, phph.
__device__ __forceinline__ Deriv rhs(const Hole& H, double eps, double inv_eps, double r,
                                     double th, double pt, double pr, double pth, double pph,
                                     double wtt, double wtp, double wpp) {
    const ThetaTerms T0 = theta_terms(H, th);
    const ThetaTerms T1 = theta_terms(H, th + eps);
    const RadialTerms R0 = radial_terms(H, r);
    const RadialTerms R1 = radial_terms(H, r + eps);
    const InvMetric g = inverse_metric(H, R0, T0);
    const InvMetric gr = inverse_metric(H, R1, T0);
    const InvMetric gh = inverse_metric(H, R0, T1);

    const double wrr = pr * pr, wth = pth * pth;
    double acc = ((gr.tt - g.tt) * inv_eps) * wtt;
    acc = fma((gr.tp - g.tp) * inv_eps, wtp, acc);
    acc = fma((gr.rr - g.rr) * inv_eps, wrr, acc);
    acc = fma((gr.hh - g.hh) * inv_eps, wth, acc);
    acc = fma((gr.pp - g.pp) * inv_eps, wpp, acc);
    Deriv d;
    d.pr = -0.5 * acc;
    acc = ((gh.tt - g.tt) * inv_eps) * wtt;
    acc = fma((gh.tp - g.tp) * inv_eps, wtp, acc);
    acc = fma((gh.rr - g.rr) * inv_eps, wrr, acc);
    acc = fma((gh.hh - g.hh) * inv_eps, wth, acc);
    acc = fma((gh.pp - g.pp) * inv_eps, wpp, acc);
    d.ph = -0.5 * acc;

    d.qt = fma(g.tt, pt, g.tp * pph);
    d.qr = g.rr * pr;
    d.qh = g.hh * pth;
    d.qp = fma(g.tp, pt, g.pp * pph);
    return d;
}

struct Ray {
    double t, r, th, ph, pt, pr, pth, pph;
    double wtt, wtp, wpp;    // p_t^2, 2 p_t p_phi, p_phi^2 (constant along the ray)
};

__device__ __forceinline__ void start_ray(const Camera& C, int64_t pix, Ray& y) {
    const int64_t i = pix % C.W, j = pix / C.W;
    camera_ray(C, i, j, y.pt, y.pr, y.pth, y.pph);
    y.t = 0.0;
    y.r = C.r0;
    y.th = C.th0;
    y.ph = C.ph0;
    y.wtt = y.pt * y.pt;
    y.wtp = (2.0 * y.pt) * y.pph;
    y.wpp = y.pph * y.pph;
}

__device__ __forceinline__ bool finite6(const Ray& y) {
    return isfinite(y.t) && isfinite(y.r) && isfinite(y.th) && isfinite(y.ph) &&
           isfinite(y.pr) && isfinite(y.pth);
}

// One RK4 step; returns nu = |dt/dtau| of the first stage.
__device__ __forceinline__ double rk4_step(const Hole& H, const Integrator& in, Ray& y) {
    const double eps = in.eps, inv_eps = in.inv_eps;
    Deriv k = rhs(H, eps, inv_eps, y.r, y.th, y.pt, y.pr, y.pth, y.pph, y.wtt, y.wtp, y.wpp);
    const double nu = fabs(k.qt);
    const double h = in.dt / nu;
    const double hh = 0.5 * h;
    double st = k.qt, sr = k.qr, sh = k.qh, sp = k.qp, spr = k.pr, sph = k.ph;
    k = rhs(H, eps, inv_eps, fma(hh, k.qr, y.r), fma(hh, k.qh, y.th), y.pt,
            fma(hh, k.pr, y.pr), fma(hh, k.ph, y.pth), y.pph, y.wtt, y.wtp, y.wpp);
    st = st + 2.0 * k.qt; sr = sr + 2.0 * k.qr; sh = sh + 2.0 * k.qh; sp = sp + 2.0 * k.qp;
    spr = spr + 2.0 * k.pr; sph = sph + 2.0 * k.ph;
    k = rhs(H, eps, inv_eps, fma(hh, k.qr, y.r), fma(hh, k.qh, y.th), y.pt,
            fma(hh, k.pr, y.pr), fma(hh, k.ph, y.pth), y.pph, y.wtt, y.wtp, y.wpp);
    st = st + 2.0 * k.qt; sr = sr + 2.0 * k.qr; sh = sh + 2.0 * k.qh; sp = sp + 2.0 * k.qp;
    spr = spr + 2.0 * k.pr; sph = sph + 2.0 * k.ph;
    k = rhs(H, eps, inv_eps, fma(h, k.qr, y.r), fma(h, k.qh, y.th), y.pt,
            fma(h, k.pr, y.pr), fma(h, k.ph, y.pth), y.pph, y.wtt, y.wtp, y.wpp);
    st = st + k.qt; sr = sr + k.qr; sh = sh + k.qh; sp = sp + k.qp;
    spr = spr + k.pr; sph = sph + k.ph;
    const double h6 = h * (1.0 / 6.0);
    y.t = fma(h6, st, y.t);
    y.r = fma(h6, sr, y.r);
    y.th = fma(h6, sh, y.th);
    y.ph = fma(h6, sp, y.ph);
    y.pr = fma(h6, spr, y.pr);
    y.pth = fma(h6, sph, y.pth);
    return nu;
}

__device__ __forceinline__ int exit_flag(const Integrator& in, double r_esc, const Ray& y,
                                         double nu, int s) {
    if (y.r > r_esc) return GR_FLAG_ESCAPE;
    if (nu > in.hnorm) return GR_FLAG_HORIZON;
    if (!finite6(y)) return GR_FLAG_INVALID;
    if (s >= in.max_steps) return GR_FLAG_TIMEOUT;
    return RUNNING;
}

template <typename T>
__device__ __forceinline__ void put(void* p, int64_t k, double v) {
    if (p) reinterpret_cast<T*>(p)[k] = (T)v;
}

template <typename T>
__device__ __forceinline__ void write_ray(const OutPtrs& o, int64_t k, const Ray& y, int flag,
                                          int s) {
    put<T>(o.t, k, y.t);
    put<T>(o.r, k, y.r);
    put<T>(o.th, k, y.th);
    put<T>(o.ph, k, y.ph);
    put<T>(o.pt, k, y.pt);
    put<T>(o.pr, k, y.pr);
    put<T>(o.pth, k, y.pth);
    put<T>(o.pph, k, y.pph);
    o.flag[k] = (int8_t)flag;
    if (o.steps) o.steps[k] = s;
}

// Flag for a freshly started ray: invalid start or a zero step limit end it.
__device__ __forceinline__ int start_flag(const Integrator& in, const Ray& y) {
    if (!(finite6(y) && isfinite(y.pt) && isfinite(y.pph))) return GR_FLAG_INVALID;
    if (in.max_steps <= 0) return GR_FLAG_TIMEOUT;
    return RUNNING;
}

// Wave-wide work distribution: lanes with `want` set receive consecutive ids
// from the global counter (one atomic per wave), in lane order.
__device__ __forceinline__ int64_t take_ids(bool want, unsigned long long* counter) {
    const int lane = (int)__lane_id();
    const unsigned long long want_mask = __ballot(want);
    if (!want_mask) return -1;
    const int leader = __ffsll((unsigned long long)want_mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(want_mask));
    base = __shfl(base, leader);
    const unsigned long long below = want_mask & ((1ull << lane) - 1ull);
    return want ? (int64_t)(base + (unsigned long long)__popcll(below)) : -1;
}

// One lane, one ray; the grid covers every ray.
template <typename T>
__global__ void __launch_bounds__(256) trace_fp64_static(const FrameArgs A) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nray) return;
    Ray y;
    start_ray(A.cam, A.pixels ? (int64_t)A.pixels[k] : k, y);
    int s = 0;
    int f = start_flag(A.in, y);
    while (f == RUNNING) {
        const double nu = rk4_step(A.hole, A.in, y);
        ++s;
        f = exit_flag(A.in, A.r_esc, y, nu, s);
    }
    write_ray<T>(A.out, k, y, f, s);
}

// Persistent lanes with ballot refill from the global counter.
template <typename T>
__global__ void __launch_bounds__(256) trace_fp64_refill(const FrameArgs A,
                                                          unsigned long long* counter) {
    Ray y;
    int64_t k = 0;
    int s = 0;
    bool live = false;   // lane holds a ray in flight
    bool want = true;    // lane asks for a new ray
    for (;;) {
        const int64_t id = take_ids(want, counter);
        if (want) {
            want = false;
            if (id < A.nray) {
                k = id;
                start_ray(A.cam, A.pixels ? (int64_t)A.pixels[k] : k, y);
                s = 0;
                const int f = start_flag(A.in, y);
                if (f == RUNNING) {
                    live = true;
                } else {
                    write_ray<T>(A.out, k, y, f, 0);
                    want = true;
                }
            }
        }
        if (!__any(live || want)) break;
        if (live) {
            const double nu = rk4_step(A.hole, A.in, y);
            ++s;
            const int f = exit_flag(A.in, A.r_esc, y, nu, s);
            if (f != RUNNING) {
                write_ray<T>(A.out, k, y, f, s);
                live = false;
                want = true;
            }
        }
    }
}

// Many instances in one launch.  Global ray ids run over the instances in
// table order; a lane finds its instance by binary search of the prefix
// offsets and keeps that instance's black-hole constants in registers.
__device__ __forceinline__ int find_instance(const BatchArgs& B, int64_t id) {
    int lo = 0, hi = B.ninst;                     // firsts[lo] <= id < firsts[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (B.firsts[mid] <= id) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void write_batch(const BatchInstance& I, int64_t k, const Ray& y,
                                            int f, int s) {
    if (I.f32) write_ray<float>(I.out, k, y, f, s);
    else write_ray<double>(I.out, k, y, f, s);
}

__global__ void __launch_bounds__(256) trace_fp64_batch(const BatchArgs B,
                                                         unsigned long long* counter) {
    Ray y;
    Hole H;
    double r_esc = 0.0;
    int inst = 0;
    int64_t k = 0;
    int s = 0;
    bool live = false;
    bool want = true;
    for (;;) {
        const int64_t id = take_ids(want, counter);
        if (want) {
            want = false;
            if (id < B.total) {
                inst = find_instance(B, id);
                const BatchInstance& I = B.inst[inst];
                k = id - B.firsts[inst];
                H = I.hole;
                r_esc = I.r_esc;
                start_ray(I.cam, I.pixels ? (int64_t)I.pixels[k] : k, y);
                s = 0;
                const int f = start_flag(B.in, y);
                if (f == RUNNING) {
                    live = true;
                } else {
                    write_batch(I, k, y, f, 0);
                    want = true;
                }
            }
        }
        if (!__any(live || want)) break;
        if (live) {
            const double nu = rk4_step(H, B.in, y);
            ++s;
            const int f = exit_flag(B.in, r_esc, y, nu, s);
            if (f != RUNNING) {
                write_batch(B.inst[inst], k, y, f, s);
                live = false;
                want = true;
            }
        }
    }
}

__global__ void reset_counter_kernel(unsigned long long* c) { *c = 0ull; }

}  // namespace

hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_trace_fp64(const FrameArgs& A, bool f32_out, const LaunchShape& L,
                             unsigned long long* counter, hipStream_t s) {
    if (L.refill) {
        hipError_t e = launch_reset_counter(counter, s);
        if (e != hipSuccess) return e;
        if (f32_out)
            hipLaunchKernelGGL(trace_fp64_refill<float>, dim3(L.grid), dim3(L.block), 0, s, A,
                               counter);
        else
            hipLaunchKernelGGL(trace_fp64_refill<double>, dim3(L.grid), dim3(L.block), 0, s, A,
                               counter);
    } else {
        if (f32_out)
            hipLaunchKernelGGL(trace_fp64_static<float>, dim3(L.grid), dim3(L.block), 0, s, A);
        else
            hipLaunchKernelGGL(trace_fp64_static<double>, dim3(L.grid), dim3(L.block), 0, s, A);
    }
    return hipGetLastError();
}

hipError_t launch_trace_fp64_batch(const BatchArgs& B, const LaunchShape& L,
                                   unsigned long long* counter, hipStream_t s) {
    hipError_t e = launch_reset_counter(counter, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(trace_fp64_batch, dim3(L.grid), dim3(L.block), 0, s, B, counter);
    return hipGetLastError();
}

int occupancy_trace_fp64_batch(int block) {
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, trace_fp64_batch, block, 0) ==
                   hipSuccess
               ? n
               : 0;
}

int occupancy_trace_fp64(int block, bool f32_out) {
    int n = 0;
    hipError_t e = f32_out ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                 &n, trace_fp64_refill<float>, block, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                 &n, trace_fp64_refill<double>, block, 0);
    return e == hipSuccess ? n : 0;
}

}  // namespace gr
