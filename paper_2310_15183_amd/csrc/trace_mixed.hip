// Mixed-precision tracer for gfx950: binary32 RK4 stages and contraction;
// binary64 metric evaluations and forward differences (a difference of step
// 1e-8 needs binary64: the binary32 spacing near r = 20 is 1.9e-6); whole
// binary64 steps near the horizon and near radial turning points.
//
// Same method as the binary64 tracer (arXiv 2310.15183, Sec. 2.1 eq.
// hamGeodesic, Sec. 3.1.2 RK4 in coordinate-time steps, forward differences
// of the appendix listing, exits of Sec. 3.3.2, camera of Sec. 3.3.1).
// Evaluation choices, none of which changes the method:
//  - a stage runs on the binary32-rounded state: its point, right-hand side,
//    contraction and the RK4 combination are binary32; the step's increment
//    is added to the state in binary64 (one add per component), because
//    binary32 rounding of theta and phi alone random-walks ~5e-6 rad over
//    1e4 steps;
//  - sin and cos of the step's binary32 angle are evaluated in binary32; the
//    later stages rotate that pair by their binary32 increment (short series,
//    below the binary32 rounding for |increment| <= 1/4; a larger increment
//    evaluates sin and cos of the stage angle afresh); the pair is widened,
//    and sin at theta+eps follows by the angle-addition identity in binary64
//    (cos eps rounds to 1, sin eps to eps), so both evaluations of the theta
//    difference see one consistent angle and the step is exactly eps;
//  - the metric's reciprocals follow the binary64 tracer's scheme with
//    v_rcp_f64 refined by two Newton steps (about 1 ulp) in place of its two
//    divisions per stage;
//    the binary32 step divides by |dt/dtau| with v_rcp_f32;
//  - -1/(2 eps) is folded into the binary32 contraction weights;
//  - dt/dtau and dphi/dtau are linear in the ray's constant p_t, p_phi, so
//    the step sums g^tt, g^tphi, g^phph over the stages in binary64 and
//    contracts them once.
// A ray switches to whole binary64 steps (the binary64 tracer's own step)
// when r < 1.2 r_+ or |p_r| < 1e-3, and back when r > 1.25 r_+ and
// |p_r| > 2e-3.

#include "internal.h"
#include "step_fp64.h"

namespace gr {
namespace {

using namespace detail;

constexpr double R64_ENTER = 1.2, R64_LEAVE = 1.25;   // in units of r_+
constexpr double PR_ENTER = 1e-3, PR_LEAVE = 2e-3;

__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

struct DerivF {
    float qt, qr, qh, pr, ph;
    double gtt, gtp, gpp;       // g^tt, g^tphi, g^phph at the stage point
};

struct ConstF {
    float pt, pph;              // binary32 copies of the ray constants
    float wtt, wtp, wpp;        // -p_t^2/(2 eps), -p_t p_phi/eps, -p_phi^2/(2 eps)
    float ie;                   // -1/(2 eps)
};

// sin and cos in binary32: x = k pi/2 + r, |r| <= pi/4 (two-part pi/2), then
// Taylor polynomials through r^9 and r^10 (truncation below 2e-9).
__device__ __forceinline__ void sincos_f32(float x, float& s_out, float& c_out) {
    const float k = rintf(x * 0.636619772f);
    float r = fmaf(-k, 1.57079637f, x);
    r = fmaf(-k, -4.37113883e-8f, r);
    const float z = r * r;
    float ps = 2.75573192e-6f;                   //  1/9!
    ps = fmaf(ps, z, -1.98412698e-4f);           // -1/7!
    ps = fmaf(ps, z, 8.33333333e-3f);            //  1/5!
    ps = fmaf(ps, z, -1.66666667e-1f);           // -1/3!
    float pc = -2.75573192e-7f;                  // -1/10!
    pc = fmaf(pc, z, 2.48015873e-5f);            //  1/8!
    pc = fmaf(pc, z, -1.38888889e-3f);           // -1/6!
    pc = fmaf(pc, z, 4.16666667e-2f);            //  1/4!
    pc = fmaf(pc, z, -0.5f);                     // -1/2!
    const float sr = fmaf(r * z, ps, r);
    const float cr = fmaf(z, pc, 1.0f);
    const int q = (int)k & 3;
    const float s = (q & 1) ? cr : sr;
    const float c = (q & 1) ? sr : cr;
    s_out = (q & 2) ? -s : s;
    c_out = (q == 1 || q == 2) ? -c : c;
}

// Largest stage increment of theta that the binary32 rotation takes.
constexpr float ROT_F32_MAX = 0.25f;

// (sf, cf) rotated by d: sin d = d - d^3/6 + d^5/120 and cos d - 1 =
// -d^2/2 + d^4/24, omitted terms below 2^-25 for |d| <= 1/4.
__device__ __forceinline__ void rotate_f32(float sf, float cf, float d, float& s_out,
                                           float& c_out) {
    const float z = d * d;
    const float sd = fmaf(d * z, fmaf(z, 1.0f / 120.0f, -1.0f / 6.0f), d);
    const float cm1 = z * fmaf(z, 1.0f / 24.0f, -0.5f);
    s_out = fmaf(cf, sd, fmaf(sf, cm1, sf));
    c_out = fmaf(-sf, sd, fmaf(cf, cm1, cf));
}

// sin and cos at the stage angle th + d from those at th.
__device__ __forceinline__ void stage_sc(float th, float s1, float c1, float d, float& sf,
                                         float& cf) {
    if (fabsf(d) <= ROT_F32_MAX) rotate_f32(s1, c1, d, sf, cf);
    else sincos_f32(fmaf(1.0f, d, th), sf, cf);
}

__device__ __forceinline__ DerivF rhs_mixed(const Hole& H, double eps, float r, float sf,
                                            float cf, float pr, float pth, const ConstF& K) {
    const double s = (double)sf, c = (double)cf;
    const ThetaTerms T0 = theta_terms_s(H, s);
    const ThetaTerms T1 = theta_terms_s(H, fma(eps, c, s));
    const RadialTerms R0 = radial_terms(H, (double)r);
    const RadialTerms R1 = radial_terms(H, (double)r + eps);
    // the binary64 tracer's reciprocal scheme, with v_rcp_f64 and two Newton
    // steps in place of its two divisions
    const double is = rcp_nr(rho2_delta(H, R0, T0) * T0.s2);
    const double inv = is * T0.s2;
    const double is_r = recip_newton(rho2_delta(H, R1, T0) * T0.s2, is);
    const double is_t = rcp_nr(rho2_delta(H, R0, T1) * T1.s2);
    const InvMetric g = metric_from(H, R0, T0, inv, is);
    const InvMetric dr = metric_diff(H, R1, T0, is_r * T0.s2, is_r, g);
    const InvMetric dh = metric_diff(H, R0, T1, is_t * T1.s2, is_t, g);

    const float wrr = (pr * pr) * K.ie, wth = (pth * pth) * K.ie;
    float acc = (float)dr.tt * K.wtt;
    acc = fmaf((float)dr.tp, K.wtp, acc);
    acc = fmaf((float)dr.rr, wrr, acc);
    acc = fmaf((float)dr.hh, wth, acc);
    acc = fmaf((float)dr.pp, K.wpp, acc);
    DerivF d;
    d.pr = acc;
    acc = (float)dh.tt * K.wtt;
    acc = fmaf((float)dh.tp, K.wtp, acc);
    acc = fmaf((float)dh.rr, wrr, acc);
    acc = fmaf((float)dh.hh, wth, acc);
    acc = fmaf((float)dh.pp, K.wpp, acc);
    d.ph = acc;

    d.qt = fmaf((float)g.tt, K.pt, (float)g.tp * K.pph);
    d.qr = (float)g.rr * pr;
    d.qh = (float)g.hh * pth;
    d.gtt = g.tt;
    d.gtp = g.tp;
    d.gpp = g.pp;
    return d;
}

// One RK4 step with binary32 stages; the increment is added in binary64.
__device__ __forceinline__ double rk4_step_mixed(const Hole& H, const Integrator& in,
                                                 const ConstF& K, float dt, Ray& y) {
    const float r = (float)y.r, th = (float)y.th;
    const float pr = (float)y.pr, pth = (float)y.pth;
    const double eps = in.eps;
    float s1, c1, sf, cf;
    sincos_f32(th, s1, c1);
    DerivF k = rhs_mixed(H, eps, r, s1, c1, pr, pth, K);
    const float nu = fabsf(k.qt);
    const float h = dt * __builtin_amdgcn_rcpf(nu);
    const float hh = 0.5f * h;
    double stt = k.gtt, stp = k.gtp, spp = k.gpp;
    float sr = k.qr, sh = k.qh, spr = k.pr, sph = k.ph;
    stage_sc(th, s1, c1, hh * k.qh, sf, cf);
    k = rhs_mixed(H, eps, fmaf(hh, k.qr, r), sf, cf, fmaf(hh, k.pr, pr), fmaf(hh, k.ph, pth), K);
    stt = fma(2.0, k.gtt, stt); stp = fma(2.0, k.gtp, stp); spp = fma(2.0, k.gpp, spp);
    sr = fmaf(2.0f, k.qr, sr); sh = fmaf(2.0f, k.qh, sh);
    spr = fmaf(2.0f, k.pr, spr); sph = fmaf(2.0f, k.ph, sph);
    stage_sc(th, s1, c1, hh * k.qh, sf, cf);
    k = rhs_mixed(H, eps, fmaf(hh, k.qr, r), sf, cf, fmaf(hh, k.pr, pr), fmaf(hh, k.ph, pth), K);
    stt = fma(2.0, k.gtt, stt); stp = fma(2.0, k.gtp, stp); spp = fma(2.0, k.gpp, spp);
    sr = fmaf(2.0f, k.qr, sr); sh = fmaf(2.0f, k.qh, sh);
    spr = fmaf(2.0f, k.pr, spr); sph = fmaf(2.0f, k.ph, sph);
    stage_sc(th, s1, c1, h * k.qh, sf, cf);
    k = rhs_mixed(H, eps, fmaf(h, k.qr, r), sf, cf, fmaf(h, k.pr, pr), fmaf(h, k.ph, pth), K);
    stt += k.gtt; stp += k.gtp; spp += k.gpp;
    sr += k.qr; sh += k.qh; spr += k.pr; sph += k.ph;
    const float h6 = h * (1.0f / 6.0f);
    const double h6d = (double)h6;
    y.t = fma(h6d, fma(stt, y.pt, stp * y.pph), y.t);
    y.r += (double)(h6 * sr);
    y.th += (double)(h6 * sh);
    y.ph = fma(h6d, fma(stp, y.pt, spp * y.pph), y.ph);
    y.pr += (double)(h6 * spr);
    y.pth += (double)(h6 * sph);
    return (double)nu;
}

struct MixedArgs {
    FrameArgs f;
    double r_enter, r_leave;   // binary64 mode boundaries (R64_* times r_+)
};

// Constants of ray y's binary32 right-hand side.
__device__ __forceinline__ void mixed_constants(const FrameArgs& A, const Ray& y, ConstF& K) {
    K.pt = (float)y.pt;
    K.pph = (float)y.pph;
    K.ie = -0.5f * (float)A.in.inv_eps;
    K.wtt = (K.pt * K.pt) * K.ie;
    K.wtp = ((2.0f * K.pt) * K.pph) * K.ie;
    K.wpp = (K.pph * K.pph) * K.ie;
}

// One step of ray y in its current mode; in64 switches with hysteresis.
__device__ __forceinline__ double mixed_step(const MixedArgs& X, const ConstF& K, float dtf,
                                             bool& in64, Ray& y) {
    const FrameArgs& A = X.f;
    const double apr = fabs(y.pr);
    if (!in64 && (y.r < X.r_enter || apr < PR_ENTER)) in64 = true;
    else if (in64 && y.r > X.r_leave && apr > PR_LEAVE) in64 = false;
    return in64 ? rk4_step_direct(A.hole, A.in, y) : rk4_step_mixed(A.hole, A.in, K, dtf, y);
}

// One lane, one ray (static_ray: 8x8 pixel tiles per wave); the grid covers
// every ray.
template <typename T>
__global__ void __launch_bounds__(256) trace_mixed_static(const MixedArgs X) {
    const FrameArgs& A = X.f;
    int64_t k, pix;
    if (!static_ray(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, k, pix)) return;
    const float dtf = (float)A.in.dt;
    Ray y;
    ConstF K;
    start_ray(A.cam, pix, y);
    mixed_constants(A, y, K);
    bool in64 = false;
    int s = 0;
    int f = start_flag(A.in, y);
    while (f == RUNNING) {
        const double nu = mixed_step(X, K, dtf, in64, y);
        ++s;
        f = exit_flag(A.in, A.r_esc, y, nu, s);
    }
    write_ray<T>(A.out, k, y, f, s);
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
trace_mixed_refill(const MixedArgs X,
                                                           unsigned long long* counter) {
    const FrameArgs& A = X.f;
    const float dtf = (float)A.in.dt;
    Ray y;
    ConstF K;
    int64_t k = 0;
    int s = 0;
    bool live = false, want = true, in64 = false;
    for (;;) {
        const int64_t id = take_ids(want, counter);
        if (want) {
            want = false;
            if (id < A.nray) {
                k = A.order ? (int64_t)A.order[id] : id;
                start_ray(A.cam, A.pixels ? (int64_t)A.pixels[k] : k, y);
                s = 0;
                in64 = false;
                mixed_constants(A, y, K);
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
            const double nu = mixed_step(X, K, dtf, in64, y);
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

}  // namespace

hipError_t launch_trace_mixed(const FrameArgs& A, double r_plus, bool f32_out,
                              const LaunchShape& L, unsigned long long* counter,
                              hipStream_t s) {
    MixedArgs X;
    X.f = A;
    X.r_enter = R64_ENTER * r_plus;
    X.r_leave = R64_LEAVE * r_plus;
    if (!L.refill) {
        if (f32_out)
            hipLaunchKernelGGL(trace_mixed_static<float>, dim3(L.grid), dim3(L.block), 0, s, X);
        else
            hipLaunchKernelGGL(trace_mixed_static<double>, dim3(L.grid), dim3(L.block), 0, s, X);
        return hipGetLastError();
    }
    hipError_t e = launch_reset_counter(counter, s);
    if (e != hipSuccess) return e;
    if (f32_out)
        hipLaunchKernelGGL(trace_mixed_refill<float>, dim3(L.grid), dim3(L.block), 0, s, X,
                           counter);
    else
        hipLaunchKernelGGL(trace_mixed_refill<double>, dim3(L.grid), dim3(L.block), 0, s, X,
                           counter);
    return hipGetLastError();
}

int occupancy_trace_mixed(int block, bool f32_out) {
    int n = 0;
    hipError_t e = f32_out ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                 &n, trace_mixed_refill<float>, block, 0)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                 &n, trace_mixed_refill<double>, block, 0);
    return e == hipSuccess ? n : 0;
}

}  // namespace gr
