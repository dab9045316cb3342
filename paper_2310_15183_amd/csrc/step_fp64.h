// Binary64 RK4 step of the tracer and the per-ray helpers shared by the
// kernels (device code).  Include only from translation units compiled with
// -ffp-contract=off: the operation sequence is the specified one.
#pragma once

#include "internal.h"

namespace gr {
namespace detail {

enum { RUNNING = -1 };

// Correctly rounded 1/x and a/x for the step's operands (finite, normal, with
// a normal quotient): the hardware reciprocal estimate, two Newton-Raphson
// refinements y <- y + y (1 - x y), then Markstein's correction q + (a - x q) y
// with the residual exact in fma.  IEEE division wraps the same steps in
// operand scaling and special-value fixup, which leave such operands
// untouched; a zero, infinite or NaN divisor gives NaN here, on a ray that is
// invalid either way.
static __device__ __forceinline__ double rcp_rn(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(e, y, y);
}

static __device__ __forceinline__ double div_rn(double a, double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    const double q = a * y;
    return fma(fma(-x, q, a), y, q);
}

// Largest |1 - x y0| from which the theta-displaced point's reciprocal is
// refined from the base point's (three Newton steps: e0^8 <= 2^-64, so within
// about an ulp) instead of divided: 2^-8.  rho2 Delta sin^2 moves by the
// factor 1 - 2 eps cot(theta) + O(eps) over the displacement, so only points
// within about 5e5 eps of the polar axis divide.
constexpr double NEWTON_SEED_MAX = 0x1p-8;

struct Deriv {
    double qt, qr, qh, qp;   // dq^mu/dtau
    double pr, ph;           // dp_r/dtau, dp_theta/dtau
    double gtt, gtp, gpp;    // g^tt, g^tphi, g^phph at the point (dt/dtau and dphi/dtau are
                             // linear in them with the ray's constant p_t, p_phi)
};

// Componentwise a - b (each difference rounded once).
static __device__ __forceinline__ InvMetric minus(const InvMetric& a, const InvMetric& b) {
    InvMetric d;
    d.tt = a.tt - b.tt;
    d.tp = a.tp - b.tp;
    d.rr = a.rr - b.rr;
    d.hh = a.hh - b.hh;
    d.pp = a.pp - b.pp;
    return d;
}

// Hamilton's equations from the inverse metric g at the stage point and the
// component differences dr, dh from there to (r + eps, theta) and
// (r, theta + eps): p-dot = -1/(2 eps) times the sum of the five component
// differences times p_nu p_sigma, in the order tt, tphi (weight 2 p_t p_phi),
// rr, thth, phph.  RAW leaves the sums unscaled (the caller folds -1/(2 eps)
// into its step sizes).
template <bool RAW = false>
static __device__ __forceinline__ Deriv deriv_from(const InvMetric& g, const InvMetric& dr,
                                                   const InvMetric& dh, const Integrator& in,
                                                   double pt, double pr, double pth, double pph,
                                                   double wtt, double wtp, double wpp) {
    const double wrr = pr * pr, wth = pth * pth;
    double acc = dr.tt * wtt;
    acc = fma(dr.tp, wtp, acc);
    acc = fma(dr.rr, wrr, acc);
    acc = fma(dr.hh, wth, acc);
    acc = fma(dr.pp, wpp, acc);
    Deriv d;
    d.pr = RAW ? acc : acc * in.scale;
    acc = dh.tt * wtt;
    acc = fma(dh.tp, wtp, acc);
    acc = fma(dh.rr, wrr, acc);
    acc = fma(dh.hh, wth, acc);
    acc = fma(dh.pp, wpp, acc);
    d.ph = RAW ? acc : acc * in.scale;
    d.qt = fma(g.tt, pt, g.tp * pph);
    d.qr = g.rr * pr;
    d.qh = g.hh * pth;
    d.qp = fma(g.tp, pt, g.pp * pph);
    d.gtt = g.tt;
    d.gtp = g.tp;
    d.gpp = g.pp;
    return d;
}

// Right-hand side at one stage point: metric at (r, th), (r+eps, th) and
// (r, th+eps), sin at th+eps by angle addition from sin/cos at th and eps
// (the Kerr-Newman terms need sin^2 only: rho2 comes from it);
// each displaced component is formed together with its difference from the
// base point's (metric_diff: one rounding for the difference);
// p-dot = -1/(2 eps) times the sum of the five component differences times
// p_nu p_sigma, in the order tt, tphi (weight 2 p_t p_phi), rr, thth, phph.
// Reciprocals: is = 1/(rho2 Delta sin^2) divided at (r, th), inv = is
// sin^2; at (r+eps, th), where only rho2 Delta moves, by a factor 1 + O(eps),
// is is refined from the base point's by two Newton steps; at (r, th+eps)
// by three where the refinement starts within NEWTON_SEED_MAX and divided
// where it does not (near the axis sin^2 changes by a large factor over eps),
// inv = is sin^2 there too.
// s, c: sin and cos of the stage point's theta.
// UNIT_COS: cos eps is 1.0 (it rounds to 1 for eps below 1.05e-8, the
// paper's 1e-8 included), so the products with it are exact and are left
// out; chosen per launch, it gives the same bits as the general form.
// SEEDED: the theta-displaced reciprocal is refined whatever its starting
// residual, whose largest magnitude is kept in emax (a step whose emax exceeds
// NEWTON_SEED_MAX is not the canonical one and is redone by the caller).
template <bool UNIT_COS = false, bool RAW = false, bool SEEDED = false>
static __device__ __forceinline__ Deriv rhs_sc(const Hole& H, const Integrator& in, double r,
                                               double s, double c, double pt, double pr,
                                               double pth, double pph, double wtt, double wtp,
                                               double wpp, double* emax = nullptr) {
    const ThetaTerms T0 = theta_terms_s(H, s);
    const ThetaTerms T1 = theta_terms_s(H, fma(c, in.sin_eps, UNIT_COS ? s : s * in.cos_eps));
    const RadialTerms R0 = radial_terms(H, r);
    const RadialTerms R1 = radial_terms(H, r + in.eps);
    const double is = rcp_rn(rho2_delta(H, R0, T0) * T0.s2);
    const double inv = is * T0.s2;
    const double is_r = recip_newton(rho2_delta(H, R1, T0) * T0.s2, is);
    // at (r, th+eps): refined from the base point's where that starts within
    // NEWTON_SEED_MAX, divided elsewhere (near the axis); SEEDED refines
    // always and returns the largest starting residual in emax instead
    const double xt = rho2_delta(H, R0, T1) * T1.s2;
    const double et = fma(-xt, is, 1.0);
    double is_t;
    if constexpr (SEEDED) {
        *emax = fmax(*emax, fabs(et));
        is_t = recip_newton3(xt, is);
    } else {
        is_t = fabs(et) <= NEWTON_SEED_MAX ? recip_newton3(xt, is) : rcp_rn(xt);
    }
    const InvMetric g = metric_from(H, R0, T0, inv, is);
    const InvMetric dr = metric_diff(H, R1, T0, is_r * T0.s2, is_r, g);
    const InvMetric dh = metric_diff(H, R0, T1, is_t * T1.s2, is_t, g);
    return deriv_from<RAW>(g, dr, dh, in, pt, pr, pth, pph, wtt, wtp, wpp);
}

// The right-hand side at (r, th): sin and cos of th by sincos_def.
static __device__ __forceinline__ Deriv rhs(const Hole& H, const Integrator& in, double r,
                                            double th, double pt, double pr, double pth,
                                            double pph, double wtt, double wtp, double wpp) {
    double s, c;
    sincos_def(th, s, c);
    return rhs_sc(H, in, r, s, c, pt, pr, pth, pph, wtt, wtp, wpp);
}

// The same right-hand side for the Manko-Novikov spacetime: three full
// evaluations of its inverse metric (y = cos theta, sin and cos at theta+eps
// by angle addition as above).
static __device__ __forceinline__ Deriv rhs_mn(const MnHole& K, const Integrator& in, double r,
                                               double th, double pt, double pr, double pth,
                                               double pph, double wtt, double wtp, double wpp) {
    double s, c;
    sincos_def(th, s, c);
    const double se = fma(c, in.sin_eps, s * in.cos_eps);
    const double ce = fma(-s, in.sin_eps, c * in.cos_eps);
    const double s2 = s * s;
    const InvMetric g = mn_inverse_metric<IeeeDiv>(K, r, c, s2);
    const InvMetric gr = mn_inverse_metric<IeeeDiv>(K, r + in.eps, c, s2);
    const InvMetric gh = mn_inverse_metric<IeeeDiv>(K, r, ce, se * se);
    return deriv_from(g, minus(gr, g), minus(gh, g), in, pt, pr, pth, pph, wtt, wtp, wpp);
}

struct Ray {
    double t, r, th, ph, pt, pr, pth, pph;
    double wtt, wtp, wpp;    // p_t^2, 2 p_t p_phi, p_phi^2 (constant along the ray)
    double sn, cs;           // sin and cos of theta carried along the ray (rk4_step)
};

static __device__ __forceinline__ void start_ray(const Camera& C, int64_t pix, Ray& y) {
    const int64_t i = pix % C.W, j = pix / C.W;
    camera_ray(C, i, j, y.pt, y.pr, y.pth, y.pph);
    y.t = 0.0;
    y.r = C.r0;
    y.th = C.th0;
    y.ph = C.ph0;
    y.sn = C.s0;
    y.cs = C.c0;
    y.wtt = y.pt * y.pt;
    y.wtp = (2.0 * y.pt) * y.pph;
    y.wpp = y.pph * y.pph;
}

static __device__ __forceinline__ bool finite6(const Ray& y) {
    return isfinite(y.t) && isfinite(y.r) && isfinite(y.th) && isfinite(y.ph) &&
           isfinite(y.pr) && isfinite(y.pth);
}

// One RK4 step with the right-hand side rhs_at(r, theta, p_r, p_theta);
// returns nu = |dt/dtau| of the first stage.  The weighted sums
// ((k1 + 2 k2) + 2 k3) + k4 are taken as fma(2, k, s): 2 k is exact, so this
// is the same single rounding as s + 2 k.
template <class Rhs>
static __device__ __forceinline__ double rk4_generic(const Rhs& rhs_at, const Integrator& in,
                                                     Ray& y) {
    Deriv k = rhs_at(y.r, y.th, y.pr, y.pth);
    const double nu = fabs(k.qt);
    const double h = div_rn(in.dt, nu);
    const double hh = 0.5 * h;
    double st = k.qt, sr = k.qr, sh = k.qh, sp = k.qp, spr = k.pr, sph = k.ph;
    k = rhs_at(fma(hh, k.qr, y.r), fma(hh, k.qh, y.th), fma(hh, k.pr, y.pr),
               fma(hh, k.ph, y.pth));
    st = fma(2.0, k.qt, st); sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
    sp = fma(2.0, k.qp, sp); spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
    k = rhs_at(fma(hh, k.qr, y.r), fma(hh, k.qh, y.th), fma(hh, k.pr, y.pr),
               fma(hh, k.ph, y.pth));
    st = fma(2.0, k.qt, st); sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
    sp = fma(2.0, k.qp, sp); spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
    k = rhs_at(fma(h, k.qr, y.r), fma(h, k.qh, y.th), fma(h, k.pr, y.pr), fma(h, k.ph, y.pth));
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

// One RK4 step with coordinate time as the parameter (RK4 of Sec. 3.1.2
// applied to dx/dt = f(x)/|dt/dtau|): each stage's derivative is multiplied
// by w = 1/|dt/dtau| of that stage, the stage points are x + (dt/2) k1,
// x + (dt/2) k2, x + dt k3, and the update is x += dt/6 (k1 + 2 k2 + 2 k3 +
// k4), so t advances by dt every step; returns nu of the first stage.
// Divisions IEEE (1/inf = 0 near the Manko-Novikov ring).
template <class Rhs>
static __device__ __forceinline__ double rk4t_generic(const Rhs& rhs_at, const Integrator& in,
                                                      Ray& y) {
    const auto per_t = [](Deriv& k) {
        const double w = 1.0 / fabs(k.qt);
        k.qt = k.qt * w; k.qr = k.qr * w; k.qh = k.qh * w; k.qp = k.qp * w;
        k.pr = k.pr * w; k.ph = k.ph * w;
    };
    const double hh = 0.5 * in.dt;
    Deriv k = rhs_at(y.r, y.th, y.pr, y.pth);
    const double nu = fabs(k.qt);
    per_t(k);
    double st = k.qt, sr = k.qr, sh = k.qh, sp = k.qp, spr = k.pr, sph = k.ph;
    k = rhs_at(fma(hh, k.qr, y.r), fma(hh, k.qh, y.th), fma(hh, k.pr, y.pr),
               fma(hh, k.ph, y.pth));
    per_t(k);
    st = fma(2.0, k.qt, st); sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
    sp = fma(2.0, k.qp, sp); spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
    k = rhs_at(fma(hh, k.qr, y.r), fma(hh, k.qh, y.th), fma(hh, k.pr, y.pr),
               fma(hh, k.ph, y.pth));
    per_t(k);
    st = fma(2.0, k.qt, st); sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
    sp = fma(2.0, k.qp, sp); spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
    k = rhs_at(fma(in.dt, k.qr, y.r), fma(in.dt, k.qh, y.th), fma(in.dt, k.pr, y.pr),
               fma(in.dt, k.ph, y.pth));
    per_t(k);
    st = st + k.qt; sr = sr + k.qr; sh = sh + k.qh; sp = sp + k.qp;
    spr = spr + k.pr; sph = sph + k.ph;
    const double h6 = in.dt * (1.0 / 6.0);
    y.t = fma(h6, st, y.t);
    y.r = fma(h6, sr, y.r);
    y.th = fma(h6, sh, y.th);
    y.ph = fma(h6, sp, y.ph);
    y.pr = fma(h6, spr, y.pr);
    y.pth = fma(h6, sph, y.pth);
    return nu;
}

// One explicit Euler step x += h f(x) with the same h = dt/|dt/dtau| (paper
// Sec. 3.1.1); returns nu.
template <class Rhs>
static __device__ __forceinline__ double euler_generic(const Rhs& rhs_at, const Integrator& in,
                                                       Ray& y) {
    const Deriv k = rhs_at(y.r, y.th, y.pr, y.pth);
    const double nu = fabs(k.qt);
    const double h = div_rn(in.dt, nu);
    y.t = fma(h, k.qt, y.t);
    y.r = fma(h, k.qr, y.r);
    y.th = fma(h, k.qh, y.th);
    y.ph = fma(h, k.qp, y.ph);
    y.pr = fma(h, k.pr, y.pr);
    y.pth = fma(h, k.ph, y.pth);
    return nu;
}

// One Kerr-Newman RK4 step with theta entering through its sin and cos
// only (the carried form): the ray carries (sin, cos) of its angle, each
// stage point's pair is that pair rotated (rotate_sc) by the stage's
// increment c_k h dtheta/dtau, and the update rotates the carried pair by the
// step's increment h/6 S_theta while theta itself is summed as before.  Same
// RK4 as rk4_generic; the metric sees sin and cos of the unrounded stage
// angles, and the carried pair departs from sin/cos of the summed theta only
// by the accumulated rounding of the rotations (a random walk of ~1e-16 per
// step).
// dt/dtau = g^tt p_t + g^tphi p_phi and dphi/dtau = g^tphi p_t + g^phph p_phi
// with p_t, p_phi constant along the ray, so the weighted sums of t and phi
// are taken over the three components and contracted once per step.
// GENERAL = false takes no branch: it rotates by rotate_small and refines
// every theta-displaced reciprocal from the base point's (rhs_sc SEEDED), and
// returns in dmax the largest |increment| or the largest starting residual of
// those refinements times ROT_SERIES_MAX / NEWTON_SEED_MAX, whichever is
// larger; the step equals the GENERAL one when dmax <= ROT_SERIES_MAX.
template <bool GENERAL, bool UNIT_COS = false>
static __device__ __forceinline__ double rk4_carry(const Hole& H, const Integrator& in, Ray& y,
                                                   double& dmax) {
    // p-dot comes unscaled (RAW): -1/(2 eps) is folded into the step sizes
    // of the momentum components, hh in.scale, h in.scale and h/6 in.scale
    double emax = 0.0;
    const auto f = [&](double r, double sn, double cs, double pr, double pth) {
        return rhs_sc<UNIT_COS, true, !GENERAL>(H, in, r, sn, cs, y.pt, pr, pth, y.pph, y.wtt,
                                                y.wtp, y.wpp, &emax);
    };
    dmax = 0.0;
    const auto rot = [&](double d, double& sn, double& cs) {
        if constexpr (GENERAL) {
            rotate_sc(y.sn, y.cs, d, sn, cs);
        } else {
            dmax = fmax(dmax, fabs(d));
            rotate_small(y.sn, y.cs, d, sn, cs);
        }
    };
    double sn, cs;
    Deriv k = f(y.r, y.sn, y.cs, y.pr, y.pth);
    const double nu = fabs(k.qt);
    const double h = div_rn(in.dt, nu);
    const double hh = 0.5 * h;
    const double hhs = hh * in.scale;
    double stt = k.gtt, stp = k.gtp, spp = k.gpp, sr = k.qr, sh = k.qh, spr = k.pr, sph = k.ph;
    rot(hh * k.qh, sn, cs);
    k = f(fma(hh, k.qr, y.r), sn, cs, fma(hhs, k.pr, y.pr), fma(hhs, k.ph, y.pth));
    stt = fma(2.0, k.gtt, stt); stp = fma(2.0, k.gtp, stp); spp = fma(2.0, k.gpp, spp);
    sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
    spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
    rot(hh * k.qh, sn, cs);
    k = f(fma(hh, k.qr, y.r), sn, cs, fma(hhs, k.pr, y.pr), fma(hhs, k.ph, y.pth));
    stt = fma(2.0, k.gtt, stt); stp = fma(2.0, k.gtp, stp); spp = fma(2.0, k.gpp, spp);
    sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
    spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
    rot(h * k.qh, sn, cs);
    const double hs = h * in.scale;
    k = f(fma(h, k.qr, y.r), sn, cs, fma(hs, k.pr, y.pr), fma(hs, k.ph, y.pth));
    stt = stt + k.gtt; stp = stp + k.gtp; spp = spp + k.gpp;
    sr = sr + k.qr; sh = sh + k.qh;
    spr = spr + k.pr; sph = sph + k.ph;
    const double st = fma(stt, y.pt, stp * y.pph);
    const double sp = fma(stp, y.pt, spp * y.pph);
    const double h6 = h * (1.0 / 6.0);
    const double h6s = h6 * in.scale;
    rot(h6 * sh, sn, cs);
    y.t = fma(h6, st, y.t);
    y.r = fma(h6, sr, y.r);
    y.th = fma(h6, sh, y.th);
    y.ph = fma(h6, sp, y.ph);
    y.pr = fma(h6s, spr, y.pr);
    y.pth = fma(h6s, sph, y.pth);
    y.sn = sn;
    y.cs = cs;
    if constexpr (!GENERAL) dmax = fmax(dmax, emax * (ROT_SERIES_MAX / NEWTON_SEED_MAX));
    return nu;
}

// The tracing kernels take the branch-free step; a ray one of whose steps
// rotates by more than 1/32 (it needs h |dtheta/dtau| > 1/32: on the
// configured workloads only rays that graze the polar axis, where dp_theta/dtau
// swings within a step) is not finished there: its flag is set to PENDING and
// a second pass over the outputs traces it again from its start with the
// general step.  Either way each ray's result is that of the general step.
enum { PENDING = -2 };

template <bool UNIT_COS = false>
static __device__ __forceinline__ double rk4_step(const Hole& H, const Integrator& in, Ray& y,
                                                  bool& pending) {
    double dmax;
    const double nu = rk4_carry<false, UNIT_COS>(H, in, y, dmax);
    pending = dmax > ROT_SERIES_MAX;
    return nu;
}

static __device__ __forceinline__ double rk4_step_general(const Hole& H, const Integrator& in,
                                                          Ray& y) {
    double dmax;
    return rk4_carry<true>(H, in, y, dmax);
}

// One Kerr-Newman RK4 step from theta itself (sincos_def at every stage
// point): the binary64 steps of the mixed-precision tracer, whose binary32
// steps do not carry the (sin, cos) pair.
static __device__ __forceinline__ double rk4_step_direct(const Hole& H, const Integrator& in,
                                                         Ray& y) {
    return rk4_generic(
        [&](double r, double th, double pr, double pth) {
            return rhs(H, in, r, th, y.pt, pr, pth, y.pph, y.wtt, y.wtp, y.wpp);
        },
        in, y);
}

// Methods of the one-ray-per-lane kernels (the values of gr_integrator.method).
enum { M_RK4 = 0, M_EULER = 1, M_RK4_TIME = 2 };

// One explicit Euler or coordinate-time RK4 step on Kerr-Newman in the
// carried form of rk4_carry: the ray's (sin, cos) pair, rotated by each stage
// point's increment of theta and, after the update, by the step's; the same
// Euler and coordinate-time RK4 as euler_generic and rk4t_generic otherwise
// (p-dot scaled in the right-hand side, correctly rounded 1/|dt/dtau| per
// stage).
// GENERAL and dmax as for rk4_carry.
template <int METHOD, bool GENERAL, bool UNIT_COS = false>
static __device__ __forceinline__ double kn_carry_step(const Hole& H, const Integrator& in,
                                                       Ray& y, double& dmax) {
    double emax = 0.0;
    const auto f = [&](double r, double sn, double cs, double pr, double pth) {
        return rhs_sc<UNIT_COS, false, !GENERAL>(H, in, r, sn, cs, y.pt, pr, pth, y.pph, y.wtt,
                                                 y.wtp, y.wpp, &emax);
    };
    const auto seeded = [&]() {
        if constexpr (!GENERAL) dmax = fmax(dmax, emax * (ROT_SERIES_MAX / NEWTON_SEED_MAX));
    };
    dmax = 0.0;
    const auto rot = [&](double d, double& sn, double& cs) {
        if constexpr (GENERAL) {
            rotate_sc(y.sn, y.cs, d, sn, cs);
        } else {
            dmax = fmax(dmax, fabs(d));
            rotate_small(y.sn, y.cs, d, sn, cs);
        }
    };
    double sn, cs;
    if constexpr (METHOD == M_EULER) {
        const Deriv k = f(y.r, y.sn, y.cs, y.pr, y.pth);
        const double nu = fabs(k.qt);
        const double h = div_rn(in.dt, nu);
        rot(h * k.qh, sn, cs);
        y.t = fma(h, k.qt, y.t);
        y.r = fma(h, k.qr, y.r);
        y.th = fma(h, k.qh, y.th);
        y.ph = fma(h, k.qp, y.ph);
        y.pr = fma(h, k.pr, y.pr);
        y.pth = fma(h, k.ph, y.pth);
        y.sn = sn;
        y.cs = cs;
        seeded();
        return nu;
    } else {
        // w = 1/|dt/dtau| correctly rounded (rcp_rn: the same bits as IEEE
        // division for the finite, normal values a stage produces)
        const auto per_t = [](Deriv& k) {
            const double w = rcp_rn(fabs(k.qt));
            k.qt = k.qt * w; k.qr = k.qr * w; k.qh = k.qh * w; k.qp = k.qp * w;
            k.pr = k.pr * w; k.ph = k.ph * w;
        };
        const double hh = 0.5 * in.dt;
        Deriv k = f(y.r, y.sn, y.cs, y.pr, y.pth);
        const double nu = fabs(k.qt);
        per_t(k);
        double st = k.qt, sr = k.qr, sh = k.qh, sp = k.qp, spr = k.pr, sph = k.ph;
        rot(hh * k.qh, sn, cs);
        k = f(fma(hh, k.qr, y.r), sn, cs, fma(hh, k.pr, y.pr), fma(hh, k.ph, y.pth));
        per_t(k);
        st = fma(2.0, k.qt, st); sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
        sp = fma(2.0, k.qp, sp); spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
        rot(hh * k.qh, sn, cs);
        k = f(fma(hh, k.qr, y.r), sn, cs, fma(hh, k.pr, y.pr), fma(hh, k.ph, y.pth));
        per_t(k);
        st = fma(2.0, k.qt, st); sr = fma(2.0, k.qr, sr); sh = fma(2.0, k.qh, sh);
        sp = fma(2.0, k.qp, sp); spr = fma(2.0, k.pr, spr); sph = fma(2.0, k.ph, sph);
        rot(in.dt * k.qh, sn, cs);
        k = f(fma(in.dt, k.qr, y.r), sn, cs, fma(in.dt, k.pr, y.pr), fma(in.dt, k.ph, y.pth));
        per_t(k);
        st = st + k.qt; sr = sr + k.qr; sh = sh + k.qh; sp = sp + k.qp;
        spr = spr + k.pr; sph = sph + k.ph;
        const double h6 = in.dt * (1.0 / 6.0);
        rot(h6 * sh, sn, cs);
        y.t = fma(h6, st, y.t);
        y.r = fma(h6, sr, y.r);
        y.th = fma(h6, sh, y.th);
        y.ph = fma(h6, sp, y.ph);
        y.pr = fma(h6, spr, y.pr);
        y.pth = fma(h6, sph, y.pth);
        y.sn = sn;
        y.cs = cs;
        seeded();
        return nu;
    }
}

template <int METHOD>
static __device__ __forceinline__ double mn_step(const MnHole& K, const Integrator& in, Ray& y) {
    const auto f = [&](double r, double th, double pr, double pth) {
        return rhs_mn(K, in, r, th, y.pt, pr, pth, y.pph, y.wtt, y.wtp, y.wpp);
    };
    if constexpr (METHOD == M_EULER) return euler_generic(f, in, y);
    else if constexpr (METHOD == M_RK4_TIME) return rk4t_generic(f, in, y);
    else return rk4_generic(f, in, y);
}

// Exit tests after an update: the ring (kernels built with DISK), escape,
// horizon, a non-finite state, the step limit.
template <bool DISK = false>
static __device__ __forceinline__ int exit_flag(const Integrator& in, double r_esc, const Ray& y,
                                         double nu, int s) {
    if (DISK && y.r >= in.disk_r_in && y.r <= in.disk_r_out &&
        fabs(y.th - PI2_HI) <= in.disk_dth)
        return GR_FLAG_DISK;
    if (y.r > r_esc) return GR_FLAG_ESCAPE;
    if (nu > in.hnorm) return GR_FLAG_HORIZON;
    if (!finite6(y)) return GR_FLAG_INVALID;
    if (s >= in.max_steps) return GR_FLAG_TIMEOUT;
    return RUNNING;
}

template <typename T>
static __device__ __forceinline__ void put(void* p, int64_t k, double v) {
    if (p) reinterpret_cast<T*>(p)[k] = (T)v;
}

template <typename T>
static __device__ __forceinline__ void write_ray(const OutPtrs& o, int64_t k, const Ray& y, int flag,
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

// Ray of lane g in a one-ray-per-lane launch, false for a lane without one.
// A frame is cut into 8x8 pixel tiles, one per wave (row-major over the
// tiles), so that a wave's rays start side by side and take nearly the same
// number of steps; lanes of a ragged edge tile that fall outside the frame
// have no ray, and the grid needs 64 lanes per tile.  With a pixel list, lane
// g traces list entry g.  k: output index, pix: pixel.
static __device__ __forceinline__ bool static_ray(const FrameArgs& A, int64_t g, int64_t& k,
                                                  int64_t& pix) {
    if (A.pixels) {
        k = g;
        if (k >= A.nray) return false;
        pix = (int64_t)A.pixels[k];
        return true;
    }
    const int64_t W = A.cam.W, H = A.cam.H;
    const int64_t tiles_x = (W + 7) >> 3;
    const int64_t wave = g >> 6;
    const int lane = (int)(g & 63);
    const int64_t i = (wave % tiles_x) * 8 + (lane & 7);
    const int64_t j = (wave / tiles_x) * 8 + (lane >> 3);
    if (i >= W || j >= H) return false;
    k = pix = j * W + i;
    return true;
}

// Flag for a freshly started ray: invalid start or a zero step limit end it.
static __device__ __forceinline__ int start_flag(const Integrator& in, const Ray& y) {
    if (!(finite6(y) && isfinite(y.pt) && isfinite(y.pph))) return GR_FLAG_INVALID;
    if (in.max_steps <= 0) return GR_FLAG_TIMEOUT;
    return RUNNING;
}

// Wave-wide work distribution: lanes with `want` set receive consecutive ids
// from the global counter (one atomic per wave), in lane order.
static __device__ __forceinline__ int64_t take_ids(bool want, unsigned long long* counter) {
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

}  // namespace detail
}  // namespace gr
