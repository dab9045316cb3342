// Binary64 arithmetic of the tracer, usable on the host and on gfx950.
//
// The operation sequence here is fixed: every product that is fused is an
// explicit fma(), nothing else may be contracted (translation units that
// include this file are compiled with -ffp-contract=off), and sin/cos follow
// the series definition below.  The forward difference of step 1e-8 divides
// rounding noise by 1e-8, so a one-ulp difference anywhere in a ray's state
// moves its end angles by ~1e-9 rad; results are only reproducible when every
// operation is specified.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define GR_HD __host__ __device__ __forceinline__

namespace gr {

// ---------------------------------------------------------------- sin / cos
// x = k pi/2 + r, k = rint(x * fl(2/pi)), r = (x - k PI2_HI) - k PI2_LO via two
// fma (the first is exact for moderate |x|); then
//   sin r = r + (r z) (S1 + z (S2 + ... + z S8)),   S_n = (-1)^n/(2n+1)!
//   cos r = 1 + z (C1 + z (C2 + ... + z C8)),       C_n = (-1)^n/(2n)!
// with z = r*r, Horner in fma, and the quadrant k mod 4 selecting/negating.
// Accurate to 1.4 ulp; truncation below 1e-18 on |r| <= pi/4.

constexpr double factorial(int m) {
    double f = 1.0;
    for (int i = 2; i <= m; ++i) f *= (double)i;   // exact for m <= 18
    return f;
}
constexpr double series_coef(int m) {             // (-1)^(m/2) / m!, one rounding
    return ((m / 2) % 2 ? -1.0 : 1.0) * (1.0 / factorial(m));
}

constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;   // fl(2/pi)
constexpr double PI2_HI = 0x1.921fb54442d18p+0;        // fl(pi/2)
constexpr double PI2_LO = 0x1.1a62633145c07p-54;       // fl(pi/2 - PI2_HI)

GR_HD void sincos_def(double x, double& s_out, double& c_out) {
    const double k = rint(x * TWO_OVER_PI);
    double r = fma(-k, PI2_HI, x);
    r = fma(-k, PI2_LO, r);
    const double z = r * r;
    double ps = series_coef(17);
    ps = fma(ps, z, series_coef(15));
    ps = fma(ps, z, series_coef(13));
    ps = fma(ps, z, series_coef(11));
    ps = fma(ps, z, series_coef(9));
    ps = fma(ps, z, series_coef(7));
    ps = fma(ps, z, series_coef(5));
    ps = fma(ps, z, series_coef(3));
    double pc = series_coef(16);
    pc = fma(pc, z, series_coef(14));
    pc = fma(pc, z, series_coef(12));
    pc = fma(pc, z, series_coef(10));
    pc = fma(pc, z, series_coef(8));
    pc = fma(pc, z, series_coef(6));
    pc = fma(pc, z, series_coef(4));
    pc = fma(pc, z, series_coef(2));
    const double sr = fma(r * z, ps, r);
    const double cr = fma(z, pc, 1.0);
    const double quad = k - 4.0 * floor(0.25 * k);     // k mod 4, exact
    const bool swap = (quad == 1.0) || (quad == 3.0);
    double s = swap ? cr : sr;
    double c = swap ? sr : cr;
    s = (quad >= 2.0) ? -s : s;
    c = (quad == 1.0 || quad == 2.0) ? -c : c;
    s_out = s;
    c_out = c;
}

// Rotation of a (sin, cos) pair by an angle d: (sin(x + d), cos(x + d)) from
// s = sin x, c = cos x by the angle-addition identity.  sin and cos - 1 of
// u = d 2^-m, m the least count of halvings with |u| <= 1/32 (at most 64),
// come from their Taylor series through u^7 and u^6 (the first omitted terms
// are below 8e-20 and 2.3e-17 there, the latter multiplied by s or c in the
// rotation: at most a fifth of an ulp of the result, and far less at the
// increments of ordinary steps), then m double-angle steps
// sin 2u = 2 sin u (1 + (cos u - 1)), cos 2u - 1 = -2 sin^2 u give those of d;
// each result takes two fma, s (1 + (cos d - 1)) first, then the sin d term.  rotate_small is the case m = 0 alone (no branch), equal to
// rotate_sc bit for bit wherever |d| <= 1/32.
constexpr double ROT_SERIES_MAX = 0.03125;

GR_HD void small_angle(double u, double& sd, double& cm1) {
    const double z = u * u;
    double ps = series_coef(7);
    ps = fma(ps, z, series_coef(5));
    ps = fma(ps, z, series_coef(3));
    sd = fma(u * z, ps, u);
    double pc = series_coef(6);
    pc = fma(pc, z, series_coef(4));
    pc = fma(pc, z, series_coef(2));
    cm1 = z * pc;
}

GR_HD void rotate_by(double s, double c, double sd, double cm1, double& s_out, double& c_out) {
    s_out = fma(c, sd, fma(s, cm1, s));      // s cos d, then + c sin d
    c_out = fma(-s, sd, fma(c, cm1, c));     // c cos d, then - s sin d
}

GR_HD void rotate_small(double s, double c, double d, double& s_out, double& c_out) {
    double sd, cm1;
    small_angle(d, sd, cm1);
    rotate_by(s, c, sd, cm1, s_out, c_out);
}

GR_HD void rotate_sc(double s, double c, double d, double& s_out, double& c_out) {
    double u = d;
    int m = 0;
    while (m < 64 && fabs(u) > ROT_SERIES_MAX) {
        u *= 0.5;
        ++m;
    }
    double sd, cm1;
    small_angle(u, sd, cm1);
    for (int i = 0; i < m; ++i) {
        const double s2 = 2.0 * fma(sd, cm1, sd);
        cm1 = -2.0 * (sd * sd);
        sd = s2;
    }
    rotate_by(s, c, sd, cm1, s_out, c_out);
}

// ------------------------------------------------------------ black hole
// Uniform per-hole constants.  a2 = a*a, aq = a2 + Q*Q, M2 = 2M, Q2 = Q*Q,
// aM2 = a M2, aQ2 = a Q2.
struct Hole {
    double a, a2, aq, M2, Q2;
    double aM2, aQ2;           // a (2M) and a Q^2: a(2Mr - Q^2) = fma(aM2, r, -aQ2)
};

GR_HD Hole make_hole(double M, double a, double Q) {
    Hole h;
    h.a = a;
    h.a2 = a * a;
    h.Q2 = Q * Q;
    h.aq = h.a2 + h.Q2;
    h.M2 = 2.0 * M;
    h.aM2 = a * h.M2;
    h.aQ2 = a * h.Q2;
    return h;
}

// Terms of the metric that depend on theta only.
struct ThetaTerms {
    double s2, w;              // sin^2, a^2 sin^2
};

GR_HD ThetaTerms theta_terms_s(const Hole& H, double s) {
    ThetaTerms T;
    T.s2 = s * s;
    T.w = H.a2 * T.s2;
    return T;
}

GR_HD ThetaTerms theta_terms(const Hole& H, double theta) {
    double s, c;
    sincos_def(theta, s, c);
    return theta_terms_s(H, s);
}

// Terms that depend on r only.
struct RadialTerms {
    double r2, ra, rara, Delta, aF, DD;   // r^2, r^2+a^2, (r^2+a^2)^2, Delta, a(2Mr - Q^2), Delta^2
};

GR_HD RadialTerms radial_terms(const Hole& H, double r) {
    RadialTerms R;
    R.r2 = r * r;
    R.ra = R.r2 + H.a2;
    R.rara = R.ra * R.ra;
    R.Delta = fma(r, r - H.M2, H.aq);
    R.aF = fma(H.aM2, r, -H.aQ2);
    R.DD = R.Delta * R.Delta;
    return R;
}

// Inverse Kerr-Newman metric, the five independent components
//   g^tt = -Sigma2/(rho2 Delta), g^tphi = -a(2Mr - Q^2)/(rho2 Delta),
//   g^rr = Delta/rho2, g^thth = 1/rho2,
//   g^phph = (Delta - a^2 sin^2)/(rho2 Delta sin^2),
// rho2 = r^2 + a^2 cos^2, Sigma2 = (r^2+a^2)^2 - a^2 Delta sin^2.
struct InvMetric {
    double tt, tp, rr, hh, pp;
};

// rho2 Delta at (r-terms, theta-terms), with rho2 = r^2 + a^2 cos^2 formed
// as (r^2 + a^2) - a^2 sin^2 from the terms the other components use: outside
// a horizon r >= a, so the subtraction keeps rho2 to a few ulp.
GR_HD double rho2_delta(const Hole& H, const RadialTerms& R, const ThetaTerms& T) {
    return (R.ra - T.w) * R.Delta;
}

// The five components from the shared reciprocals inv = 1/(rho2 Delta) and
// is = 1/(rho2 Delta sin^2).
GR_HD InvMetric metric_from(const Hole& H, const RadialTerms& R, const ThetaTerms& T,
                            double inv, double is) {
    const double Sigma2 = fma(-T.w, R.Delta, R.rara);
    InvMetric g;
    g.tt = -(Sigma2 * inv);
    g.tp = -(R.aF * inv);
    g.rr = R.DD * inv;
    g.hh = R.Delta * inv;
    g.pp = (R.Delta - T.w) * is;
    return g;
}

// The forward difference of the five components between a displaced point
// (R, T, inv, is) and the base point's g0: each displaced component's last
// product and its difference from g0 in one fma, so the difference is
// rounded once (the displaced component itself is never rounded).
GR_HD InvMetric metric_diff(const Hole& H, const RadialTerms& R, const ThetaTerms& T,
                            double inv, double is, const InvMetric& g0) {
    const double Sigma2 = fma(-T.w, R.Delta, R.rara);
    InvMetric d;
    d.tt = fma(-Sigma2, inv, -g0.tt);
    d.tp = fma(-R.aF, inv, -g0.tp);
    d.rr = fma(R.DD, inv, -g0.rr);
    d.hh = fma(R.Delta, inv, -g0.hh);
    d.pp = fma(R.Delta - T.w, is, -g0.pp);
    return d;
}

// Full inverse metric at one point: is divided, inv = is sin^2.
GR_HD InvMetric inverse_metric(const Hole& H, const RadialTerms& R, const ThetaTerms& T) {
    const double is = 1.0 / (rho2_delta(H, R, T) * T.s2);
    return metric_from(H, R, T, is * T.s2, is);
}

// 1/x from y0 = 1/x0 for a nearby x0: two Newton steps y <- y + y (1 - x y).
// Each squares the relative error e0 = 1 - x y0; for the displacements of the
// forward differences |e0| is about eps times a logarithmic derivative of
// rho2 Delta (below 1e-4 even at the horizon cutoff), so e0^4 is at or below
// the rounding of the result.
GR_HD double recip_newton(double x, double y0) {
    double e = fma(-x, y0, 1.0);
    const double y = fma(y0, e, y0);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Three Newton steps: relative error e0^8 plus rounding, within about an
// ulp for |e0| <= 2^-8.
GR_HD double recip_newton3(double x, double y0) {
    double e = fma(-x, y0, 1.0);
    double y = fma(y0, e, y0);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// -------------------------------------------------------------------- exp
// x = k ln2 + r, k = rint(x * fl(1/ln2)), r = (x - k LN2_HI) - k LN2_LO via
// two fma (|r| <= ln2/2); exp r = sum_{n=0}^{13} r^n/n! by Horner in fma
// (truncation below 5e-18 relative), exp x = 2^k exp r.  Within 1 ulp.
// Overflow gives +inf, x < -746 gives 0, NaN stays NaN.
constexpr double LOG2E = 0x1.71547652b82fep+0;         // fl(1/ln2)
constexpr double LN2_HI = 0x1.62e42fefa39efp-1;        // fl(ln2)
constexpr double LN2_LO = 0x1.abc9e3b39803fp-56;       // fl(ln2 - LN2_HI)
constexpr double exp_coef(int n) { return 1.0 / factorial(n); }   // one rounding

GR_HD double exp_def(double x) {
    // no branches: x is clamped to [-746, 710], where exp(710) overflows to
    // inf and exp(-746) rounds to 0 through the scaling, as the out-of-range
    // values should; NaN is restored at the end
    const double xr = fmin(fmax(x, -746.0), 710.0);
    const double k = rint(xr * LOG2E);
    double r = fma(-k, LN2_HI, xr);
    r = fma(-k, LN2_LO, r);
    double p = exp_coef(13);
    p = fma(p, r, exp_coef(12));
    p = fma(p, r, exp_coef(11));
    p = fma(p, r, exp_coef(10));
    p = fma(p, r, exp_coef(9));
    p = fma(p, r, exp_coef(8));
    p = fma(p, r, exp_coef(7));
    p = fma(p, r, exp_coef(6));
    p = fma(p, r, exp_coef(5));
    p = fma(p, r, exp_coef(4));
    p = fma(p, r, exp_coef(3));
    p = fma(p, r, exp_coef(2));
    p = fma(p, r, exp_coef(1));
    p = fma(p, r, 1.0);
    const double e = ldexp(p, (int)k);
    return x != x ? x : e;
}

// ----------------------------------------------------------- Manko-Novikov
// The quadrupole Manko-Novikov spacetime (arXiv 2310.15183, Sec. 2.2.3;
// inverse components of the appendix listing's metricAtPoint):
//   ds^2 = -f (dt - omega dphi)^2
//          + f^{-1} [e^{2 gamma} rho^2 (dr^2/Delta + dtheta^2) + Delta sin^2 dphi^2]
// in prolate spheroidal x = (r - M)/k, y = cos(theta), with rho^2 = k^2 (x^2 - y^2),
// Delta = k^2 (x^2 - 1) and, R = sqrt(x^2 + y^2 - 1), P_l = P_l(x y / R),
//   a_ = -alpha exp(-2 beta (sum_l (x - y) P_l / R^{l+1} - 1)),
//   b_ =  alpha exp( 2 beta (1 + sum_l (-1)^{3-l} (x + y) P_l / R^{l+1})),
//   A = (x^2-1)(1+a_b_)^2 - (1-y^2)(b_-a_)^2,
//   B = [x+1 + (x-1) a_b_]^2 + [(1+y) a_ + (1-y) b_]^2,
//   C = (x^2-1)(1+a_b_)[b_-a_ - y(a_+b_)] + (1-y^2)(b_-a_)[1+a_b_ + x(1-a_b_)],
//   f = e^{2 psi} A/B, psi = beta P_2/R^3,
//   omega = 2k e^{-2 psi} C/A - 4k alpha/(1-alpha^2),
//   e^{2 gamma} rho^2 = k^2 e^{2G} A/(1-alpha^2)^2,
//   G = 3 beta^2 (P_3^2 - P_2^2)/(2 R^6) + beta (sum_l [x-y + (-1)^l (x+y)] P_l/R^{l+1} - 2),
// sums over l = 0..2; alpha = (-M + sqrt(M^2 - (S/M)^2))/(S/M),
// k = M (1-alpha^2)/(1+alpha^2), beta = q M^3/k^3.
struct MnHole {
    double M, alpha, k, beta;
    double ik, k2, twok;   // 1/k, k^2, 2k
    double om0;            // 4 k alpha / (1 - alpha^2)
    double iw2;            // 1 / (1 - alpha^2)^2
};

inline MnHole make_mn_hole(double M, double S, double q) {
    MnHole h;
    const double chi = S / M;
    h.M = M;
    h.alpha = (-M + sqrt(M * M - chi * chi)) / chi;
    const double al2 = h.alpha * h.alpha;
    h.k = M * ((1.0 - al2) / (1.0 + al2));
    h.beta = (q * (M * M * M)) / (h.k * h.k * h.k);
    h.ik = 1.0 / h.k;
    h.k2 = h.k * h.k;
    h.twok = 2.0 * h.k;
    h.om0 = (4.0 * h.k * h.alpha) / (1.0 - al2);
    h.iw2 = 1.0 / ((1.0 - al2) * (1.0 - al2));
    return h;
}

// IEEE division (correctly rounded, with IEEE special values: near the
// singular ring of the Manko-Novikov horizon the exponentials overflow and
// 1/inf = 0 has to stay 0).
struct IeeeDiv {
    GR_HD static double rcp(double x) { return 1.0 / x; }
    GR_HD static double div(double a, double x) { return a / x; }
};

// The five inverse components at (r, theta) from y = cos(theta) and
// s2 = sin^2(theta); Div supplies correctly rounded 1/x and a/x.
template <class Div>
GR_HD InvMetric mn_inverse_metric(const MnHole& K, double r, double y, double s2) {
    const double beta = K.beta;
    const double x = (r - K.M) * K.ik;
    const double x2 = x * x, y2 = y * y;
    const double R = sqrt((x2 + y2) - 1.0);
    const double iR = Div::rcp(R);
    const double iR2 = iR * iR, iR3 = iR2 * iR;
    const double u = (x * y) * iR;
    const double P1 = u;
    const double P2 = fma(1.5 * u, u, -0.5);
    const double P3 = u * fma(2.5 * u, u, -1.5);
    const double L1 = fma(P2, iR3, fma(P1, iR2, iR));      // sum P_l / R^{l+1}
    const double L2 = fma(P2, iR3, fma(-P1, iR2, iR));     // sum (-1)^l P_l / R^{l+1}
    const double Sa = (x - y) * L1;
    const double Sb = -((x + y) * L2);
    const double Sg = fma(x - y, L1, (x + y) * L2);
    const double ea = exp_def((-2.0 * beta) * (Sa - 1.0));
    const double eb = exp_def((2.0 * beta) * (1.0 + Sb));
    const double am = -(K.alpha * ea);
    const double bm = K.alpha * eb;
    const double psi = (beta * P2) * iR3;
    const double iR6 = iR3 * iR3;
    const double G = fma((1.5 * (beta * beta)) * iR6, (P3 * P3) - (P2 * P2), beta * (Sg - 2.0));
    const double ab = am * bm;
    const double opab = 1.0 + ab, omab = 1.0 - ab;
    const double bma = bm - am, apb = am + bm;
    const double xm1 = x2 - 1.0, ym1 = 1.0 - y2;
    const double A = fma(xm1, opab * opab, -(ym1 * (bma * bma)));
    const double B1 = fma(x - 1.0, ab, x + 1.0);
    const double B2 = fma(1.0 + y, am, (1.0 - y) * bm);
    const double B = fma(B1, B1, B2 * B2);
    const double C = fma(xm1 * opab, fma(-y, apb, bma), (ym1 * bma) * fma(x, omab, opab));
    const double e2psi = exp_def(2.0 * psi);
    const double fA = e2psi * A;
    const double f = Div::div(fA, B);
    const double omega = Div::div(K.twok * C, fA) - K.om0;
    const double e2g_rho2 = ((K.k2 * exp_def(2.0 * G)) * A) * K.iw2;
    const double Delta = K.k2 * xm1;
    const double iD = Div::rcp(Delta * s2);
    const double ie = Div::rcp(e2g_rho2);
    const double fo = f * omega;
    InvMetric g;
    g.tt = fma(fo * omega, iD, -Div::rcp(f));
    g.tp = fo * iD;
    g.rr = (f * Delta) * ie;
    g.hh = f * ie;
    g.pp = f * iD;
    return g;
}

// ----------------------------------------------------------------- camera
// Frame constants of the pinhole camera (host side, once per frame):
// half-extents tan(fov/2) and tan(fov/2) H/W, the orthonormal-frame scale
// factors sqrt(g_rr), sqrt(g_thth), sqrt(g_phph) of the covariant metric, and
// the inverse metric at the camera.
struct Camera {
    double r0, th0, ph0;
    double s0, c0;                 // sincos_def(th0)
    double tan_h, tan_v;
    double er, eth, eph;
    InvMetric g;
    int32_t W, H;
};

inline Camera make_camera(const Hole& Hh, double r0, double th0, double ph0, double fov,
                          int32_t W, int32_t H) {
    Camera C;
    C.r0 = r0;
    C.th0 = th0;
    C.ph0 = ph0;
    C.W = W;
    C.H = H;
    double sf, cf;
    sincos_def(0.5 * fov, sf, cf);
    C.tan_h = sf / cf;
    C.tan_v = (C.tan_h * (double)H) / (double)W;
    sincos_def(th0, C.s0, C.c0);
    const ThetaTerms T = theta_terms_s(Hh, C.s0);
    const RadialTerms R = radial_terms(Hh, r0);
    const double rho2 = fma(Hh.a2, C.c0 * C.c0, R.r2);
    const double Sigma2 = fma(-T.w, R.Delta, R.rara);
    C.er = sqrt(rho2 / R.Delta);                 // sqrt(g_rr)
    C.eth = sqrt(rho2);                          // sqrt(g_thth)
    C.eph = sqrt((Sigma2 * T.s2) / rho2);        // sqrt(g_phph)
    C.g = inverse_metric(Hh, R, T);
    return C;
}

// The same frame constants for a Manko-Novikov spacetime: the orthonormal
// scale factors from the inverse metric at the camera, g_rr = 1/g^rr,
// g_thth = 1/g^thth and g_phph = g^tt / (g^tt g^phph - (g^tphi)^2) (inverse of
// the (t, phi) block).
inline Camera make_camera_mn(const MnHole& K, double r0, double th0, double ph0, double fov,
                             int32_t W, int32_t H) {
    Camera C;
    C.r0 = r0;
    C.th0 = th0;
    C.ph0 = ph0;
    C.W = W;
    C.H = H;
    double sf, cf;
    sincos_def(0.5 * fov, sf, cf);
    C.tan_h = sf / cf;
    C.tan_v = (C.tan_h * (double)H) / (double)W;
    sincos_def(th0, C.s0, C.c0);
    C.g = mn_inverse_metric<IeeeDiv>(K, r0, C.c0, C.s0 * C.s0);
    C.er = sqrt(1.0 / C.g.rr);
    C.eth = sqrt(1.0 / C.g.hh);
    C.eph = sqrt(C.g.tt / ((C.g.tt * C.g.pp) - (C.g.tp * C.g.tp)));
    return C;
}

// Initial covector of pixel (i, j): direction n = (-1, -y, x)/|.| in the
// camera's (e_r, e_theta, e_phi) frame, p_j = n_j sqrt(g_jj), p_t the root of
// H = 0 with dt/dtau < 0, all scaled so that dt/dtau = -1.
GR_HD void camera_ray(const Camera& C, int64_t i, int64_t j, double& pt, double& pr,
                      double& pth, double& pph) {
    const double x = ((double)(2 * i + 1 - C.W) / (double)C.W) * C.tan_h;
    const double y = ((double)(C.H - 2 * j - 1) / (double)C.H) * C.tan_v;
    const double inv_n = 1.0 / sqrt((1.0 + x * x) + y * y);
    const double qr = (-inv_n) * C.er;
    const double qh = ((-y) * inv_n) * C.eth;
    const double qp = (x * inv_n) * C.eph;
    const double S = (C.g.rr * (qr * qr) + C.g.hh * (qh * qh)) + C.g.pp * (qp * qp);
    const double b = C.g.tp * qp;
    const double D = b * b - C.g.tt * S;
    const double sD = sqrt(D);
    const double qt = (-b - sD) / C.g.tt;
    const double k = 1.0 / sD;
    pt = qt * k;
    pr = qr * k;
    pth = qh * k;
    pph = qp * k;
}

}  // namespace gr
