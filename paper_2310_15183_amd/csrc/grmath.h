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

// ------------------------------------------------------------ black hole
// Uniform per-hole constants.  a2 = a*a, aq = a2 + Q*Q, M2 = 2M, Q2 = Q*Q.
struct Hole {
    double a, a2, aq, M2, Q2;
};

GR_HD Hole make_hole(double M, double a, double Q) {
    Hole h;
    h.a = a;
    h.a2 = a * a;
    h.Q2 = Q * Q;
    h.aq = h.a2 + h.Q2;
    h.M2 = 2.0 * M;
    return h;
}

// Terms of the metric that depend on theta only.
struct ThetaTerms {
    double s2, c2, w;          // sin^2, cos^2, a^2 sin^2
};

GR_HD ThetaTerms theta_terms_sc(const Hole& H, double s, double c) {
    ThetaTerms T;
    T.s2 = s * s;
    T.c2 = c * c;
    T.w = H.a2 * T.s2;
    return T;
}

GR_HD ThetaTerms theta_terms(const Hole& H, double theta) {
    double s, c;
    sincos_def(theta, s, c);
    return theta_terms_sc(H, s, c);
}

// Terms that depend on r only.
struct RadialTerms {
    double r2, rara, Delta, aF, DD;   // r^2, (r^2+a^2)^2, Delta, a(2Mr - Q^2), Delta^2
};

GR_HD RadialTerms radial_terms(const Hole& H, double r) {
    RadialTerms R;
    R.r2 = r * r;
    const double ra = R.r2 + H.a2;
    R.rara = ra * ra;
    R.Delta = fma(r, r - H.M2, H.aq);
    R.aF = H.a * fma(H.M2, r, -H.Q2);
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

// rho2 Delta at (r-terms, theta-terms).
GR_HD double rho2_delta(const Hole& H, const RadialTerms& R, const ThetaTerms& T) {
    return fma(H.a2, T.c2, R.r2) * R.Delta;
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

// ----------------------------------------------------------------- camera
// Frame constants of the pinhole camera (host side, once per frame):
// half-extents tan(fov/2) and tan(fov/2) H/W, the orthonormal-frame scale
// factors sqrt(g_rr), sqrt(g_thth), sqrt(g_phph) of the covariant metric, and
// the inverse metric at the camera.
struct Camera {
    double r0, th0, ph0;
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
    const ThetaTerms T = theta_terms(Hh, th0);
    const RadialTerms R = radial_terms(Hh, r0);
    const double rho2 = fma(Hh.a2, T.c2, R.r2);
    const double Sigma2 = fma(-T.w, R.Delta, R.rara);
    C.er = sqrt(rho2 / R.Delta);                 // sqrt(g_rr)
    C.eth = sqrt(rho2);                          // sqrt(g_thth)
    C.eph = sqrt((Sigma2 * T.s2) / rho2);        // sqrt(g_phph)
    C.g = inverse_metric(Hh, R, T);
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
