/*
 * CPU reference ("oracle") for backward null-geodesic ray tracing around a
 * Kerr-Newman black hole in Boyer-Lindquist coordinates, and around the
 * quadrupole Manko-Novikov spacetime (paper Sec. 2.2.3).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this file;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code with the HIP implementation.
 *
 * What it computes (paper: Sec. 2.1 "The Equation of Motion", eq. hamGeodesic,
 * Appendix A "The Legendre Transform for Pseudo-Riemannian geodesics";
 * Sec. 3.1.2 "Runge Kutta Integrators"; Sec. 3.3 "Raytracing"; the appendix
 * listing "Code for propagation of rays"):
 *
 *   H(q,p) = 1/2 g^{mu nu}(r,theta) p_mu p_nu,
 *   dq^mu/dtau = g^{mu nu} p_nu,
 *   dp_mu/dtau = -1/2 d_mu g^{nu sigma} p_nu p_sigma,
 *
 * integrated with classical RK4 whose step h = dt / |dq^t/dtau| is fixed for
 * the whole step from the first stage, so that coordinate time advances by
 * about dt per step (or, on request, with explicit Euler and the same h,
 * Sec. 3.1.1).  Optionally a solid ring around the equator stops the rays
 * that enter it (Sec. 3.3.2), and the redshift of its light is computed from
 * the end states (Sec. 3.3.3, see redshift_rays).  d_r g and d_theta g are one-sided forward differences
 * with step eps; the t and phi derivatives vanish (stationary, axisymmetric),
 * so p_t and p_phi never change.  A ray stops when r exceeds escape_factor
 * times its starting radius (escape), else when |dq^t/dtau| exceeds
 * horizon_norm (step collapse at the horizon), else when its state is no
 * longer finite, else after max_steps updates.
 *
 * Everything is IEEE binary64.  Build with -O2 -ffp-contract=off
 * -fno-fast-math: every fused multiply-add below is an explicit fma() and no
 * other product is fused.  sin and cos are evaluated from their definition
 * (reduction by multiples of pi/2, then the Taylor series with coefficients
 * 1/n!, see trig_sincos) rather than taken from the C library: the forward
 * difference divides rounding noise by eps, so a one-ulp change anywhere in a
 * ray's state moves its end angles by ~1e-9 rad, and a reproducible result
 * needs every operation to be defined.  The C library's sin/cos can be
 * selected instead (trig_mode 1) to show that the physics does not depend
 * on that choice.
 *
 * Parity status: pinned (flat space, Schwarzschild critical impact parameter
 * and deflection integral, Kerr/Kerr-Newman capture by the radial potential,
 * conserved p_t, p_phi, H and Carter constant, mirror symmetries; for
 * Manko-Novikov: the Kerr limit q = 0, vacuum field equations, asymptotic
 * flatness, the far-field quadrupole, equatorial symmetry, H along rays;
 * the ring: Keplerian orbits, closed-form redshifts, flat-space hits).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { FLAG_TIMEOUT = 0, FLAG_ESCAPE = 1, FLAG_HORIZON = 2, FLAG_INVALID = 3, FLAG_DISK = 4 };

/* Constants of a Manko-Novikov spacetime (mass M, spin S, quadrupole
 * deviation q; see mn_inverse_metric). */
typedef struct {
    double M, alpha, k, beta;
    double ik;                   /* 1/k */
    double k2;                   /* k^2 */
    double twok;                 /* 2k */
    double om0;                  /* 4 k alpha / (1 - alpha^2) */
    double iw2;                  /* 1 / (1 - alpha^2)^2 */
} mn_consts;

enum { METRIC_KN = 0, METRIC_MN = 1 };

typedef struct {
    double M, a, Q;              /* mass, spin length a = J/M, charge (G=c=1) */
    double dt, eps;              /* coordinate-time step, finite-difference step */
    double horizon_norm;         /* stop when |dq^t/dtau| exceeds this */
    double escape_factor;        /* stop when r > escape_factor * r_start */
    int max_steps;
    int trig_mode;               /* 0: trig_sincos below; 1: C library sin/cos */
    int kind;                    /* METRIC_KN or METRIC_MN */
    int method;                  /* 0: RK4 (Sec. 3.1.2); 1: explicit Euler (Sec. 3.1.1);
                                    2: RK4 with coordinate time as the parameter */
    /* solid equatorial ring (Sec. 3.3.2, 3.3.3): a ray stops when a step ends
     * with disk_r_in <= r <= disk_r_out and |theta - pi/2| <= disk_dth;
     * off when disk_dth <= 0 */
    double disk_r_in, disk_r_out, disk_dth;
    mn_consts mn;                /* METRIC_MN only */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* sin and cos from their definitions.
 *   x = k pi/2 + r with k the integer nearest to x (2/pi) and |r| <= pi/4;
 *   pi/2 is split as PIO2_HI + PIO2_LO (PIO2_HI = fl(pi/2)) so that
 *   x - k PIO2_HI is exact in one fma for moderate |x|.
 *   sin r = r + r z (S1 + z (S2 + ... + z S8)),  S_n = (-1)^n / (2n+1)!
 *   cos r = 1 + z (C1 + z (C2 + ... + z C8)),    C_n = (-1)^n / (2n)!
 *   with z = r^2 (truncation error below 1e-18 on |r| <= pi/4).
 *   Quadrant k mod 4 = 0, 1, 2, 3 maps (sin x, cos x) to (s, c), (c, -s),
 *   (-s, -c), (-c, s) of the reduced pair (s, c).
 * Each coefficient is 1/m! rounded once (m! is exact in binary64 for m <= 18). */
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;   /* fl(2/pi) */
static const double PIO2_HI = 0x1.921fb54442d18p+0;       /* fl(pi/2) */
static const double PIO2_LO = 0x1.1a62633145c07p-54;      /* fl(pi/2 - PIO2_HI) */

static double SIN_C[9], COS_C[9];                          /* index n = 1..8 */
static pthread_once_t trig_once = PTHREAD_ONCE_INIT;

static void exp_init(void);

static void trig_init(void)
{
    exp_init();
    double fact = 1.0;                                     /* m! */
    for (int m = 1; m <= 17; ++m) {
        fact *= (double)m;
        const double sign = ((m / 2) % 2) ? -1.0 : 1.0;    /* (-1)^n, n = floor(m/2) */
        if (m % 2) SIN_C[m / 2] = sign * (1.0 / fact);     /* m = 2n+1 */
        else       COS_C[m / 2] = sign * (1.0 / fact);     /* m = 2n   */
    }
}

static void trig_sincos(double x, double *s_out, double *c_out)
{
    const double k = rint(x * TWO_OVER_PI);
    double r = fma(-k, PIO2_HI, x);
    r = fma(-k, PIO2_LO, r);
    const double z = r * r;
    double ps = SIN_C[8], pc = COS_C[8];
    for (int n = 7; n >= 1; --n) {
        ps = fma(ps, z, SIN_C[n]);
        pc = fma(pc, z, COS_C[n]);
    }
    const double sr = fma(r * z, ps, r);
    const double cr = fma(z, pc, 1.0);
    const double quad = k - 4.0 * floor(0.25 * k);         /* k mod 4 */
    const int swap = (quad == 1.0) || (quad == 3.0);
    double s = swap ? cr : sr, c = swap ? sr : cr;
    if (quad >= 2.0) s = -s;
    if (quad == 1.0 || quad == 2.0) c = -c;
    *s_out = s;
    *c_out = c;
}

static void sincos_mode(int mode, double x, double *s, double *c)
{
    if (mode == 1) {
        *s = sin(x);
        *c = cos(x);
    } else {
        trig_sincos(x, s, c);               /* tables set by make_params */
    }
}

/* Rotation of the pair (s, c) = (sin x, cos x) by an angle d, giving
 * (sin(x + d), cos(x + d)) by the angle-addition identity:
 *   sin(x + d) = s + (c sin d + s (cos d - 1)),
 *   cos(x + d) = c + (-s sin d + c (cos d - 1)).
 * sin d and cos d - 1 are formed for u = d / 2^m, with m the smallest number
 * of halvings that brings |u| to 1/32 or below (at most 64), from the Taylor
 * series u + u^3 (S1 + u^2 (S2 + u^2 S3)) and u^2 (C1 + u^2 (C2 + u^2 C3))
 * (S_n, C_n as above; the next terms are below 8e-20 and 2.3e-17 for
 * |u| <= 1/32, the latter entering the result multiplied by s or c: at most
 * a fifth of its ulp), and then doubled m times:
 * sin 2u = 2 sin u (1 + (cos u - 1)), cos 2u - 1 = -2 sin^2 u.
 * The results are formed by two fma each, s (1 + (cos d - 1)) first and then
 * the sin d term.  The twin form carries sin/cos of theta along a
 * Kerr-Newman RK4 ray this way instead of evaluating them at every stage
 * point. */
static long g_halved_rotations = 0;       /* rotations that needed halving (test statistics) */

static void rotate_pair(double s, double c, double d, double *s_out, double *c_out)
{
    double u = d;
    int m = 0;
    while (m < 64 && fabs(u) > 0.03125) {
        u *= 0.5;
        ++m;
    }
    if (m > 0) __atomic_fetch_add(&g_halved_rotations, 1, __ATOMIC_RELAXED);
    const double z = u * u;
    double ps = SIN_C[3], pc = COS_C[3];
    for (int n = 2; n >= 1; --n) {
        ps = fma(ps, z, SIN_C[n]);
        pc = fma(pc, z, COS_C[n]);
    }
    double sd = fma(u * z, ps, u);
    double cm1 = z * pc;
    for (int i = 0; i < m; ++i) {
        const double s2 = 2.0 * fma(sd, cm1, sd);
        cm1 = -2.0 * (sd * sd);
        sd = s2;
    }
    *s_out = fma(c, sd, fma(s, cm1, s));      /* s cos d, then + c sin d */
    *c_out = fma(-s, sd, fma(c, cm1, c));     /* c cos d, then - s sin d */
}

/* ------------------------------------------------------------------------ */
/* exp from its definition (the Manko-Novikov metric needs it; as with sin and
 * cos, a library exp would make the forward differences irreproducible).
 *   x = k ln2 + r with k the integer nearest to x / ln2, |r| <= ln2 / 2;
 *   ln2 is split as LN2_HI + LN2_LO (LN2_HI = fl(ln2)), r = (x - k LN2_HI) -
 *   k LN2_LO in two fma;
 *   exp r = sum_{n=0}^{13} r^n / n!  (Horner in fma; truncation below 5e-18
 *   relative on |r| <= ln2/2), then exp x = 2^k exp r (exact scaling).
 * Overflow gives +inf, x < -746 gives 0, NaN stays NaN. */
static const double LOG2E = 0x1.71547652b82fep+0;         /* fl(1/ln2) */
static const double LN2_HI = 0x1.62e42fefa39efp-1;        /* fl(ln2) */
static const double LN2_LO = 0x1.abc9e3b39803fp-56;       /* fl(ln2 - LN2_HI) */
static double EXP_C[14];                                   /* 1/n!, n = 0..13 */

static void exp_init(void)
{
    double fact = 1.0;
    EXP_C[0] = 1.0;
    for (int n = 1; n <= 13; ++n) {
        fact *= (double)n;
        EXP_C[n] = 1.0 / fact;
    }
}

static double exp_def(double x)
{
    if (x != x) return x;
    if (x > 710.0) return INFINITY;
    if (x < -746.0) return 0.0;
    const double k = rint(x * LOG2E);
    double r = fma(-k, LN2_HI, x);
    r = fma(-k, LN2_LO, r);
    double p = EXP_C[13];
    for (int n = 12; n >= 0; --n) p = fma(p, r, EXP_C[n]);
    return ldexp(p, (int)k);
}

/* ------------------------------------------------------------------------ */
/* Inverse Manko-Novikov metric (paper Sec. 2.2.3, the quadrupole member of
 * the family; the inverse components as in the appendix listing's
 * metricAtPoint).  In Boyer-Lindquist-like coordinates the line element is
 *   ds^2 = -f (dt - omega dphi)^2
 *          + f^{-1} [ e^{2 gamma} rho^2 (dr^2 / Delta + dtheta^2)
 *                     + Delta sin^2(theta) dphi^2 ],
 *   rho^2 = (r - M)^2 - k^2 cos^2(theta) = k^2 (x^2 - y^2),
 *   Delta = (r - M)^2 - k^2             = k^2 (x^2 - 1),
 * with prolate spheroidal x = (r - M)/k, y = cos(theta), and
 *   alpha = (-M + sqrt(M^2 - (S/M)^2)) / (S/M),  k = M (1 - alpha^2)/(1 + alpha^2),
 *   beta = q M^3 / k^3,  R = sqrt(x^2 + y^2 - 1),  P_l = P_l(x y / R),
 *   a_ = -alpha exp(-2 beta (-1 + sum_{l=0}^2 (x - y) P_l / R^{l+1})),
 *   b_ =  alpha exp( 2 beta ( 1 + sum_{l=0}^2 (-1)^{3-l} (x + y) P_l / R^{l+1})),
 *   A = (x^2 - 1)(1 + a_ b_)^2 - (1 - y^2)(b_ - a_)^2,
 *   B = [x + 1 + (x - 1) a_ b_]^2 + [(1 + y) a_ + (1 - y) b_]^2,
 *   C = (x^2 - 1)(1 + a_ b_)[b_ - a_ - y (a_ + b_)]
 *       + (1 - y^2)(b_ - a_)[1 + a_ b_ + x (1 - a_ b_)],
 *   psi = beta P_2 / R^3,   f = e^{2 psi} A / B,
 *   omega = 2 k e^{-2 psi} C / A - 4 k alpha / (1 - alpha^2),
 *   gamma' = ln sqrt((x^2 - 1)/(x^2 - y^2)) + 3 beta^2 (P_3^2 - P_2^2) / (2 R^6)
 *            + beta (-2 + sum_{l=0}^2 [x - y + (-1)^{2-l} (x + y)] P_l / R^{l+1}),
 *   e^{2 gamma} = e^{2 gamma'} A / ((x^2 - 1)(1 - alpha^2)^2).
 * Readings of the printed formulas (garbled in places): the first term of
 * the line element is squared, the theta term is e^{2 gamma} rho^2 dtheta^2 / f,
 * B is a sum of two squares, and the beta term of gamma' is beta (-2 + sum):
 * these are the forms for which q = 0 gives Kerr and the metric is a vacuum
 * solution (both are tested), and with them gamma' vanishes at infinity.
 * The logarithm cancels: e^{2 gamma} rho^2 = k^2 e^{2 G} A / (1 - alpha^2)^2
 * with G = gamma' - ln sqrt((x^2 - 1)/(x^2 - y^2)).  Inverse components
 * (D = Delta sin^2 theta):
 *   g^{tt} = -1/f + f omega^2 / D,  g^{t phi} = f omega / D,
 *   g^{rr} = f Delta / (e^{2 gamma} rho^2),  g^{theta theta} = f / (e^{2 gamma} rho^2),
 *   g^{phi phi} = f / D.
 * y = cos(theta) and s2 = sin^2(theta) are passed in (the forward difference
 * in theta evaluates them by angle addition). */
static void mn_consts_make(double M, double S, double q, mn_consts *K)
{
    const double chi = S / M;                                  /* a = S/M */
    K->M = M;
    K->alpha = (-M + sqrt(M * M - chi * chi)) / chi;
    const double al2 = K->alpha * K->alpha;
    K->k = M * ((1.0 - al2) / (1.0 + al2));
    K->beta = (q * (M * M * M)) / (K->k * K->k * K->k);
    K->ik = 1.0 / K->k;
    K->k2 = K->k * K->k;
    K->twok = 2.0 * K->k;
    K->om0 = (4.0 * K->k * K->alpha) / (1.0 - al2);
    K->iw2 = 1.0 / ((1.0 - al2) * (1.0 - al2));
}

static void mn_inverse_metric(const mn_consts *K, double r, double y, double s2, double g[5])
{
    const double beta = K->beta;
    const double x = (r - K->M) * K->ik;
    const double x2 = x * x, y2 = y * y;
    const double R = sqrt((x2 + y2) - 1.0);
    const double iR = 1.0 / R;
    const double iR2 = iR * iR, iR3 = iR2 * iR;
    const double u = (x * y) * iR;                             /* argument of P_l */
    const double P1 = u;
    const double P2 = fma(1.5 * u, u, -0.5);                   /* (3u^2 - 1)/2 */
    const double P3 = u * fma(2.5 * u, u, -1.5);               /* (5u^3 - 3u)/2 */
    /* the l = 0..2 sums: L1 = sum P_l / R^{l+1}, L2 = sum (-1)^l P_l / R^{l+1} */
    const double L1 = fma(P2, iR3, fma(P1, iR2, iR));
    const double L2 = fma(P2, iR3, fma(-P1, iR2, iR));
    const double Sa = (x - y) * L1;                            /* sum (x - y) P_l / R^{l+1} */
    const double Sb = -((x + y) * L2);                         /* sum (-1)^{3-l} (x + y) ... */
    const double Sg = fma(x - y, L1, (x + y) * L2);            /* sum [x - y + (-1)^l (x + y)] ... */
    const double ea = exp_def((-2.0 * beta) * (Sa - 1.0));
    const double eb = exp_def((2.0 * beta) * (1.0 + Sb));
    const double am = -(K->alpha * ea);                        /* a_ */
    const double bm = K->alpha * eb;                           /* b_ */
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
    const double f = fA / B;
    const double omega = (K->twok * C) / fA - K->om0;
    const double e2g_rho2 = ((K->k2 * exp_def(2.0 * G)) * A) * K->iw2;
    const double Delta = K->k2 * xm1;
    const double iD = 1.0 / (Delta * s2);
    const double ie = 1.0 / e2g_rho2;
    const double fo = f * omega;
    g[0] = fma(fo * omega, iD, -(1.0 / f));                   /* g^{tt} */
    g[1] = fo * iD;                                            /* g^{t phi} */
    g[2] = (f * Delta) * ie;                                   /* g^{rr} */
    g[3] = f * ie;                                             /* g^{theta theta} */
    g[4] = f * iD;                                             /* g^{phi phi} */
}

/* ------------------------------------------------------------------------ */
/* Inverse Kerr-Newman metric at (r, theta).  Paper Sec. 2.2.2 "The Kerr
 * Metric" (Boyer-Lindquist coordinates in Carroll's convention; the printed
 * covariant metric has typos, the textbook form is used) extended by the
 * charge term Q^2 in Delta.  Five independent components:
 *   g[0] = g^{tt}, g[1] = g^{t phi}, g[2] = g^{rr}, g[3] = g^{theta theta},
 *   g[4] = g^{phi phi}.
 *
 *   Delta  = r^2 - 2 M r + a^2 + Q^2
 *   rho^2  = r^2 + a^2 cos^2 theta
 *   Sigma2 = (r^2 + a^2)^2 - a^2 Delta sin^2 theta
 *   g^{tt}   = -Sigma2 / (rho^2 Delta)
 *   g^{tphi} = -a (2 M r - Q^2) / (rho^2 Delta)
 *   g^{rr}   = Delta / rho^2
 *   g^{thth} = 1 / rho^2
 *   g^{phph} = (Delta - a^2 sin^2 theta) / (rho^2 Delta sin^2 theta)
 *
 * The sequence of roundings is fixed (it matters: the forward difference
 * divides rounding noise by eps).  sin^2 is passed in so that the same
 * rounded value serves every evaluation at one theta; rho^2 is formed from it
 * as (r^2 + a^2) - a^2 sin^2 (cos^2 = 1 - sin^2), which outside a horizon
 * (r >= a) keeps it to a few ulp.  The components
 * share the reciprocals inv = 1/(rho^2 Delta) and is = inv / sin^2 (see
 * metric_recips for how they are formed). */
/* a (2 M r - Q^2), with a 2M and a Q^2 rounded once each. */
static double a_term(const oracle_params *P, double r)
{
    return fma(P->a * (2.0 * P->M), r, -(P->a * (P->Q * P->Q)));
}

static void metric_from(const oracle_params *P, double r, double s2, double inv, double is,
                        double g[5])
{
    const double a2 = P->a * P->a;
    const double r2 = r * r;
    const double ra = r2 + a2;                                 /* r^2 + a^2 */
    const double Delta = fma(r, r - 2.0 * P->M, a2 + P->Q * P->Q);
    const double w = a2 * s2;                                  /* a^2 sin^2 */
    const double Sigma2 = fma(-w, Delta, ra * ra);
    g[0] = -(Sigma2 * inv);
    g[1] = -(a_term(P, r) * inv);
    g[2] = (Delta * Delta) * inv;
    g[3] = Delta * inv;
    g[4] = (Delta - w) * is;
}

/* The differences d[k] = g^{k}(displaced point) - g0[k] of the five
 * components between a displaced point (r, sin^2 = s2, the reciprocals inv
 * and is formed there) and the base point's g0: each displaced component's
 * last product is fused with its subtraction of g0[k] (one fma), so the
 * difference is rounded once and the displaced component itself never is;
 * the other terms are rounded as in metric_from. */
static void metric_diff(const oracle_params *P, double r, double s2, double inv, double is,
                        const double g0[5], double d[5])
{
    const double a2 = P->a * P->a;
    const double r2 = r * r;
    const double ra = r2 + a2;
    const double Delta = fma(r, r - 2.0 * P->M, a2 + P->Q * P->Q);
    const double w = a2 * s2;
    const double Sigma2 = fma(-w, Delta, ra * ra);
    d[0] = fma(-Sigma2, inv, -g0[0]);
    d[1] = fma(-a_term(P, r), inv, -g0[1]);
    d[2] = fma(Delta * Delta, inv, -g0[2]);
    d[3] = fma(Delta, inv, -g0[3]);
    d[4] = fma(Delta - w, is, -g0[4]);
}

/* rho^2 Delta at (r, theta), sin^2 theta = s2. */
static double rho2_delta(const oracle_params *P, double r, double s2)
{
    const double a2 = P->a * P->a;
    const double rho2 = (r * r + a2) - a2 * s2;                /* r^2 + a^2 cos^2 */
    const double Delta = fma(r, r - 2.0 * P->M, a2 + P->Q * P->Q);
    return rho2 * Delta;
}

/* 1/x from y0 = 1/x0 for a nearby x0: two Newton steps y <- y + y (1 - x y).
 * Each squares the relative error e0 = 1 - x y0; for the displacements of the
 * forward differences |e0| is about eps times a logarithmic derivative of
 * rho^2 Delta (below 1e-4 even at the horizon cutoff), so e0^4 is at or below
 * the rounding of the result. */
static double recip_newton(double x, double y0)
{
    double e = fma(-x, y0, 1.0);
    const double y = fma(y0, e, y0);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

/* Three Newton steps: relative error e0^8 plus rounding. */
static double recip_newton3(double x, double y0)
{
    double e = fma(-x, y0, 1.0);
    double y = fma(y0, e, y0);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

/* Largest |1 - x y0| from which the theta-displaced point's reciprocal is
 * refined (three Newton steps: e0^8 <= 2^-64, within about an ulp) rather
 * than divided: 2^-8.  Over the theta displacement rho^2 Delta sin^2 moves by
 * the factor 1 - 2 eps cot(theta) + O(eps), so only points within about
 * 5e5 eps of the polar axis divide. */
#define NEWTON_SEED_MAX 0x1p-8

/* Full inverse metric at one point: is = 1/(rho^2 Delta sin^2) divided,
 * inv = is sin^2. */
static void inverse_metric(const oracle_params *P, double r, double s2, double g[5])
{
    const double is = 1.0 / (rho2_delta(P, r, s2) * s2);
    metric_from(P, r, s2, is * s2, is, g);
}

/* g^{mu nu} at (r, theta) from the angle itself (the listing's metricAtPoint). */
static void metric_at_point(const oracle_params *P, double r, double theta, double g[5])
{
    double s, c;
    sincos_mode(P->trig_mode, theta, &s, &c);
    if (P->kind == METRIC_MN)
        mn_inverse_metric(&P->mn, r, c, s * s, g);
    else
        inverse_metric(P, r, s * s, g);
}

/* Right-hand side of Hamilton's equations at one RK4 stage point.
 * Paper eq. hamGeodesic with the factor 1/2 of Appendix A; derivatives by
 * forward differences of step eps as in the listing: the metric (Kerr-Newman
 * or Manko-Novikov) at (r,theta), (r+eps,theta) and (r,theta+eps), given s and c,
 * the sine and cosine of the point's theta.  sin (and, for Manko-Novikov,
 * cos) at theta+eps are the angle-addition identity applied to those at theta
 * and at eps (for eps = 1e-8, cos eps rounds to 1 and sin eps to eps), so the
 * theta step is eps itself; the Kerr-Newman terms need sin^2 only.  For Kerr-Newman each displaced component is formed together with
 * its difference from the base point's (metric_diff, one rounding for the
 * difference); the Manko-Novikov metric is evaluated in full at the three
 * points and subtracted.  The contraction sums the differences of the five
 * independent components times p_nu p_sigma in the order tt, t-phi (weight
 * 2 p_t p_phi), rr, theta-theta, phi-phi, then scales once by -1/(2 eps). */
/* -1/(2 eps): the scaling of the contracted differences into p-dot. */
static double fd_scale(const oracle_params *P)
{
    return -0.5 * (1.0 / P->eps);
}

static void rhs_core(const oracle_params *P, const double eps_sc[2], double r, double s,
                     double c, double pt, double pr, double pth, double pph, double qdot[4],
                     double pdot[2], int raw, double gtp[3])
{
    double g[5], dr[5], dth[5];        /* base metric; differences to the displaced points */
    const double se = fma(c, eps_sc[0], s * eps_sc[1]);      /* sin(theta + eps) */
    const double ce = fma(-s, eps_sc[0], c * eps_sc[1]);     /* cos(theta + eps) */
    const double s2 = s * s, se2 = se * se;
    /* reciprocals: is = 1/(rho^2 Delta sin^2) divided at (r, theta),
     * inv = is sin^2; at (r + eps, theta), where only rho^2 Delta moves, by a
     * factor 1 + O(eps), is is refined from the base point's; at
     * (r, theta + eps) by three Newton steps where the refinement starts
     * within NEWTON_SEED_MAX, divided where it does not (within about 5e5 eps
     * of the axis, where sin^2 changes by a large factor over eps) */
    if (P->kind == METRIC_MN) {
        /* full evaluations at the three points, then the differences */
        double gr[5], gth[5];
        mn_inverse_metric(&P->mn, r, c, s2, g);
        mn_inverse_metric(&P->mn, r + P->eps, c, s2, gr);
        mn_inverse_metric(&P->mn, r, ce, se2, gth);
        for (int k = 0; k < 5; ++k) {
            dr[k] = gr[k] - g[k];
            dth[k] = gth[k] - g[k];
        }
    } else {
        const double is = 1.0 / (rho2_delta(P, r, s2) * s2);
        const double inv = is * s2;
        const double is_r = recip_newton(rho2_delta(P, r + P->eps, s2) * s2, is);
        const double xt = rho2_delta(P, r, se2) * se2;
        const double is_t = fabs(fma(-xt, is, 1.0)) <= NEWTON_SEED_MAX ? recip_newton3(xt, is)
                                                                       : 1.0 / xt;
        metric_from(P, r, s2, inv, is, g);
        metric_diff(P, r + P->eps, s2, is_r * s2, is_r, g, dr);
        metric_diff(P, r, se2, is_t * se2, is_t, g, dth);
    }

    /* weights p_nu p_sigma of the five independent components */
    const double wtt = pt * pt, wtp = (2.0 * pt) * pph, wpp = pph * pph;
    const double wrr = pr * pr, wth = pth * pth;
    const double scale = fd_scale(P);

    double acc = dr[0] * wtt;
    acc = fma(dr[1], wtp, acc);
    acc = fma(dr[2], wrr, acc);
    acc = fma(dr[3], wth, acc);
    acc = fma(dr[4], wpp, acc);
    pdot[0] = raw ? acc : acc * scale;                         /* dp_r/dtau */

    acc = dth[0] * wtt;
    acc = fma(dth[1], wtp, acc);
    acc = fma(dth[2], wrr, acc);
    acc = fma(dth[3], wth, acc);
    acc = fma(dth[4], wpp, acc);
    pdot[1] = raw ? acc : acc * scale;                         /* dp_theta/dtau */

    qdot[0] = fma(g[0], pt, g[1] * pph);                       /* dt/dtau */
    qdot[1] = g[2] * pr;                                       /* dr/dtau */
    qdot[2] = g[3] * pth;                                      /* dtheta/dtau */
    qdot[3] = fma(g[1], pt, g[4] * pph);                       /* dphi/dtau */
    if (gtp) {                                                 /* g^tt, g^tphi, g^phph */
        gtp[0] = g[0];
        gtp[1] = g[1];
        gtp[2] = g[4];
    }
}

/* The right-hand side with p-dot scaled, and unscaled (the contracted sums
 * alone: the carried Kerr-Newman RK4 folds -1/(2 eps) into its step sizes;
 * it also takes g^tt, g^tphi, g^phph, of which dt/dtau and dphi/dtau are
 * linear combinations with the ray's constant p_t, p_phi). */
static void hamilton_rhs_sc(const oracle_params *P, const double eps_sc[2], double r,
                            double s, double c, double pt, double pr, double pth, double pph,
                            double qdot[4], double pdot[2])
{
    rhs_core(P, eps_sc, r, s, c, pt, pr, pth, pph, qdot, pdot, 0, NULL);
}

static void hamilton_rhs_sc_raw(const oracle_params *P, const double eps_sc[2], double r,
                                double s, double c, double pt, double pr, double pth,
                                double pph, double qdot[4], double pdot[2], double gtp[3])
{
    rhs_core(P, eps_sc, r, s, c, pt, pr, pth, pph, qdot, pdot, 1, gtp);
}

/* The same at (r, theta), sin and cos of theta from the stated definition. */
static void hamilton_rhs(const oracle_params *P, const double eps_sc[2], double r,
                         double theta, double pt, double pr, double pth, double pph,
                         double qdot[4], double pdot[2])
{
    double s, c;
    sincos_mode(P->trig_mode, theta, &s, &c);
    hamilton_rhs_sc(P, eps_sc, r, s, c, pt, pr, pth, pph, qdot, pdot);
}

static int in_disk(const oracle_params *P, const double q[4])
{
    return P->disk_dth > 0.0 && q[1] >= P->disk_r_in && q[1] <= P->disk_r_out &&
           fabs(q[2] - PIO2_HI) <= P->disk_dth;                 /* PIO2_HI = fl(pi/2) */
}

static int all_finite(const double q[4], double pr, double pth)
{
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3]) &&
           isfinite(pr) && isfinite(pth);
}

/* One stage of the coordinate-time RK4 at r and the stage angle theta0 +
 * coef k_theta, into (kq, kp) multiplied by w = 1/|dt/dtau| there; returns
 * |dt/dtau|.  Manko-Novikov takes the angle fma(coef, k_theta, theta0);
 * Kerr-Newman the carried pair (sn, cs) of theta0 rotated by coef k_theta
 * (the stage at theta0 itself takes the pair as it is). */
static double rk4t_stage(const oracle_params *P, const double eps_sc[2], double r, double th0,
                         double sn, double cs, double coef, double kth, double pt, double pr,
                         double pth, double pph, double kq[4], double kp[2])
{
    if (P->kind == METRIC_MN) {
        hamilton_rhs(P, eps_sc, r, fma(coef, kth, th0), pt, pr, pth, pph, kq, kp);
    } else if (coef == 0.0) {
        hamilton_rhs_sc(P, eps_sc, r, sn, cs, pt, pr, pth, pph, kq, kp);
    } else {
        double s2, c2;
        rotate_pair(sn, cs, coef * kth, &s2, &c2);
        hamilton_rhs_sc(P, eps_sc, r, s2, c2, pt, pr, pth, pph, kq, kp);
    }
    const double nu = fabs(kq[0]);
    const double w = 1.0 / nu;
    for (int m = 0; m < 4; ++m) kq[m] = kq[m] * w;
    kp[0] = kp[0] * w;
    kp[1] = kp[1] * w;
    return nu;
}

/* Integrate one ray.  q = (t, r, theta, phi), p = (p_t, p_r, p_theta, p_phi)
 * are updated in place; returns the flag, *nsteps = updates taken.
 * Paper: listing loop body (stages K1..K4, update, exit tests), Sec. 3.1.2
 * (RK4 weights 1/6, 2/6, 2/6, 1/6), Sec. 3.3.2 "Propagation". */
int oracle_integrate(const oracle_params *P, double q[4], double p[4], int *nsteps)
{
    double eps_sc[2];                                          /* sin eps, cos eps */
    sincos_mode(P->trig_mode, P->eps, &eps_sc[0], &eps_sc[1]);
    const double r_esc = P->escape_factor * q[1];
    const double pt = p[0], pph = p[3];
    double pr = p[1], pth = p[2];
    int flag = FLAG_TIMEOUT, s = 0;
    double sn, cs;                                             /* sin, cos of theta, carried */
    sincos_mode(P->trig_mode, q[2], &sn, &cs);
    *nsteps = 0;
    if (!(all_finite(q, pr, pth) && isfinite(pt) && isfinite(pph)))
        return FLAG_INVALID;

    for (s = 1; s <= P->max_steps; ++s) {
        double k1q[4], k1p[2], k2q[4], k2p[2], k3q[4], k3p[2], k4q[4], k4p[2];
        if (P->method == 1) {
            /* explicit Euler: x += h f(x), h = dt / |dt/dtau| from f(x); on
             * Kerr-Newman f from the carried pair, which then turns by the
             * step's increment of theta */
            double nu, h;
            if (P->kind == METRIC_MN) {
                hamilton_rhs(P, eps_sc, q[1], q[2], pt, pr, pth, pph, k1q, k1p);
                nu = fabs(k1q[0]);
                h = P->dt / nu;
            } else {
                double s2, c2;
                hamilton_rhs_sc(P, eps_sc, q[1], sn, cs, pt, pr, pth, pph, k1q, k1p);
                nu = fabs(k1q[0]);
                h = P->dt / nu;
                rotate_pair(sn, cs, h * k1q[2], &s2, &c2);
                sn = s2;
                cs = c2;
            }
            for (int m = 0; m < 4; ++m) q[m] = fma(h, k1q[m], q[m]);
            pr = fma(h, k1p[0], pr);
            pth = fma(h, k1p[1], pth);
            if (in_disk(P, q)) { flag = FLAG_DISK; break; }
            if (q[1] > r_esc) { flag = FLAG_ESCAPE; break; }
            if (nu > P->horizon_norm) { flag = FLAG_HORIZON; break; }
            if (!all_finite(q, pr, pth)) { flag = FLAG_INVALID; break; }
            continue;
        }
        if (P->method == 2) {
            /* RK4 with coordinate time as the parameter (each stage
             * reparametrised): a stage's derivative is multiplied by
             * w = 1/|dt/dtau| at that stage, so every stage moves t at the
             * same rate, and the step is dt itself. */
            const double hh = 0.5 * P->dt;
            const double nu = rk4t_stage(P, eps_sc, q[1], q[2], sn, cs, 0.0, 0.0, pt, pr, pth,
                                         pph, k1q, k1p);
            rk4t_stage(P, eps_sc, fma(hh, k1q[1], q[1]), q[2], sn, cs, hh, k1q[2], pt,
                       fma(hh, k1p[0], pr), fma(hh, k1p[1], pth), pph, k2q, k2p);
            rk4t_stage(P, eps_sc, fma(hh, k2q[1], q[1]), q[2], sn, cs, hh, k2q[2], pt,
                       fma(hh, k2p[0], pr), fma(hh, k2p[1], pth), pph, k3q, k3p);
            rk4t_stage(P, eps_sc, fma(P->dt, k3q[1], q[1]), q[2], sn, cs, P->dt, k3q[2], pt,
                       fma(P->dt, k3p[0], pr), fma(P->dt, k3p[1], pth), pph, k4q, k4p);
            const double h6 = P->dt * (1.0 / 6.0);
            double S[4];
            for (int m = 0; m < 4; ++m) {
                S[m] = ((k1q[m] + 2.0 * k2q[m]) + 2.0 * k3q[m]) + k4q[m];
                q[m] = fma(h6, S[m], q[m]);
            }
            pr = fma(h6, ((k1p[0] + 2.0 * k2p[0]) + 2.0 * k3p[0]) + k4p[0], pr);
            pth = fma(h6, ((k1p[1] + 2.0 * k2p[1]) + 2.0 * k3p[1]) + k4p[1], pth);
            if (P->kind != METRIC_MN) {
                double s2, c2;
                rotate_pair(sn, cs, h6 * S[2], &s2, &c2);  /* the carried pair follows theta */
                sn = s2;
                cs = c2;
            }
            if (in_disk(P, q)) { flag = FLAG_DISK; break; }
            if (q[1] > r_esc) { flag = FLAG_ESCAPE; break; }
            if (nu > P->horizon_norm) { flag = FLAG_HORIZON; break; }
            if (!all_finite(q, pr, pth)) { flag = FLAG_INVALID; break; }
            continue;
        }
        double nu, h;
        double g1[3], g2[3], g3[3], g4[3];     /* Kerr-Newman: g^tt, g^tphi, g^phph per stage */
        const double pscale = fd_scale(P);
        if (P->kind == METRIC_MN) {
            /* K1 at the current point; its dt/dtau fixes the step. */
            hamilton_rhs(P, eps_sc, q[1], q[2], pt, pr, pth, pph, k1q, k1p);
            nu = fabs(k1q[0]);
            h = P->dt / nu;
            const double hh = 0.5 * h;
            /* K2, K3 at half steps, K4 at the full step. */
            hamilton_rhs(P, eps_sc, fma(hh, k1q[1], q[1]), fma(hh, k1q[2], q[2]), pt,
                         fma(hh, k1p[0], pr), fma(hh, k1p[1], pth), pph, k2q, k2p);
            hamilton_rhs(P, eps_sc, fma(hh, k2q[1], q[1]), fma(hh, k2q[2], q[2]), pt,
                         fma(hh, k2p[0], pr), fma(hh, k2p[1], pth), pph, k3q, k3p);
            hamilton_rhs(P, eps_sc, fma(h, k3q[1], q[1]), fma(h, k3q[2], q[2]), pt,
                         fma(h, k3p[0], pr), fma(h, k3p[1], pth), pph, k4q, k4p);
        } else {
            /* Kerr-Newman: theta enters through its sine and cosine only, and
             * the ray carries them; each stage point's pair is the carried
             * pair rotated by that stage's increment of theta.  p-dot comes
             * unscaled and -1/(2 eps) multiplies the momenta's step sizes. */
            double s2, c2;
            hamilton_rhs_sc_raw(P, eps_sc, q[1], sn, cs, pt, pr, pth, pph, k1q, k1p, g1);
            nu = fabs(k1q[0]);
            h = P->dt / nu;
            const double hh = 0.5 * h;
            const double hhs = hh * pscale, hs = h * pscale;
            rotate_pair(sn, cs, hh * k1q[2], &s2, &c2);
            hamilton_rhs_sc_raw(P, eps_sc, fma(hh, k1q[1], q[1]), s2, c2, pt,
                                fma(hhs, k1p[0], pr), fma(hhs, k1p[1], pth), pph, k2q, k2p,
                                g2);
            rotate_pair(sn, cs, hh * k2q[2], &s2, &c2);
            hamilton_rhs_sc_raw(P, eps_sc, fma(hh, k2q[1], q[1]), s2, c2, pt,
                                fma(hhs, k2p[0], pr), fma(hhs, k2p[1], pth), pph, k3q, k3p,
                                g3);
            rotate_pair(sn, cs, h * k3q[2], &s2, &c2);
            hamilton_rhs_sc_raw(P, eps_sc, fma(h, k3q[1], q[1]), s2, c2, pt,
                                fma(hs, k3p[0], pr), fma(hs, k3p[1], pth), pph, k4q, k4p,
                                g4);
        }
        /* x += h/6 (k1 + 2 k2 + 2 k3 + k4) */
        const double h6 = h * (1.0 / 6.0);
        double S[4];
        for (int m = 0; m < 4; ++m)
            S[m] = ((k1q[m] + 2.0 * k2q[m]) + 2.0 * k3q[m]) + k4q[m];
        if (P->kind != METRIC_MN) {
            /* Kerr-Newman: the sums of dt/dtau and dphi/dtau through those of
             * g^tt, g^tphi and g^phph, contracted once with p_t and p_phi */
            double G[3];
            for (int m = 0; m < 3; ++m)
                G[m] = ((g1[m] + 2.0 * g2[m]) + 2.0 * g3[m]) + g4[m];
            S[0] = fma(G[0], pt, G[1] * pph);
            S[3] = fma(G[1], pt, G[2] * pph);
        }
        for (int m = 0; m < 4; ++m)
            q[m] = fma(h6, S[m], q[m]);
        const double h6p = P->kind == METRIC_MN ? h6 : h6 * pscale;   /* see above */
        pr = fma(h6p, ((k1p[0] + 2.0 * k2p[0]) + 2.0 * k3p[0]) + k4p[0], pr);
        pth = fma(h6p, ((k1p[1] + 2.0 * k2p[1]) + 2.0 * k3p[1]) + k4p[1], pth);
        if (P->kind != METRIC_MN) {
            double s2, c2;
            rotate_pair(sn, cs, h6 * S[2], &s2, &c2);     /* the carried pair follows theta */
            sn = s2;
            cs = c2;
        }

        if (in_disk(P, q)) { flag = FLAG_DISK; break; }
        if (q[1] > r_esc) { flag = FLAG_ESCAPE; break; }
        if (nu > P->horizon_norm) { flag = FLAG_HORIZON; break; }
        if (!all_finite(q, pr, pth)) { flag = FLAG_INVALID; break; }
    }
    if (s > P->max_steps) s = P->max_steps;
    p[1] = pr;
    p[2] = pth;
    *nsteps = s;
    return flag;
}

/* ------------------------------------------------------------------------ */
/* Pinhole camera (paper Sec. 3.3.1 "Initial positions"; listing lightlikeT).
 * A static camera at (r0, theta0, phi0) looks toward the hole.  Pixel (i, j),
 * column i from the left and row j from the top, has image-plane coordinates
 *   x = ((2i+1-W)/W) tan(fov/2),  y = ((H-2j-1)/H) tan(fov/2) H/W
 * (fov is the full horizontal angle, square pixels).  Its line-of-sight unit
 * vector in the orthonormal frame (e_r, e_theta, e_phi) of the locally
 * non-rotating observer is n = (-1, -y, x)/sqrt(1 + x^2 + y^2): image right is
 * +phi, image up is -theta.  The spatial covector is p_j = n_j sqrt(g_jj);
 * p_t is the root of H = 0 that makes dt/dtau negative (past-directed, the
 * ray is traced backward), and the whole covector is then scaled so that
 * dt/dtau = -1 at the camera (the normalisation the paper uses for redshift). */
typedef struct {
    double tan_half, tan_half_v;       /* horizontal and vertical half-extent */
    double er, eth, eph;               /* sqrt(g_rr), sqrt(g_thth), sqrt(g_phph) */
    double g[5];                       /* inverse metric at the camera */
} camera_consts;

static void camera_setup(const oracle_params *P, double r0, double th0, double fov,
                         int W, int H, camera_consts *C)
{
    double sf, cf, s, c;
    sincos_mode(P->trig_mode, 0.5 * fov, &sf, &cf);
    C->tan_half = sf / cf;
    C->tan_half_v = (C->tan_half * (double)H) / (double)W;
    sincos_mode(P->trig_mode, th0, &s, &c);
    const double s2 = s * s, c2 = c * c;
    if (P->kind == METRIC_MN) {
        /* covariant g_rr = 1/g^rr, g_thth = 1/g^thth and, from the inverse of
         * the (t, phi) block, g_phph = g^tt / (g^tt g^phph - (g^tphi)^2) */
        mn_inverse_metric(&P->mn, r0, c, s2, C->g);
        C->er = sqrt(1.0 / C->g[2]);
        C->eth = sqrt(1.0 / C->g[3]);
        C->eph = sqrt(C->g[0] / ((C->g[0] * C->g[4]) - (C->g[1] * C->g[1])));
        return;
    }
    const double a2 = P->a * P->a;
    const double r2 = r0 * r0;
    const double ra = r2 + a2;
    const double rho2 = fma(a2, c2, r2);
    const double Delta = fma(r0, r0 - 2.0 * P->M, a2 + P->Q * P->Q);
    const double Sigma2 = fma(-(a2 * s2), Delta, ra * ra);
    /* covariant g_rr = rho^2/Delta, g_thth = rho^2, g_phph = Sigma2 sin^2/rho^2 */
    C->er = sqrt(rho2 / Delta);
    C->eth = sqrt(rho2);
    C->eph = sqrt((Sigma2 * s2) / rho2);
    inverse_metric(P, r0, s2, C->g);
}

static void camera_ray(const camera_consts *C, int W, int H, int64_t pix,
                       double r0, double th0, double ph0, double q[4], double p[4])
{
    const int64_t i = pix % W, j = pix / W;
    /* (2i+1-W)/W is exactly antisymmetric under i -> W-1-i (integer numerator) */
    const double x = ((double)(2 * i + 1 - W) / (double)W) * C->tan_half;
    const double y = ((double)(H - 2 * j - 1) / (double)H) * C->tan_half_v;
    const double inv_n = 1.0 / sqrt(1.0 + x * x + y * y);
    const double pr = (-inv_n) * C->er;
    const double pth = (-y * inv_n) * C->eth;
    const double pph = (x * inv_n) * C->eph;
    /* null condition g^tt p_t^2 + 2 g^tph p_t p_ph + S = 0 */
    const double S = C->g[2] * (pr * pr) + C->g[3] * (pth * pth) + C->g[4] * (pph * pph);
    const double b = C->g[1] * pph;
    const double D = b * b - C->g[0] * S;
    const double sD = sqrt(D);
    const double pt = (-b - sD) / C->g[0];     /* gives dt/dtau = -sqrt(D) */
    const double k = 1.0 / sD;                 /* rescale to dt/dtau = -1 */
    q[0] = 0.0; q[1] = r0; q[2] = th0; q[3] = ph0;
    p[0] = pt * k; p[1] = pr * k; p[2] = pth * k; p[3] = pph * k;
}

/* ------------------------------------------------------------------------ */
/* Multithreaded drivers: one ray per work item, dynamic chunks of rays. */

typedef struct {
    const oracle_params *P;
    /* frame mode */
    const camera_consts *C;
    double r0, th0, ph0;
    int W, H;
    const int64_t *pixels;            /* NULL: ray k is pixel k */
    /* ray-list mode (C == NULL): initial states, 8 doubles per ray */
    const double *init;
    int64_t n;
    /* outputs, any may be NULL except flag */
    double *t, *r, *th, *ph, *pr, *pth, *p0;
    int8_t *flag;
    int32_t *steps;
    int64_t next;                     /* shared work counter */
} job;

static void run_one(job *J, int64_t k)
{
    double q[4], p[4];
    if (J->C) {
        const int64_t pix = J->pixels ? J->pixels[k] : k;
        camera_ray(J->C, J->W, J->H, pix, J->r0, J->th0, J->ph0, q, p);
    } else {
        memcpy(q, J->init + 8 * k, 4 * sizeof(double));
        memcpy(p, J->init + 8 * k + 4, 4 * sizeof(double));
    }
    if (J->p0) memcpy(J->p0 + 4 * k, p, 4 * sizeof(double));
    int ns = 0;
    const int f = oracle_integrate(J->P, q, p, &ns);
    if (J->t) J->t[k] = q[0];
    if (J->r) J->r[k] = q[1];
    if (J->th) J->th[k] = q[2];
    if (J->ph) J->ph[k] = q[3];
    if (J->pr) J->pr[k] = p[1];
    if (J->pth) J->pth[k] = p[2];
    J->flag[k] = (int8_t)f;
    if (J->steps) J->steps[k] = ns;
}

static void *worker(void *arg)
{
    job *J = (job *)arg;
    const int64_t chunk = 8;
    for (;;) {
        const int64_t b = __atomic_fetch_add(&J->next, chunk, __ATOMIC_RELAXED);
        if (b >= J->n) break;
        const int64_t e = b + chunk < J->n ? b + chunk : J->n;
        for (int64_t k = b; k < e; ++k) run_one(J, k);
    }
    return NULL;
}

static void run_job(job *J, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t tid[256];
    int started = 0;
    J->next = 0;
    for (int i = 1; i < nthreads; ++i)
        if (pthread_create(&tid[started], NULL, worker, J) == 0) ++started;
    worker(J);
    for (int i = 0; i < started; ++i) pthread_join(tid[i], NULL);
}

static int g_trig_mode = 0;

/* Select the sin/cos used by later calls: 0 (default) the definition above,
 * 1 the C library. */
void oracle_set_trig_mode(int mode) { g_trig_mode = mode; }

/* Accuracy checks of the sin/cos definition: n values in, 2n out (s, c). */
void oracle_sincos(const double *x, int64_t n, double *sc)
{
    pthread_once(&trig_once, trig_init);
    for (int64_t k = 0; k < n; ++k) trig_sincos(x[k], sc + 2 * k, sc + 2 * k + 1);
}

/* rotate_pair on n triples (x_sin, x_cos, d): out[2k], out[2k+1]. */
void oracle_rotate(const double *in3, int64_t n, double *out2)
{
    pthread_once(&trig_once, trig_init);
    for (int64_t k = 0; k < n; ++k)
        rotate_pair(in3[3 * k], in3[3 * k + 1], in3[3 * k + 2], &out2[2 * k], &out2[2 * k + 1]);
}

/* Number of rotations so far that needed halving (reset = 1 clears it). */
long oracle_halved_rotations(int reset)
{
    const long v = __atomic_load_n(&g_halved_rotations, __ATOMIC_RELAXED);
    if (reset) __atomic_store_n(&g_halved_rotations, 0, __ATOMIC_RELAXED);
    return v;
}

/* Accuracy checks of the Newton-refined reciprocals: out[k] = recip_newton(x[k], y0[k])
 * (two steps) or recip_newton3 (three). */
void oracle_recip_newton(const double *x, const double *y0, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = recip_newton(x[k], y0[k]);
}

void oracle_recip_newton3(const double *x, const double *y0, int64_t n, double *out)
{
    for (int64_t k = 0; k < n; ++k) out[k] = recip_newton3(x[k], y0[k]);
}

static oracle_params make_params(double M, double a, double Q, double dt, double eps,
                                 double horizon_norm, double escape_factor, int max_steps)
{
    oracle_params P;
    P.M = M; P.a = a; P.Q = Q; P.dt = dt; P.eps = eps;
    P.horizon_norm = horizon_norm; P.escape_factor = escape_factor;
    P.max_steps = max_steps; P.trig_mode = g_trig_mode;
    P.kind = METRIC_KN;
    P.method = 0;
    P.disk_r_in = P.disk_r_out = P.disk_dth = 0.0;
    memset(&P.mn, 0, sizeof P.mn);
    pthread_once(&trig_once, trig_init);
    return P;
}

/* Parameters of a Manko-Novikov spacetime (mass M, spin S with 0 < |S| < M^2,
 * quadrupole deviation q). */
static oracle_params make_params_mn(double M, double S, double q, double dt, double eps,
                                    double horizon_norm, double escape_factor, int max_steps)
{
    oracle_params P = make_params(M, S / M, 0.0, dt, eps, horizon_norm, escape_factor,
                                  max_steps);
    P.kind = METRIC_MN;
    mn_consts_make(M, S, q, &P.mn);
    return P;
}

/* Trace pixels of a W x H frame.  pixels == NULL traces all W*H pixels in
 * raster order, else n pixel indices (row-major, j*W + i).  Outputs have n
 * entries (p0: 4 per ray, the initial covector).  Returns the ray count. */
int64_t oracle_trace_frame(double M, double a, double Q,
                           double r0, double th0, double ph0, double fov, int W, int H,
                           double dt, double eps, double horizon_norm,
                           double escape_factor, int max_steps,
                           const int64_t *pixels, int64_t n,
                           double *t, double *r, double *th, double *ph,
                           double *pr, double *pth, double *p0,
                           int8_t *flag, int32_t *steps, int nthreads, int method,
                           const double *disk)
{
    oracle_params P = make_params(M, a, Q, dt, eps, horizon_norm, escape_factor, max_steps);
    P.method = method;
    if (disk) { P.disk_r_in = disk[0]; P.disk_r_out = disk[1]; P.disk_dth = disk[2]; }
    camera_consts C;
    camera_setup(&P, r0, th0, fov, W, H, &C);
    job J;
    memset(&J, 0, sizeof J);
    J.P = &P; J.C = &C; J.r0 = r0; J.th0 = th0; J.ph0 = ph0; J.W = W; J.H = H;
    J.pixels = pixels;
    J.n = pixels ? n : (int64_t)W * H;
    J.t = t; J.r = r; J.th = th; J.ph = ph; J.pr = pr; J.pth = pth; J.p0 = p0;
    J.flag = flag; J.steps = steps;
    run_job(&J, nthreads);
    return J.n;
}

/* Trace n rays from given initial states init[8k..8k+7] = (q^0..q^3, p_0..p_3). */
int64_t oracle_trace_rays(double M, double a, double Q, double dt, double eps,
                          double horizon_norm, double escape_factor, int max_steps,
                          const double *init, int64_t n,
                          double *t, double *r, double *th, double *ph,
                          double *pr, double *pth, int8_t *flag, int32_t *steps,
                          int nthreads)
{
    oracle_params P = make_params(M, a, Q, dt, eps, horizon_norm, escape_factor, max_steps);
    job J;
    memset(&J, 0, sizeof J);
    J.P = &P; J.init = init; J.n = n;
    J.t = t; J.r = r; J.th = th; J.ph = ph; J.pr = pr; J.pth = pth;
    J.flag = flag; J.steps = steps;
    run_job(&J, nthreads);
    return n;
}

/* Initial states (q, p), 8 doubles per ray, of the given pixels. */
void oracle_camera(double M, double a, double Q, double r0, double th0, double ph0,
                   double fov, int W, int H, const int64_t *pixels, int64_t n,
                   double *init)
{
    oracle_params P = make_params(M, a, Q, 0.01, 1e-8, 1e4, 1.5, 1);
    camera_consts C;
    camera_setup(&P, r0, th0, fov, W, H, &C);
    const int64_t cnt = pixels ? n : (int64_t)W * H;
    for (int64_t k = 0; k < cnt; ++k)
        camera_ray(&C, W, H, pixels ? pixels[k] : k, r0, th0, ph0, init + 8 * k,
                   init + 8 * k + 4);
}

/* Inverse metric components at (r, theta) (tests). */
void oracle_inverse_metric(double M, double a, double Q, double r, double theta,
                           double *g5)
{
    oracle_params P = make_params(M, a, Q, 0.01, 1e-8, 1e4, 1.5, 1);
    metric_at_point(&P, r, theta, g5);
}

/* Right-hand side at a state (tests): qdot[4], pdot[2] (p_r, p_theta). */
void oracle_rhs(double M, double a, double Q, double eps, double r, double theta,
                double pt, double pr, double pth, double pph, double *qdot, double *pdot)
{
    oracle_params P = make_params(M, a, Q, 0.01, eps, 1e4, 1.5, 1);
    double eps_sc[2];
    sincos_mode(P.trig_mode, eps, &eps_sc[0], &eps_sc[1]);
    hamilton_rhs(&P, eps_sc, r, theta, pt, pr, pth, pph, qdot, pdot);
}

/* ------------------------------------------------------------------------ */
/* Manko-Novikov entry points: as oracle_trace_frame / oracle_inverse_metric
 * with (M, S, q) in place of (M, a, Q). */
int64_t oracle_trace_frame_mn(double M, double S, double q,
                              double r0, double th0, double ph0, double fov, int W, int H,
                              double dt, double eps, double horizon_norm,
                              double escape_factor, int max_steps,
                              const int64_t *pixels, int64_t n,
                              double *t, double *r, double *th, double *ph,
                              double *pr, double *pth, double *p0,
                              int8_t *flag, int32_t *steps, int nthreads, int method,
                              const double *disk)
{
    oracle_params P = make_params_mn(M, S, q, dt, eps, horizon_norm, escape_factor, max_steps);
    P.method = method;
    if (disk) { P.disk_r_in = disk[0]; P.disk_r_out = disk[1]; P.disk_dth = disk[2]; }
    camera_consts C;
    camera_setup(&P, r0, th0, fov, W, H, &C);
    job J;
    memset(&J, 0, sizeof J);
    J.P = &P; J.C = &C; J.r0 = r0; J.th0 = th0; J.ph0 = ph0; J.W = W; J.H = H;
    J.pixels = pixels;
    J.n = pixels ? n : (int64_t)W * H;
    J.t = t; J.r = r; J.th = th; J.ph = ph; J.pr = pr; J.pth = pth; J.p0 = p0;
    J.flag = flag; J.steps = steps;
    run_job(&J, nthreads);
    return J.n;
}

void oracle_inverse_metric_mn(double M, double S, double q, double r, double theta,
                              double *g5)
{
    oracle_params P = make_params_mn(M, S, q, 0.01, 1e-8, 1e4, 1.5, 1);
    metric_at_point(&P, r, theta, g5);
}

/* Right-hand side at a state (tests), Manko-Novikov. */
void oracle_rhs_mn(double M, double S, double q, double eps, double r, double theta,
                   double pt, double pr, double pth, double pph, double *qdot, double *pdot)
{
    oracle_params P = make_params_mn(M, S, q, 0.01, eps, 1e4, 1.5, 1);
    double eps_sc[2];
    sincos_mode(P.trig_mode, eps, &eps_sc[0], &eps_sc[1]);
    hamilton_rhs(&P, eps_sc, r, theta, pt, pr, pth, pph, qdot, pdot);
}

/* Accuracy checks of the exp definition. */
void oracle_exp(const double *x, int64_t n, double *out)
{
    pthread_once(&trig_once, trig_init);
    for (int64_t k = 0; k < n; ++k) out[k] = exp_def(x[k]);
}

/* Constants (alpha, k, beta) of a Manko-Novikov spacetime (tests). */
void oracle_mn_consts(double M, double S, double q, double *out3)
{
    mn_consts K;
    mn_consts_make(M, S, q, &K);
    out3[0] = K.alpha;
    out3[1] = K.k;
    out3[2] = K.beta;
}

/* ------------------------------------------------------------------------ */
/* Shading of a traced frame (32-bit colours, bytes R, G, B, A in memory).
 *
 * Mode 0, background lines (Sec. 4, the "perspective" and "flat space"
 * figures): the sky an escaping ray reaches is dark blue, with three lines
 * drawn on it, each a narrow interval in one Boyer-Lindquist angle of the
 * ray's end position:
 *   - red, the great circle through the poles in the camera's meridian plane
 *     (phi = 0 or pi): a vertical line through the hole in the image;
 *   - green, the great circle through the poles across the line of sight
 *     (phi = +-pi/2): seen from the camera, a circle around the hole;
 *   - light blue, the equator theta = pi/2 (the interval in 2 theta also
 *     covers the poles, theta = 0 and pi).
 * A line is drawn where the squared sine of the angle's offset from its
 * centre is below 0.01 (a band about 11.5 degrees wide); where lines cross,
 * the one listed first is drawn.  Rays that did not escape are black.
 *
 * Mode 1, exit time (Sec. 4, the exit-time figures): tau = |t| at the end;
 * escaped rays with tau < t_max go from dark blue (tau = 0) to cyan, with
 * level = floor(255 tau / t_max) dimmed to 7/8 on every other band of width
 * `band` (band > 0); rays that did not escape (captured, step limit) and
 * escaped rays with tau >= t_max are cyan; invalid rays are black.
 *
 * Mode 2, texture (Sec. 4, the textured figures): an escaping ray shows the
 * colour of an equirectangular sky texture (tw x th texels, row 0 at theta =
 * 0, column 0 at phi = 0, phi increasing with the column) at its end
 * direction, with bilinear filtering; other rays are black.  theta is first
 * brought into [0, pi] (theta mod 2 pi; above pi it is reflected, 2 pi -
 * theta, and phi turned by pi, the same direction), u = frac(phi / 2 pi),
 * v = theta / pi; texel (i, j) is centred at ((i + 1/2)/tw, (j + 1/2)/th), so
 * x = u tw - 1/2, y = v th - 1/2, (i0, j0) = floor(x, y), (fx, fy) their
 * fractions; columns wrap around (i0 and i0 + 1 modulo tw), rows clamp to
 * [0, th - 1].  Each channel is the linear interpolation of the four texels,
 * first along the row and then between the rows:
 *   a = c00 + fx (c10 - c00),  b = c01 + fx (c11 - c01),  c = a + fy (b - a)
 * (each a single fma in binary64) and the byte is floor(c + 1/2). */
enum { BAND_PHI = 0, BAND_TWO_THETA = 1 };
enum { BAND_SIN = 0, BAND_COS = 1 };
typedef struct {
    int angle, part;
    uint32_t rgba;
} sky_line;

static const sky_line SKY_LINES[3] = {
    {BAND_PHI, BAND_SIN, 0xff0000ffu},        /* red: phi = 0, pi */
    {BAND_PHI, BAND_COS, 0xff00ff00u},        /* green: phi = +-pi/2 */
    {BAND_TWO_THETA, BAND_SIN, 0xffff0000u},  /* light blue: equator (and poles) */
};
static const double SKY_LINE_SIN2 = 0.01;
static const uint32_t SKY = 0xff3c0000u;      /* dark blue */

static uint32_t sky_lines(double theta, double phi)
{
    double sc[2][2];                          /* [angle][sin, cos] */
    trig_sincos(phi, &sc[BAND_PHI][0], &sc[BAND_PHI][1]);
    trig_sincos(2.0 * theta, &sc[BAND_TWO_THETA][0], &sc[BAND_TWO_THETA][1]);
    for (int k = 0; k < 3; ++k) {
        const double v = sc[SKY_LINES[k].angle][SKY_LINES[k].part];
        if (v * v < SKY_LINE_SIN2) return SKY_LINES[k].rgba;
    }
    return SKY;
}

static uint32_t texture_lookup(const uint32_t *tex, int tw, int th, double theta, double phi)
{
    const double two_pi = 2.0 * PIO2_HI * 2.0;                 /* fl(2 pi) */
    const double pi = 2.0 * PIO2_HI;                           /* fl(pi) */
    double t = theta - two_pi * floor(theta / two_pi);
    double p = phi;
    if (t > pi) {
        t = two_pi - t;
        p = p + pi;
    }
    double u = p / two_pi;
    u = u - floor(u);
    const double v = t / pi;
    const double x = u * (double)tw - 0.5, y = v * (double)th - 0.5;
    const double xf = floor(x), yf = floor(y);
    const double fx = x - xf, fy = y - yf;
    int64_t i0 = (int64_t)xf % tw;
    if (i0 < 0) i0 += tw;
    const int64_t i1 = (i0 + 1) % tw;
    int64_t j0 = (int64_t)yf, j1 = j0 + 1;
    j0 = j0 < 0 ? 0 : (j0 > th - 1 ? th - 1 : j0);
    j1 = j1 < 0 ? 0 : (j1 > th - 1 ? th - 1 : j1);
    const uint32_t q00 = tex[j0 * tw + i0], q10 = tex[j0 * tw + i1];
    const uint32_t q01 = tex[j1 * tw + i0], q11 = tex[j1 * tw + i1];
    uint32_t out = 0;
    for (int ch = 0; ch < 4; ++ch) {
        const int sh = 8 * ch;
        const double c00 = (double)((q00 >> sh) & 255u), c10 = (double)((q10 >> sh) & 255u);
        const double c01 = (double)((q01 >> sh) & 255u), c11 = (double)((q11 >> sh) & 255u);
        const double a = fma(fx, c10 - c00, c00);
        const double b = fma(fx, c11 - c01, c01);
        const double c = fma(fy, b - a, a);
        out |= ((uint32_t)floor(c + 0.5)) << sh;
    }
    return out;
}

static uint32_t shade_one(int mode, double t_max, double band, const uint32_t *tex, int tw,
                          int th, double t, double theta, double phi, int flag)
{
    const uint32_t BLACK = 0xff000000u, CYAN = 0xffffff00u;
    if (mode == 0) return flag == FLAG_ESCAPE ? sky_lines(theta, phi) : BLACK;
    if (mode == 2) return flag == FLAG_ESCAPE ? texture_lookup(tex, tw, th, theta, phi) : BLACK;
    if (flag == FLAG_INVALID) return BLACK;
    if (flag != FLAG_ESCAPE) return CYAN;
    const double tau = fabs(t);
    const double u = tau / t_max;
    if (!(u < 1.0)) return CYAN;
    uint32_t level = (uint32_t)(u * 255.0);
    if (band > 0.0 && (((int64_t)(tau / band)) & 1)) level = (level * 7u) / 8u;
    const uint32_t blue = 64u + (level * 191u) / 255u;
    return 0xff000000u | (blue << 16) | (level << 8);
}

void oracle_shade(int mode, double t_max, double band, const uint32_t *tex, int tw, int th,
                  const double *t, const double *theta, const double *phi, const int8_t *flag,
                  int64_t n, uint32_t *out)
{
    pthread_once(&trig_once, trig_init);
    for (int64_t k = 0; k < n; ++k)
        out[k] = shade_one(mode, t_max, band, tex, tw, th, t ? t[k] : 0.0,
                           theta ? theta[k] : 0.0, phi ? phi[k] : 0.0, flag[k]);
}

/* ------------------------------------------------------------------------ */
/* Redshift of light from the ring (Sec. 3.3.3 "Redshift").  The ring's matter
 * moves on circular equatorial-type orbits: p_r = p_theta = 0 and dp/dtau = 0,
 * so with s_t = -1 its s_phi solves
 *   s_phi^2 d_r g^{phph} - 2 s_phi d_r g^{tph} + d_r g^{tt} = 0
 * (d_r by the same forward difference of step eps as the integrator); of the
 * two roots the orbit with the larger dphi/dt is taken (prograde: the ring
 * turns toward +phi when the hole does).  s is rescaled to g^{mu nu} s_mu
 * s_nu = -1 and S^mu = g^{mu nu} s_nu.  A ray whose covector p is scaled to
 * dt/dtau = -1 at the camera (the camera rays of this tracer) reaches the
 * ring's matter with frequency p_mu S^mu, and the camera's locally
 * non-rotating observer receives it with frequency sqrt(-1/g^{tt}) at the
 * camera, so z = lambda_O / lambda_S = (p_t S^t + p_phi S^phi) /
 * sqrt(-1/g^{tt}(camera)).  NaN where no timelike circular orbit exists. */
static int disk_orbit(const oracle_params *P, double r, double theta, double out[3])
{
    double g[5], gr[5], s, c;
    trig_sincos(theta, &s, &c);
    if (P->kind == METRIC_MN) {
        mn_inverse_metric(&P->mn, r, c, s * s, g);
        mn_inverse_metric(&P->mn, r + P->eps, c, s * s, gr);
    } else {
        inverse_metric(P, r, s * s, g);
        inverse_metric(P, r + P->eps, s * s, gr);
    }
    const double dtt = gr[0] - g[0], dtp = gr[1] - g[1], dpp = gr[4] - g[4];
    const double disc = dtp * dtp - dpp * dtt;                 /* (B^2 - 4AC) / 4 */
    if (!(disc >= 0.0) || dpp == 0.0) return 0;
    const double sq = sqrt(disc);
    const double x1 = (dtp + sq) / dpp, x2 = (dtp - sq) / dpp; /* s_phi with s_t = -1 */
    /* dphi/dt = (g^tph s_t + g^phph s_phi) / (g^tt s_t + g^tph s_phi) */
    const double w1 = fma(g[4], x1, -g[1]) / fma(g[1], x1, -g[0]);
    const double w2 = fma(g[4], x2, -g[1]) / fma(g[1], x2, -g[0]);
    const double x = (w1 >= w2) ? x1 : x2;
    const double norm = fma(g[4] * x, x, fma(-2.0 * g[1], x, g[0]));  /* g^{mu nu} s s */
    if (!(norm < 0.0)) return 0;
    const double k = 1.0 / sqrt(-norm);
    const double st = -k, sp = x * k;
    out[0] = fma(g[0], st, g[1] * sp);                         /* S^t */
    out[1] = fma(g[1], st, g[4] * sp);                         /* S^phi */
    out[2] = out[1] / out[0];                                  /* dphi/dt */
    return 1;
}

static void redshift_rays(const oracle_params *P, double r0, double th0, const double *r,
                          const double *theta, const double *pt, const double *pph,
                          const int8_t *flag, int64_t n, double *z)
{
    double g0[5];
    metric_at_point(P, r0, th0, g0);
    const double nu_o = sqrt(-1.0 / g0[0]);
    for (int64_t k = 0; k < n; ++k) {
        double S[3];
        if (flag[k] != FLAG_DISK || !disk_orbit(P, r[k], theta[k], S)) {
            z[k] = NAN;
            continue;
        }
        z[k] = fma(pt[k], S[0], pph[k] * S[1]) / nu_o;
    }
}

void oracle_redshift(double M, double a, double Q, double eps, double r0, double th0,
                     const double *r, const double *theta, const double *pt, const double *pph,
                     const int8_t *flag, int64_t n, double *z)
{
    oracle_params P = make_params(M, a, Q, 0.01, eps, 1e4, 1.5, 1);
    redshift_rays(&P, r0, th0, r, theta, pt, pph, flag, n, z);
}

void oracle_redshift_mn(double M, double S, double q, double eps, double r0, double th0,
                        const double *r, const double *theta, const double *pt,
                        const double *pph, const int8_t *flag, int64_t n, double *z)
{
    oracle_params P = make_params_mn(M, S, q, 0.01, eps, 1e4, 1.5, 1);
    redshift_rays(&P, r0, th0, r, theta, pt, pph, flag, n, z);
}

/* The ring's orbit at (r, theta) for tests: (S^t, S^phi, dphi/dt), 0 if none. */
int oracle_disk_orbit(int kind, double M, double a_or_S, double Q_or_q, double eps, double r,
                      double theta, double *out3)
{
    oracle_params P = kind == METRIC_MN
                          ? make_params_mn(M, a_or_S, Q_or_q, 0.01, eps, 1e4, 1.5, 1)
                          : make_params(M, a_or_S, Q_or_q, 0.01, eps, 1e4, 1.5, 1);
    return disk_orbit(&P, r, theta, out3);
}
