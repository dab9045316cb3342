/*
 * Listing-form reference tracer: the paper's method written as its plain
 * definitions.  TEST INFRASTRUCTURE ONLY: only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it; nothing in the product
 * path may call it, and it shares no code with the HIP implementation (nor
 * with the kernel-twin form in oracle.c).
 *
 * What it computes, step by step (paper: Sec. 2.1 eq. hamGeodesic with the
 * factor 1/2 of Appendix A; Sec. 2.2.2 and 2.2.3 for the metrics; Sec. 3.1
 * for RK4 and Euler; Sec. 3.3 "Raytracing"; the appendix "Code for
 * propagation of rays" for the finite differences, the step normaliser and
 * the exits):
 *
 *   - g^{mu nu}(r, theta) is a 4x4 array filled from the textbook formulas
 *     at the point itself: sin, cos, exp, log and sqrt from the C library,
 *     every component with its own division.  Kerr-Newman: the Boyer-
 *     Lindquist inverse metric with Delta = r^2 - 2Mr + a^2 + Q^2.
 *     Manko-Novikov: the inverse components of the appendix listing from
 *     f, omega, gamma of Sec. 2.2.3 (with the readings that make q = 0 Kerr
 *     and the metric a vacuum solution: the first term of the line element
 *     squared, B a sum of two squares, the beta term of gamma'
 *     beta (-2 + sum)).
 *   - d_r g = (g(fl(r + eps), theta) - g(r, theta)) / eps and
 *     d_theta g = (g(r, fl(theta + eps)) - g(r, theta)) / eps, component by
 *     component; the t and phi derivatives are zero.
 *   - dq^mu/dtau = sum_nu g^{mu nu} p_nu and
 *     dp_mu/dtau = sum_{nu, sigma} -1/2 d_mu g^{nu sigma} p_nu p_sigma over
 *     all sixteen (nu, sigma).
 *   - RK4 on the 8-vector y = (q, p) with the textbook stages
 *     y + h/2 k1, y + h/2 k2, y + h k3 and y += h/6 (k1 + 2 k2 + 2 k3 + k4),
 *     where h = dt / |dq^t/dtau| is taken from k1 and kept for the step
 *     (coordinate-time steps); or explicit Euler y += h k1.
 *   - After each update: the solid ring (if any), then escape
 *     r > escape_factor * r_start, then the horizon |dq^t/dtau| > horizon_norm
 *     (the collapse of the coordinate-time step), then a non-finite state;
 *     the step limit ends the ray otherwise.
 *   - Camera (Sec. 3.3.1): a pinhole at rest in the locally non-rotating
 *     (zero angular momentum) frame.  Pixel (i, j) looks along
 *     n = (-1, -y, x) / |.| in that frame's (r, theta, phi) unit vectors,
 *     x = ((2i + 1 - W)/W) tan(fov/2), y = ((H - 2j - 1)/W) tan(fov/2).  The
 *     backward ray's tangent is v = alpha (-u + n), u the observer's
 *     4-velocity and alpha the lapse, which makes v null with dt/dtau = -1;
 *     the covector is p_mu = g_{mu nu} v^nu with the covariant metric.
 *
 * Everything is IEEE binary64, compiled with -ffp-contract=off: no product
 * is fused.  This form and the kernel evaluate the same function values up
 * to rounding; since the forward difference divides rounding by eps, their
 * end angles differ by about what a one-ulp change of a ray's start does.
 * That sensitivity is measured per ray by re-running it from perturbed
 * starts (the conditioning probe): p_theta scaled by 1 + 2^-52, the camera
 * latitude moved up by one ulp, and the whole covector scaled by 1 + 2^-52
 * and by 1 - 2^-53 (probes 1-4); then p_theta scaled by 1 - 2^-53, the
 * latitude moved down by one ulp, and p_r scaled by 1 + 2^-52 and by
 * 1 - 2^-53 (probes 5-8).  A ray's flag and step count count as ill-conditioned when a
 * probe changes them, or when the exit was a tie: the escape or horizon test
 * was decided by a margin within TIE_K times the probes' spread of the tested
 * quantity.
 *
 * Parity status: pinned (the pins of the kernel-twin form apply to this form
 * too: flat space, Schwarzschild critical impact parameter and deflection
 * integral, capture by the radial potential, conservation, mirror
 * symmetries, the Manko-Novikov Kerr limit).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double HALF_PI = 1.57079632679489661923;   /* pi/2, rounded once */

enum { LF_TIMEOUT = 0, LF_ESCAPE = 1, LF_HORIZON = 2, LF_INVALID = 3, LF_DISK = 4 };

typedef struct {
    int mn;                          /* 0: Kerr-Newman, 1: Manko-Novikov */
    double M, a, Q;                  /* Kerr-Newman mass, spin length, charge */
    double alpha, k, beta;           /* Manko-Novikov constants from (M, S, q) */
    double dt, eps, hnorm, esc;
    int max_steps, method;           /* 0 RK4, 1 explicit Euler, 2 RK4 in coordinate time */
    double ring_in, ring_out, ring_dth;   /* ring off when ring_dth <= 0 */
} lspec;

/* ------------------------------------------------------------------ metrics */

/* Kerr-Newman, Boyer-Lindquist (Sec. 2.2.2, with the charge in Delta). */
static void kn_inverse(const lspec *L, double r, double th, double g[4][4])
{
    const double M = L->M, a = L->a, Q = L->Q;
    const double s = sin(th), c = cos(th);
    const double Delta = r * r - 2.0 * M * r + a * a + Q * Q;
    const double rho2 = r * r + a * a * c * c;
    const double Sigma2 = (r * r + a * a) * (r * r + a * a) - a * a * Delta * s * s;
    memset(g, 0, 16 * sizeof(double));
    g[0][0] = -Sigma2 / (rho2 * Delta);
    g[0][3] = -a * (2.0 * M * r - Q * Q) / (rho2 * Delta);
    g[3][0] = g[0][3];
    g[1][1] = Delta / rho2;
    g[2][2] = 1.0 / rho2;
    g[3][3] = (Delta - a * a * s * s) / (rho2 * Delta * s * s);
}

static void kn_covariant(const lspec *L, double r, double th, double g[4][4])
{
    const double M = L->M, a = L->a, Q = L->Q;
    const double s = sin(th), c = cos(th);
    const double Delta = r * r - 2.0 * M * r + a * a + Q * Q;
    const double rho2 = r * r + a * a * c * c;
    const double F = 2.0 * M * r - Q * Q;
    memset(g, 0, 16 * sizeof(double));
    g[0][0] = -(1.0 - F / rho2);
    g[0][3] = -a * s * s * F / rho2;
    g[3][0] = g[0][3];
    g[1][1] = rho2 / Delta;
    g[2][2] = rho2;
    g[3][3] = (r * r + a * a + a * a * s * s * F / rho2) * s * s;
}

/* The functions f, omega, e^{2 gamma} rho^2 and Delta sin^2 of the
 * Manko-Novikov spacetime at (r, theta) (Sec. 2.2.3). */
typedef struct {
    double f, omega, e2g_rho2, Delta, Dsin2;
} mn_fields;

static double legendre(int l, double u)
{
    if (l == 0) return 1.0;
    if (l == 1) return u;
    if (l == 2) return (3.0 * u * u - 1.0) / 2.0;
    return (5.0 * u * u * u - 3.0 * u) / 2.0;
}

static void mn_eval(const lspec *L, double r, double th, mn_fields *F)
{
    const double M = L->M, al = L->alpha, k = L->k, beta = L->beta;
    const double x = (r - M) / k, y = cos(th), s = sin(th);
    const double R = sqrt(x * x + y * y - 1.0);
    const double u = x * y / R;
    double suma = 0.0, sumb = 0.0, sumg = 0.0;
    for (int l = 0; l <= 2; ++l) {
        const double Pl = legendre(l, u), Rl = pow(R, (double)(l + 1));
        const double sgn3 = ((3 - l) % 2) ? -1.0 : 1.0;   /* (-1)^(3-l) */
        const double sgn2 = ((2 - l) % 2) ? -1.0 : 1.0;   /* (-1)^(2-l) */
        suma += (x - y) * Pl / Rl;
        sumb += sgn3 * (x + y) * Pl / Rl;
        sumg += (x - y + sgn2 * (x + y)) * Pl / Rl;
    }
    const double A_ = -al * exp(-2.0 * beta * (-1.0 + suma));    /* fraktur a */
    const double B_ = al * exp(2.0 * beta * (1.0 + sumb));       /* fraktur b */
    const double P2 = legendre(2, u), P3 = legendre(3, u);
    const double psi = beta * P2 / (R * R * R);
    const double A = (x * x - 1.0) * (1.0 + A_ * B_) * (1.0 + A_ * B_)
                     - (1.0 - y * y) * (B_ - A_) * (B_ - A_);
    const double b1 = (x + 1.0) + (x - 1.0) * A_ * B_;
    const double b2 = (1.0 + y) * A_ + (1.0 - y) * B_;
    const double B = b1 * b1 + b2 * b2;
    const double C = (x * x - 1.0) * (1.0 + A_ * B_) * ((B_ - A_) - y * (A_ + B_))
                     + (1.0 - y * y) * (B_ - A_) * ((1.0 + A_ * B_) + x * (1.0 - A_ * B_));
    const double gamma_p = log(sqrt((x * x - 1.0) / (x * x - y * y)))
                           + 3.0 * beta * beta / (2.0 * pow(R, 6.0)) * (P3 * P3 - P2 * P2)
                           + beta * (-2.0 + sumg);
    const double e2g = exp(2.0 * gamma_p) * A / ((x * x - 1.0) * (1.0 - al * al) * (1.0 - al * al));
    const double rho2 = (r - M) * (r - M) - k * k * y * y;
    F->f = exp(2.0 * psi) * A / B;
    F->omega = 2.0 * k * exp(-2.0 * psi) * C / A - 4.0 * k * al / (1.0 - al * al);
    F->e2g_rho2 = e2g * rho2;
    F->Delta = (r - M) * (r - M) - k * k;
    F->Dsin2 = F->Delta * s * s;
}

/* Inverse components as the appendix listing's metricAtPoint assigns them. */
static void mn_inverse(const lspec *L, double r, double th, double g[4][4])
{
    mn_fields F;
    mn_eval(L, r, th, &F);
    memset(g, 0, 16 * sizeof(double));
    g[0][0] = -1.0 / F.f + F.f * F.omega * F.omega / F.Dsin2;
    g[1][1] = F.f * F.Delta / F.e2g_rho2;
    g[2][2] = F.f / F.e2g_rho2;
    g[3][3] = F.f / F.Dsin2;
    g[0][3] = F.f * F.omega / F.Dsin2;
    g[3][0] = g[0][3];
}

/* ds^2 = -f (dt - omega dphi)^2 + f^-1 [e^{2 gamma} rho^2 (dr^2/Delta + dtheta^2)
 *        + Delta sin^2 dphi^2]. */
static void mn_covariant(const lspec *L, double r, double th, double g[4][4])
{
    mn_fields F;
    mn_eval(L, r, th, &F);
    memset(g, 0, 16 * sizeof(double));
    g[0][0] = -F.f;
    g[0][3] = F.f * F.omega;
    g[3][0] = g[0][3];
    g[1][1] = F.e2g_rho2 / (F.f * F.Delta);
    g[2][2] = F.e2g_rho2 / F.f;
    g[3][3] = -F.f * F.omega * F.omega + F.Dsin2 / F.f;
}

static void inverse_at(const lspec *L, double r, double th, double g[4][4])
{
    if (L->mn) mn_inverse(L, r, th, g);
    else kn_inverse(L, r, th, g);
}

static void covariant_at(const lspec *L, double r, double th, double g[4][4])
{
    if (L->mn) mn_covariant(L, r, th, g);
    else kn_covariant(L, r, th, g);
}

/* --------------------------------------------------------- Hamilton's equations */

/* dy/dtau for y = (t, r, theta, phi, p_t, p_r, p_theta, p_phi). */
static void hamilton(const lspec *L, const double y[8], double dy[8])
{
    double g[4][4], gr[4][4], gth[4][4], D[4][4][4];
    const double r = y[1], th = y[2];
    const double *p = y + 4;
    inverse_at(L, r, th, g);
    inverse_at(L, r + L->eps, th, gr);
    inverse_at(L, r, th + L->eps, gth);
    memset(D, 0, sizeof D);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            D[1][m][n] = (gr[m][n] - g[m][n]) / L->eps;
            D[2][m][n] = (gth[m][n] - g[m][n]) / L->eps;
        }
    for (int mu = 0; mu < 4; ++mu) {
        double qd = 0.0, pd = 0.0;
        for (int nu = 0; nu < 4; ++nu) {
            qd += g[mu][nu] * p[nu];
            for (int sg = 0; sg < 4; ++sg) pd += -0.5 * D[mu][nu][sg] * p[nu] * p[sg];
        }
        dy[mu] = qd;
        dy[4 + mu] = pd;
    }
}

static int finite8(const double y[8])
{
    for (int m = 0; m < 8; ++m)
        if (!isfinite(y[m])) return 0;
    return 1;
}

/* What decided a ray's escape or horizon exit: the tested quantity (r for
 * escape, |dt/dtau| for the horizon) after the final step and after the step
 * before, and its threshold (has = 0 for the other exits). */
typedef struct {
    int has;
    double now, before, thr;
} ldecision;

/* Integrate one ray in place; returns the flag and the updates taken (and,
 * if dec is given, what decided the exit). */
static int integrate(const lspec *L, double y[8], int *nsteps, ldecision *dec)
{
    const double r_esc = L->esc * y[1];
    double r_before = y[1], nu_before = 0.0;
    *nsteps = 0;
    if (dec) dec->has = 0;
    if (!finite8(y)) return LF_INVALID;
    for (int s = 1; s <= L->max_steps; ++s) {
        double k1[8], k2[8], k3[8], k4[8], z[8];
        hamilton(L, y, k1);
        const double nu = fabs(k1[0]);
        const double h = L->dt / nu;
        if (L->method == 1) {
            for (int m = 0; m < 8; ++m) y[m] = y[m] + h * k1[m];
        } else if (L->method == 2) {
            /* RK4 with coordinate time as the parameter: every stage's
             * derivative is divided by its own |dt/dtau|, and the step is dt */
            const double n1 = nu;
            for (int m = 0; m < 8; ++m) z[m] = y[m] + 0.5 * L->dt * (k1[m] / n1);
            hamilton(L, z, k2);
            const double n2 = fabs(k2[0]);
            for (int m = 0; m < 8; ++m) z[m] = y[m] + 0.5 * L->dt * (k2[m] / n2);
            hamilton(L, z, k3);
            const double n3 = fabs(k3[0]);
            for (int m = 0; m < 8; ++m) z[m] = y[m] + L->dt * (k3[m] / n3);
            hamilton(L, z, k4);
            const double n4 = fabs(k4[0]);
            for (int m = 0; m < 8; ++m)
                y[m] = y[m] + L->dt / 6.0 * (k1[m] / n1 + 2.0 * (k2[m] / n2) +
                                             2.0 * (k3[m] / n3) + k4[m] / n4);
        } else {
            for (int m = 0; m < 8; ++m) z[m] = y[m] + 0.5 * h * k1[m];
            hamilton(L, z, k2);
            for (int m = 0; m < 8; ++m) z[m] = y[m] + 0.5 * h * k2[m];
            hamilton(L, z, k3);
            for (int m = 0; m < 8; ++m) z[m] = y[m] + h * k3[m];
            hamilton(L, z, k4);
            for (int m = 0; m < 8; ++m)
                y[m] = y[m] + h / 6.0 * (k1[m] + 2.0 * k2[m] + 2.0 * k3[m] + k4[m]);
        }
        *nsteps = s;
        if (L->ring_dth > 0.0 && y[1] >= L->ring_in && y[1] <= L->ring_out &&
            fabs(y[2] - HALF_PI) <= L->ring_dth)
            return LF_DISK;
        if (y[1] > r_esc) {
            if (dec) *dec = (ldecision){1, y[1], r_before, r_esc};
            return LF_ESCAPE;
        }
        if (nu > L->hnorm) {
            if (dec) *dec = (ldecision){1, nu, nu_before, L->hnorm};
            return LF_HORIZON;
        }
        if (!finite8(y)) return LF_INVALID;
        r_before = y[1];
        nu_before = nu;
    }
    return LF_TIMEOUT;
}

/* ------------------------------------------------------------------- camera */

/* Start state of pixel (i, j) of a W x H camera at (r0, th0, ph0). */
static void camera_start(const lspec *L, double r0, double th0, double ph0, double fov,
                         int W, int H, int64_t i, int64_t j, double y[8])
{
    double g[4][4];
    covariant_at(L, r0, th0, g);
    const double tan_h = tan(fov / 2.0);
    const double x = ((double)(2 * i + 1 - W) / (double)W) * tan_h;
    const double yy = ((double)(H - 2 * j - 1) / (double)W) * tan_h;
    const double norm = sqrt(1.0 + x * x + yy * yy);
    const double n_r = -1.0 / norm, n_th = -yy / norm, n_ph = x / norm;
    /* locally non-rotating observer: angular velocity and lapse */
    const double omega = -g[0][3] / g[3][3];
    const double lapse = sqrt((g[0][3] * g[0][3] - g[0][0] * g[3][3]) / g[3][3]);
    double v[4];
    v[0] = -1.0;
    v[1] = lapse * n_r / sqrt(g[1][1]);
    v[2] = lapse * n_th / sqrt(g[2][2]);
    v[3] = -omega + lapse * n_ph / sqrt(g[3][3]);
    y[0] = 0.0;
    y[1] = r0;
    y[2] = th0;
    y[3] = ph0;
    for (int mu = 0; mu < 4; ++mu) {
        double pm = 0.0;
        for (int nu = 0; nu < 4; ++nu) pm += g[mu][nu] * v[nu];
        y[4 + mu] = pm;
    }
}

/* ------------------------------------------------------------------ drivers */

enum { NPROBE_MAX = 8 };

/* An exit is a tie when its margin from the threshold (on the side of the
 * final step or of the step before) is within TIE_K times the probes' spread
 * of the deciding quantity: an evaluation that rounds differently could then
 * exit one step earlier or later (the factor is the angle gate's). */
static const double TIE_K = 64.0;

typedef struct {
    const lspec *L;
    double r0, th0, ph0, fov;
    int W, H;
    const int64_t *pixels;
    const double *init;              /* ray-list mode: 8 doubles per ray */
    int64_t n;
    int nprobe;
    double *out8;                    /* 8 doubles per ray: end (q, p) */
    double *p0;                      /* 4 per ray: start covector (may be NULL) */
    int8_t *flag;
    int32_t *steps;
    double *sens;                    /* per ray: probe sensitivity (may be NULL) */
    int8_t *flip;                    /* per ray: a probe changed flag or steps */
    int64_t next;
} ljob;

static void start_of(const ljob *J, int64_t k, double th0, double y[8])
{
    if (J->init) {
        memcpy(y, J->init + 8 * k, 8 * sizeof(double));
        return;
    }
    const int64_t pix = J->pixels ? J->pixels[k] : k;
    camera_start(J->L, J->r0, th0, J->ph0, J->fov, J->W, J->H, pix % J->W, pix / J->W, y);
}

static double angdiff(const double a[8], const double b[8])
{
    const double d1 = fabs(a[2] - b[2]), d2 = fabs(a[3] - b[3]);
    return d1 > d2 ? d1 : d2;
}

static void run_ray(ljob *J, int64_t k)
{
    double y0[8], y[8];
    start_of(J, k, J->th0, y0);
    if (J->p0) memcpy(J->p0 + 4 * k, y0 + 4, 4 * sizeof(double));
    memcpy(y, y0, sizeof y);
    int ns = 0;
    ldecision dec;
    const int f = integrate(J->L, y, &ns, &dec);
    memcpy(J->out8 + 8 * k, y, sizeof y);
    J->flag[k] = (int8_t)f;
    if (J->steps) J->steps[k] = ns;
    if (J->nprobe <= 0) return;
    double sens = 0.0, spread = 0.0;
    int flip = 0;
    const double up = 1.0 + 0x1p-52;
    const double down = 1.0 - 0x1p-53;
    for (int pb = 0; pb < J->nprobe && pb < NPROBE_MAX; ++pb) {
        double z[8];
        if ((pb == 1 || pb == 5) && !J->init) {
            start_of(J, k, nextafter(J->th0, pb == 1 ? INFINITY : -INFINITY), z);
        } else {
            memcpy(z, y0, sizeof z);
            if (pb == 0 || pb == 4) {
                z[6] = z[6] * (pb == 0 ? up : down);                /* p_theta */
            } else if (pb == 1 || pb == 5) {
                z[2] = nextafter(z[2], pb == 1 ? INFINITY : -INFINITY);   /* theta (ray lists) */
            } else if (pb == 6 || pb == 7) {
                z[5] = z[5] * (pb == 6 ? up : down);                /* p_r */
            } else {
                /* the whole covector scaled: the same ray in coordinate time,
                 * every rounding different */
                const double lam = pb == 2 ? up : down;
                for (int m = 4; m < 8; ++m) z[m] = z[m] * lam;
            }
        }
        int nz = 0;
        ldecision dz;
        const int fz = integrate(J->L, z, &nz, &dz);
        if (fz != f || nz != ns) flip = 1;
        else if (dec.has) spread = fmax(spread, fmax(fabs(dz.now - dec.now),
                                                     fabs(dz.before - dec.before)));
        const double d = angdiff(y, z);
        if (d > sens || d != d) sens = d;
    }
    if (dec.has && !flip) {
        const double margin = fmin(dec.now - dec.thr, dec.thr - dec.before);
        if (margin <= TIE_K * spread) flip = 1;             /* a tie: see TIE_K */
    }
    if (J->sens) J->sens[k] = sens;
    if (J->flip) J->flip[k] = (int8_t)flip;
}

static void *lworker(void *arg)
{
    ljob *J = (ljob *)arg;
    const int64_t chunk = 4;
    for (;;) {
        const int64_t b = __atomic_fetch_add(&J->next, chunk, __ATOMIC_RELAXED);
        if (b >= J->n) break;
        const int64_t e = b + chunk < J->n ? b + chunk : J->n;
        for (int64_t k = b; k < e; ++k) run_ray(J, k);
    }
    return NULL;
}

static void lrun(ljob *J, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t tid[256];
    int started = 0;
    J->next = 0;
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&tid[started], NULL, lworker, J) == 0) ++started;
    lworker(J);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
}

/* Manko-Novikov constants (Sec. 2.2.3): alpha from the spin S, k, beta. */
static void mn_setup(lspec *L, double M, double S, double q)
{
    const double chi = S / M;
    L->mn = 1;
    L->M = M;
    L->a = chi;
    L->Q = 0.0;
    L->alpha = (-M + sqrt(M * M - chi * chi)) / chi;
    L->k = M * (1.0 - L->alpha * L->alpha) / (1.0 + L->alpha * L->alpha);
    L->beta = q * M * M * M / (L->k * L->k * L->k);
}

/* Trace pixels of a frame in the listing form.  kind 0: (p1, p2, p3) =
 * (M, a, Q) Kerr-Newman; kind 1: (M, S, q) Manko-Novikov.  method 0 RK4,
 * 1 Euler, 2 RK4 in coordinate time; ring = (r_in, r_out, half angle) or NULL.  out8 receives the end
 * (t, r, theta, phi, p_t, p_r, p_theta, p_phi) of every ray; with nprobe > 0
 * (at most 8) each ray is re-run from that many perturbed starts and sens/flip
 * receive the largest end-angle change and whether flag or steps changed. */
int64_t listing_trace_frame(int kind, double p1, double p2, double p3, double r0, double th0,
                            double ph0, double fov, int W, int H, double dt, double eps,
                            double horizon_norm, double escape_factor, int max_steps,
                            int method, const double *ring, const int64_t *pixels, int64_t n,
                            int nprobe, double *out8, double *p0, int8_t *flag,
                            int32_t *steps, double *sens, int8_t *flip, int nthreads)
{
    lspec L;
    memset(&L, 0, sizeof L);
    if (kind == 1) {
        mn_setup(&L, p1, p2, p3);
    } else {
        L.M = p1; L.a = p2; L.Q = p3;
    }
    L.dt = dt; L.eps = eps; L.hnorm = horizon_norm; L.esc = escape_factor;
    L.max_steps = max_steps; L.method = method;
    if (ring) { L.ring_in = ring[0]; L.ring_out = ring[1]; L.ring_dth = ring[2]; }
    ljob J;
    memset(&J, 0, sizeof J);
    J.L = &L; J.r0 = r0; J.th0 = th0; J.ph0 = ph0; J.fov = fov; J.W = W; J.H = H;
    J.pixels = pixels;
    J.n = pixels ? n : (int64_t)W * H;
    J.nprobe = nprobe;
    J.out8 = out8; J.p0 = p0; J.flag = flag; J.steps = steps; J.sens = sens; J.flip = flip;
    lrun(&J, nthreads);
    return J.n;
}

/* The same from explicit start states init[8k .. 8k+7] (Kerr-Newman or
 * Manko-Novikov as above; the third probe moves theta by one ulp). */
int64_t listing_trace_rays(int kind, double p1, double p2, double p3, double dt, double eps,
                           double horizon_norm, double escape_factor, int max_steps,
                           int method, const double *init, int64_t n, int nprobe,
                           double *out8, int8_t *flag, int32_t *steps, double *sens,
                           int8_t *flip, int nthreads)
{
    lspec L;
    memset(&L, 0, sizeof L);
    if (kind == 1) {
        mn_setup(&L, p1, p2, p3);
    } else {
        L.M = p1; L.a = p2; L.Q = p3;
    }
    L.dt = dt; L.eps = eps; L.hnorm = horizon_norm; L.esc = escape_factor;
    L.max_steps = max_steps; L.method = method;
    ljob J;
    memset(&J, 0, sizeof J);
    J.L = &L; J.init = init; J.n = n; J.nprobe = nprobe;
    J.out8 = out8; J.flag = flag; J.steps = steps; J.sens = sens; J.flip = flip;
    lrun(&J, nthreads);
    return n;
}

/* Start states (8 doubles per pixel) of a listing-form camera. */
void listing_camera(int kind, double p1, double p2, double p3, double r0, double th0,
                    double ph0, double fov, int W, int H, const int64_t *pixels, int64_t n,
                    double *init)
{
    lspec L;
    memset(&L, 0, sizeof L);
    if (kind == 1) mn_setup(&L, p1, p2, p3);
    else { L.M = p1; L.a = p2; L.Q = p3; }
    const int64_t cnt = pixels ? n : (int64_t)W * H;
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t pix = pixels ? pixels[k] : k;
        camera_start(&L, r0, th0, ph0, fov, W, H, pix % W, pix / W, init + 8 * k);
    }
}

/* g^{mu nu} (16 values, row-major) and g_{mu nu} at (r, theta) (tests). */
void listing_metric(int kind, double p1, double p2, double p3, double r, double theta,
                    double *inv16, double *cov16)
{
    lspec L;
    memset(&L, 0, sizeof L);
    if (kind == 1) mn_setup(&L, p1, p2, p3);
    else { L.M = p1; L.a = p2; L.Q = p3; }
    double g[4][4];
    inverse_at(&L, r, theta, g);
    memcpy(inv16, g, sizeof g);
    covariant_at(&L, r, theta, g);
    memcpy(cov16, g, sizeof g);
}

/* Hamilton's right-hand side at y (8 values) with step eps (tests). */
void listing_rhs(int kind, double p1, double p2, double p3, double eps, const double *y,
                 double *dy)
{
    lspec L;
    memset(&L, 0, sizeof L);
    if (kind == 1) mn_setup(&L, p1, p2, p3);
    else { L.M = p1; L.a = p2; L.Q = p3; }
    L.eps = eps;
    hamilton(&L, y, dy);
}
