// Per-ray kernels of the learned surrogate: network inputs, training targets,
// and the frame pipeline (class and direction from the network, fallback
// marking, merge of the rays re-traced with RK4).
//
// Inputs of a ray (7): pixel angles alpha = atan(x), beta = atan(y) of its
// image-plane coordinates, a/M, |Q|/M, theta0, r0/(50 M), fov (M = 1 for flat
// space).  The network's direction output is a correction d to a baseline
// u_base: where the same camera ray would cross the escape sphere
// r = escape_factor * r0 around the Reissner-Nordstrom hole with the same M
// and Q (no spin: the ray stays in a plane and its sweep is a 1-D integral),
// or, for rays that hole captures, where the straight line of flat space
// leaves the sphere; the end direction is normalise(u_base + d).  Close to
// the critical impact parameter b_c the sweep diverges and the spin moves
// the shadow, so the frame pipeline can re-trace escaping rays with
// b < min_impact b_c instead of trusting the network there.  Targets use the traced
// ray's crossing of the same sphere (its end state moved back along its own
// velocity to r_esc).
#include "internal.h"
#include "mlp_internal.h"
#include "step_fp64.h"
#include "surrogate_internal.h"

namespace gr {
namespace sur {
namespace {

__device__ __forceinline__ int find_inst(const int64_t* firsts, int ninst, int64_t id) {
    int lo = 0, hi = ninst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (firsts[mid] <= id) lo = mid; else hi = mid;
    }
    return lo;
}

// ---- Reissner-Nordstrom baseline of the end direction
// Gauss-Legendre 16-point rule on [-1, 1]: nodes +-GLX[k], weights GLW[k]
// (roots of the Legendre polynomial P_16 and their weights).
__device__ constexpr double GLX[8] = {
    0x1.852bd6676a9fap-4, 0x1.205cae642337cp-2, 0x1.d50259a43a772p-2, 0x1.3c5a466d5e8b8p-1,
    0x1.82c45dda4726bp-1, 0x1.bb3403514e483p-1, 0x1.e39f56616f9b0p-1, 0x1.fa92c264d787ep-1};
__device__ constexpr double GLW[8] = {
    0x1.83feae80e4dffp-3, 0x1.75f8c77e0c010p-3, 0x1.5a6ebbb5a75ffp-3, 0x1.325f61bca3cc0p-3,
    0x1.fe7af2bad3875p-4, 0x1.85c4ee79cc24ap-4, 0x1.fdfb1a2c12642p-5, 0x1.bcddab4b7c200p-6};

// Azimuth swept by an equatorial photon of the Reissner-Nordstrom hole (M,
// Q^2) with impact parameter b that starts inward at u0 = 1/r0, turns at its
// periapsis u_t and leaves to u1 = 1/r1.  With u = 1/r the orbit obeys
// (du/dphi)^2 = F(u) = 1/b^2 - u^2 + 2 M u^3 - Q^2 u^4; u_t is the root of F
// below the photon sphere u_ph (where dF/du = 0), which exists when b exceeds
// the critical impact parameter b_c (rn_turn).  The substitution u = u_t - s^2
// gives F = s^2 G(s), G the Taylor polynomial of F about u_t divided by -s^2,
// and dphi = 2 ds / sqrt(G(s)), integrated from 0 to sqrt(u_t - u) for each
// leg (rn_leg) by 16-point Gauss-Legendre; the sweep is rn_leg(u0) + rn_leg(u1).
struct RnTurn {
    double ut, g0, g1, g2, g3;          // turning point and G's coefficients in s^2
};

// u_t starts from the Schwarzschild periapsis of a hole whose photon sphere
// and critical impact parameter are those of (M, Q^2) -- the trigonometric
// root 1/u = 2 r_ph b_rel cos(arccos(-1/b_rel)/3) of the cubic, b_rel = b/b_c,
// exact for Q = 0 up to binary32 rounding -- and takes four Newton steps on F
// (relative error below 1e-12 for b_rel > 1 + 1e-6 and |Q| < M).  False when
// the photon does not turn outside the photon sphere.
__device__ bool rn_turn(const SurConst& S, double b, double b_rel, RnTurn& T) {
    const double M = S.M, Q2 = S.Q2;
    double ut;
    if (M == 0.0 && Q2 == 0.0) {
        if (!(b > 0.0)) return false;
        ut = 1.0 / b;                                   // straight line
    } else {
        if (!(b_rel > 1.0) || !(S.u0 < S.uph)) return false;
        const float c = cosf(acosf(-1.0f / (float)b_rel) * (1.0f / 3.0f));
        double u = (0.5 * S.uph) / (b_rel * (double)c);
        u = fmin(fmax(u, S.u0), S.uph);
        const double ib2 = 1.0 / (b * b);
        for (int it = 0; it < 4; ++it) {
            const double F = ib2 + u * u * (-1.0 + u * (2.0 * M - Q2 * u));
            const double dF = u * (-2.0 + u * (6.0 * M - 4.0 * Q2 * u));
            u -= F / dF;
        }
        ut = u;
    }
    // derivatives of F at u_t (first to fourth)
    const double F1 = ut * (-2.0 + ut * (6.0 * M - 4.0 * Q2 * ut));
    const double F2 = -2.0 + ut * (12.0 * M - 12.0 * Q2 * ut);
    const double F3 = 12.0 * M - 24.0 * Q2 * ut;
    const double F4 = -24.0 * Q2;
    T.ut = ut;
    T.g0 = -F1;
    T.g1 = 0.5 * F2;
    T.g2 = -F3 / 6.0;
    T.g3 = F4 / 24.0;
    return T.g0 > 0.0 && ut > S.u0;
}

// One leg; G in binary64, 1/sqrt(G) and the weighted sum in binary32 (the
// baseline is rounded to binary32 and its error only has to be small against
// the network's).
__device__ double rn_leg(const RnTurn& T, double u_end) {
    const double w = T.ut - u_end;
    if (!(w > 0.0)) return 0.0;
    const double half = 0.5 * sqrt(w);
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const double sk = half * (1.0 + sgn * GLX[k]);
            const double z = sk * sk;
            const double G = T.g0 + z * (T.g1 + z * (T.g2 + z * T.g3));
            acc += (float)GLW[k] * rsqrtf((float)G);
        }
    }
    return half * 2.0 * (double)acc;
}

// Everything about a pixel's ray but the sweep integrals: the features, the
// straight-line baseline, the orbit plane and the Reissner-Nordstrom turning
// point (turns: whether there is one outside the photon sphere).
struct RayGeom {
    float x[7];
    double flat[3];                   // straight-line crossing of the escape sphere
    double e[3], t[3];                // x0 / r0 and the tangential unit of the orbit plane
    double u0, u1;                    // 1/r0, 1/r_esc
    float b_rel;                      // impact parameter over the critical one (inf: flat space)
    bool turns;
    RnTurn T;
};

__device__ void ray_geom(const BatchInstance& I, int64_t pix, RayGeom& G) {
    const Camera& C = I.cam;
    const SurConst& S = I.sur;
    const int64_t i = pix % C.W, j = pix / C.W;
    const double xs = ((double)(2 * i + 1 - C.W) / (double)C.W) * C.tan_h;
    const double ys = ((double)(C.H - 2 * j - 1) / (double)C.H) * C.tan_v;
    G.x[0] = atanf((float)xs);
    G.x[1] = atanf((float)ys);
    for (int c = 0; c < 5; ++c) G.x[2 + c] = S.feat[c];
    // the camera ray's line of sight n = (-1, -y, x) in (e_r, e_theta, e_phi)
    const double inv = 1.0 / sqrt(1.0 + xs * xs + ys * ys);
    const double nr = -inv, nt = -ys * inv, np = xs * inv;
    const double d0 = nr * S.st * S.cp + nt * S.ct * S.cp - np * S.sp;
    const double d1 = nr * S.st * S.sp + nt * S.ct * S.sp + np * S.cp;
    const double d2 = nr * S.ct - nt * S.st;
    G.e[0] = S.st * S.cp;
    G.e[1] = S.st * S.sp;
    G.e[2] = S.ct;
    // flat space: the straight line's crossing of the escape sphere
    const double bb = S.r0 * nr;                      // x0 . d
    const double s = -bb + sqrt(bb * bb - (S.r0 * S.r0 - S.R * S.R));
    G.flat[0] = (S.r0 * G.e[0] + s * d0) * S.u1;
    G.flat[1] = (S.r0 * G.e[1] + s * d1) * S.u1;
    G.flat[2] = (S.r0 * G.e[2] + s * d2) * S.u1;
    // the orbit plane of x0 and the initial direction, impact parameter
    // b = r0 sin(alpha)/sqrt(f(r0)) for a static observer
    const double tt = sqrt(nt * nt + np * np);        // sin(alpha)
    const double b = S.bscale * tt;
    const double b_rel = b * S.inv_bc;
    G.b_rel = S.inv_bc > 0.0 ? (float)b_rel : INFINITY;
    G.u0 = S.u0;
    G.u1 = S.u1;
    G.turns = tt > 0.0 && rn_turn(S, b, b_rel, G.T);
    if (G.turns) {
        const double it = 1.0 / tt;
        G.t[0] = (nt * S.ct * S.cp - np * S.sp) * it;
        G.t[1] = (nt * S.ct * S.sp + np * S.cp) * it;
        G.t[2] = (-nt * S.st) * it;
    }
}

// Baseline from the geometry and the sweep (rn_leg(u0) + rn_leg(u1)): the
// Reissner-Nordstrom crossing when the ray turns, else the straight line.
__device__ void ray_baseline(const RayGeom& G, double sweep, float* u) {
    if (G.turns && isfinite(sweep)) {
        const double cs = cos(sweep), sn = sin(sweep);
        for (int c = 0; c < 3; ++c) u[c] = (float)(cs * G.e[c] + sn * G.t[c]);
    } else {
        for (int c = 0; c < 3; ++c) u[c] = (float)G.flat[c];
    }
}

// Features x (7) and baseline u (3) of pixel pix; b_rel (may be null)
// receives the ray's impact parameter over the critical one.
__device__ void ray_inputs(const BatchInstance& I, int64_t pix, float* x, float* u,
                           float* b_rel = nullptr) {
    RayGeom G;
    ray_geom(I, pix, G);
    double sweep = 0.0;
    if (G.turns) {
        sweep += rn_leg(G.T, G.u0);
        sweep += rn_leg(G.T, G.u1);
    }
    ray_baseline(G, sweep, u);
    for (int c = 0; c < 7; ++c) x[c] = G.x[c];
    if (b_rel) *b_rel = G.b_rel;
}

template <typename T>
__device__ __forceinline__ double rd(const void* p, int64_t k) {
    return (double)reinterpret_cast<const T*>(p)[k];
}

// Unit vector where an escaped ray crossed r = r_esc.
__device__ void escape_direction(const BatchInstance& I, int64_t k, float* u) {
    const OutPtrs& o = I.out;
    double th, ph, r, pt, pr, pth, pph;
    if (I.f32) {
        th = rd<float>(o.th, k); ph = rd<float>(o.ph, k); r = rd<float>(o.r, k);
        pt = rd<float>(o.pt, k); pr = rd<float>(o.pr, k); pth = rd<float>(o.pth, k);
        pph = rd<float>(o.pph, k);
    } else {
        th = rd<double>(o.th, k); ph = rd<double>(o.ph, k); r = rd<double>(o.r, k);
        pt = rd<double>(o.pt, k); pr = rd<double>(o.pr, k); pth = rd<double>(o.pth, k);
        pph = rd<double>(o.pph, k);
    }
    const Hole& H = I.hole;
    const double s = sin(th), c = cos(th);
    const double s2 = s * s, c2 = c * c;
    const double rho2 = r * r + H.a2 * c2;
    const double Delta = r * r - H.M2 * r + H.aq;
    const double grr = Delta / rho2, ghh = 1.0 / rho2;
    const double gtp = -H.a * (H.M2 * r - H.Q2) / (rho2 * Delta);
    const double gpp = (Delta - H.a2 * s2) / (rho2 * Delta * s2);
    const double lam = (I.r_esc - r) / (grr * pr);
    const double thx = th + ghh * pth * lam;
    const double phx = ph + (gtp * pt + gpp * pph) * lam;
    u[0] = (float)(sin(thx) * cos(phx));
    u[1] = (float)(sin(thx) * sin(phx));
    u[2] = (float)cos(thx);
}

__global__ void inputs_kernel(const BatchInstance* __restrict__ inst,
                              const int64_t* __restrict__ firsts, int ninst, int64_t total,
                              float* __restrict__ x, float* __restrict__ uflat) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int q = find_inst(firsts, ninst, id);
    const BatchInstance& I = inst[q];
    const int64_t k = id - firsts[q];
    const int64_t pix = I.pixels ? (int64_t)I.pixels[k] : k;
    ray_inputs(I, pix, x + id * 7, uflat + id * 3);
}

__global__ void targets_kernel(const BatchInstance* __restrict__ inst,
                               const int64_t* __restrict__ firsts, int ninst, int64_t total,
                               const float* __restrict__ uflat, float* __restrict__ target) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= total) return;
    const int q = find_inst(firsts, ninst, id);
    const BatchInstance& I = inst[q];
    const int64_t k = id - firsts[q];
    float* t = target + id * 4;
    if (I.out.flag[k] == GR_FLAG_ESCAPE) {
        float u[3];
        escape_direction(I, k, u);
        t[0] = 1.0f;
        for (int c = 0; c < 3; ++c) t[1 + c] = u[c] - uflat[id * 3 + c];
    } else {
        t[0] = t[1] = t[2] = t[3] = 0.0f;
    }
}

// ---- fused frame kernel: inputs, the five layers and the class/direction of
// FR consecutive pixels per workgroup.  The activations of the FR rays stay
// in LDS (one row of HID bfloat16 per ray, padded by 8 values so that the 16
// rows read by one MFMA operand fall in distinct banks); wave w computes the
// output features 64 w .. 64 w + 63 of every layer for all FR rays as
// D[feature][ray] = W^T (A fragments read from global memory, see
// mlp::pack_kernel) times the activations (B operand from LDS), with
// binary32 accumulation in the same k order as the training kernels.
constexpr int FR = 128;                  // rays per workgroup
constexpr int LDA = mlp::HID + 8;        // bfloat16 per LDS activation row
constexpr int FRAME_THREADS = 256;

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf4;

// One SiLU layer of mlp::HID outputs over KS k-steps of 32 inputs, in place.
template <int KS>
__device__ __forceinline__ void frame_layer(__bf16* act, const __bf16* __restrict__ frag,
                                            const float* __restrict__ bias, int wave, int lane) {
    f4 acc[4][FR / 16];
    for (int i = 0; i < 4; ++i)
        for (int t = 0; t < FR / 16; ++t) acc[i][t] = f4{0.f, 0.f, 0.f, 0.f};
    const bf8* A = reinterpret_cast<const bf8*>(frag);
    const int rn = lane & 15, kq = (lane >> 4) * 8;
    // the A fragments of the next k-step load while this one's products run
    bf8 an[4];
    for (int i = 0; i < 4; ++i) an[i] = A[((4 * wave + i) * KS + 0) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        bf8 a[4];
        for (int i = 0; i < 4; ++i) a[i] = an[i];
        if (ks + 1 < KS)
            for (int i = 0; i < 4; ++i) an[i] = A[((4 * wave + i) * KS + ks + 1) * 64 + lane];
        for (int t = 0; t < FR / 16; ++t) {
            const bf8 b =
                *reinterpret_cast<const bf8*>(act + (16 * t + rn) * LDA + 32 * ks + kq);
            for (int i = 0; i < 4; ++i)
                acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][t], 0, 0, 0);
        }
    }
    __syncthreads();                       // every wave has read this layer's inputs
    // lane holds features f .. f + 3 (f = 16 (4 wave + i) + 4 (lane / 16)) of ray 16 t + lane % 16
    for (int i = 0; i < 4; ++i) {
        const int f = 16 * (4 * wave + i) + 4 * (lane >> 4);
        const f4 bb = *reinterpret_cast<const f4*>(bias + f);
        for (int t = 0; t < FR / 16; ++t) {
            bf4 h;
            for (int e = 0; e < 4; ++e) {
                const float z = acc[i][t][e] + bb[e];
                h[e] = (__bf16)(z * mlp::sigmoid_hw(z));
            }
            *reinterpret_cast<bf4*>(act + (16 * t + rn) * LDA + f) = h;
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(FRAME_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
frame_net_kernel(const BatchInstance I, int64_t npix, const mlp::NetView net, float min_impact,
                 int8_t* __restrict__ flag, float* __restrict__ dir, float* __restrict__ logit) {
    __shared__ __attribute__((aligned(16))) __bf16 act[FR * LDA];
    __shared__ float uf[FR][3];
    __shared__ float brel[FR];
    __shared__ double legsum[FR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * FR;

    // network inputs: two threads per pixel, each integrating one leg of the
    // sweep (summed in the same order as ray_inputs); rows past the frame are zero
    {
        const int px = tid % FR, leg = tid / FR;
        const bool inside = p0 + px < npix;
        RayGeom G;
        double part = 0.0;
        if (inside) {
            ray_geom(I, p0 + px, G);
            if (G.turns) part = rn_leg(G.T, leg ? G.u1 : G.u0);
        }
        if (leg) legsum[px] = part;
        __syncthreads();
        if (!leg) {
            float u[3] = {0.f, 0.f, 0.f};
            __bf16* row = act + px * LDA;
            brel[px] = inside ? G.b_rel : INFINITY;
            if (inside) {
                double sweep = 0.0;
                if (G.turns) {
                    sweep += part;
                    sweep += legsum[px];
                }
                ray_baseline(G, sweep, u);
            }
            for (int c = 0; c < mlp::IN_PAD; ++c)
                row[c] = (inside && c < mlp::IN) ? (__bf16)G.x[c] : (__bf16)0.0f;
            for (int c = 0; c < 3; ++c) uf[px][c] = u[c];
        }
    }
    __syncthreads();
    frame_layer<mlp::IN_PAD / 32>(act, net.frag[0], net.bias[0], wave, lane);
    frame_layer<mlp::HID / 32>(act, net.frag[1], net.bias[1], wave, lane);
    frame_layer<mlp::HID / 32>(act, net.frag[2], net.bias[2], wave, lane);
    frame_layer<mlp::HID / 32>(act, net.frag[3], net.bias[3], wave, lane);

    // output layer: one 16-feature tile (features 0..3 real); wave w takes rays 32 w .. 32 w + 31
    const bf8* A = reinterpret_cast<const bf8*>(net.frag[4]);
    const int rn = lane & 15, kq = (lane >> 4) * 8;
    f4 acc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int ks = 0; ks < mlp::HID / 32; ++ks) {
        const bf8 a = A[ks * 64 + lane];
        for (int t = 0; t < 2; ++t) {
            const bf8 b =
                *reinterpret_cast<const bf8*>(act + (32 * wave + 16 * t + rn) * LDA + 32 * ks + kq);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
    if (lane < 16) {                       // lanes 0..15 hold features 0..3 of their ray
        const float* bo = net.bias[4];
        for (int t = 0; t < 2; ++t) {
            const int ray = 32 * wave + 16 * t + lane;
            const int64_t p = p0 + ray;
            if (p >= npix) continue;
            const float y0 = acc[t][0] + bo[0];
            const bool esc = y0 > 0.0f;
            float u[3];
            float nn = 0.0f;
            for (int c = 0; c < 3; ++c) {
                u[c] = uf[ray][c] + (acc[t][1 + c] + bo[1 + c]);
                nn += u[c] * u[c];
            }
            const float inv = esc && nn > 0.0f ? 1.0f / sqrtf(nn) : 0.0f;
            flag[p] = esc ? GR_FLAG_ESCAPE : GR_FLAG_HORIZON;
            for (int c = 0; c < 3; ++c) dir[p * 3 + c] = u[c] * inv;
            // an escaping ray too close to the critical impact parameter gets a
            // NaN logit, which the fallback selection always re-traces
            logit[p] = esc && brel[ray] < min_impact ? NAN : y0;
        }
    }
}

// A pixel falls back to RK4 when its logit is small, a pixel within
// Chebyshev distance `edge` has the other class, or (max_chord2 > 0) an
// escaping pixel and an escaping 8-neighbour have predicted directions more
// than sqrt(max_chord2) apart (chord of unit vectors): the image is strongly
// magnified there and the network's direction least reliable.  Fallback
// pixels are appended to list with one atomic per wave (order unspecified).
__global__ void fallback_kernel(const float* __restrict__ logit, const int8_t* __restrict__ flag,
                                const float* __restrict__ dir, int32_t W, int32_t H,
                                float logit_min, int32_t edge, float max_chord2,
                                int8_t* __restrict__ fb, int32_t* __restrict__ list,
                                unsigned long long* __restrict__ count) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool f = false;
    if (p < (int64_t)W * H) {
        const int i = (int)(p % W), j = (int)(p / W);
        f = !(fabsf(logit[p]) >= logit_min);          // NaN: always
        const int8_t mine = flag[p];
        for (int dj = -edge; dj <= edge && !f; ++dj) {
            const int jj = j + dj;
            if (jj < 0 || jj >= H) continue;
            for (int di = -edge; di <= edge; ++di) {
                const int ii = i + di;
                if (ii < 0 || ii >= W) continue;
                if (flag[(int64_t)jj * W + ii] != mine) {
                    f = true;
                    break;
                }
            }
        }
        if (!f && max_chord2 > 0.0f && mine == GR_FLAG_ESCAPE) {
            const float u0 = dir[p * 3], u1 = dir[p * 3 + 1], u2 = dir[p * 3 + 2];
            for (int dj = -1; dj <= 1 && !f; ++dj) {
                const int jj = j + dj;
                if (jj < 0 || jj >= H) continue;
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di;
                    if (ii < 0 || ii >= W) continue;
                    const int64_t q = (int64_t)jj * W + ii;
                    if (flag[q] != GR_FLAG_ESCAPE) continue;
                    const float d0 = dir[q * 3] - u0, d1 = dir[q * 3 + 1] - u1,
                                d2 = dir[q * 3 + 2] - u2;
                    if ((d0 * d0 + d1 * d1) + d2 * d2 > max_chord2) {
                        f = true;
                        break;
                    }
                }
            }
        }
        fb[p] = f ? 1 : 0;
    }
    const int64_t slot = detail::take_ids(f, count);     // every lane of the wave takes part
    if (f) list[slot] = (int32_t)p;
}

// Results of the re-traced pixels replace the network's; the number of
// fallback pixels is read from the device (grid-stride over it).
__global__ void merge_kernel(const BatchInstance* __restrict__ inst, const int32_t* __restrict__ list,
                             const unsigned long long* __restrict__ count, int8_t* __restrict__ flag,
                             float* __restrict__ dir) {
    const int64_t n = (int64_t)*count;
    const BatchInstance& I = inst[0];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = list[k];
        const int8_t f = I.out.flag[k];
        flag[p] = f;
        float u[3] = {0.f, 0.f, 0.f};
        if (f == GR_FLAG_ESCAPE) escape_direction(I, k, u);
        for (int c = 0; c < 3; ++c) dir[p * 3 + c] = u[c];
    }
}

// Prefix offsets of a one-instance batch whose size is the fallback count.
__global__ void set_firsts_kernel(const unsigned long long* __restrict__ count,
                                  int64_t* __restrict__ firsts) {
    firsts[0] = 0;
    firsts[1] = (int64_t)*count;
}

__global__ void zero_u64(unsigned long long* c) { *c = 0ull; }

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t inputs(const BatchInstance* inst, const int64_t* firsts, int ninst, int64_t total,
                  float* x, float* uflat, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(inputs_kernel, dim3(blocks(total)), dim3(256), 0, s, inst, firsts, ninst,
                       total, x, uflat);
    return hipGetLastError();
}

hipError_t targets(const BatchInstance* inst, const int64_t* firsts, int ninst, int64_t total,
                   const float* uflat, float* target, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(targets_kernel, dim3(blocks(total)), dim3(256), 0, s, inst, firsts, ninst,
                       total, uflat, target);
    return hipGetLastError();
}

hipError_t frame_net(const BatchInstance& I, int64_t npix, const mlp::NetView& net,
                     float min_impact, int8_t* flag, float* dir, float* logit, hipStream_t s) {
    if (npix <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((npix + FR - 1) / FR);
    hipLaunchKernelGGL(frame_net_kernel, dim3(grid), dim3(FRAME_THREADS), 0, s, I, npix, net,
                       min_impact, flag, dir, logit);
    return hipGetLastError();
}

hipError_t fallback(const float* logit, const int8_t* flag, const float* dir, int32_t W,
                    int32_t H, float logit_min, int32_t edge, float max_chord2, int8_t* fb,
                    int32_t* list, unsigned long long* count, hipStream_t s) {
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, count);
    hipLaunchKernelGGL(fallback_kernel, dim3(blocks((int64_t)W * H)), dim3(256), 0, s, logit, flag,
                       dir, W, H, logit_min, edge, max_chord2, fb, list, count);
    return hipGetLastError();
}

hipError_t set_firsts(const unsigned long long* count, int64_t* firsts, hipStream_t s) {
    hipLaunchKernelGGL(set_firsts_kernel, dim3(1), dim3(1), 0, s, count, firsts);
    return hipGetLastError();
}

hipError_t merge(const BatchInstance* inst, const int32_t* list, const unsigned long long* count,
                 int64_t max_n, int8_t* flag, float* dir, hipStream_t s) {
    if (max_n <= 0) return hipSuccess;
    const unsigned grid = blocks(max_n) < 2048u ? blocks(max_n) : 2048u;
    hipLaunchKernelGGL(merge_kernel, dim3(grid), dim3(256), 0, s, inst, list, count, flag, dir);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace gr
