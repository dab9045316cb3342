// Shading of traced frames (arXiv 2310.15183, Sec. 4): the three lines on
// the sky of the exit-position figures, the exit-time map and the bilinearly
// filtered sky texture.  Streaming kernels: one pixel per thread,
// grid-stride, reading only the arrays the mode needs.  The decisions are
// taken in binary64 with the tracer's sin/cos, so colours are reproducible
// bit for bit.
//
// Colours are 32-bit words with bytes R, G, B, A in memory.

#include "internal.h"

namespace gr {
namespace {

constexpr uint32_t BLACK = 0xff000000u, CYAN = 0xffffff00u, SKY = 0xff3c0000u;

// The lines on the sky, in order of precedence where they cross: each is a
// narrow interval of one angle of the ray's end position, drawn where the
// square of the sine (or cosine) of that angle is below LINE_SIN2.
enum { ANGLE_PHI = 0, ANGLE_TWO_THETA = 1 };
struct SkyLine {
    int angle;       // ANGLE_PHI or ANGLE_TWO_THETA
    bool cosine;     // test the cosine (a line at +-pi/2) instead of the sine
    uint32_t rgba;
};
constexpr SkyLine LINES[3] = {
    {ANGLE_PHI, false, 0xff0000ffu},        // red: the meridian through the camera, phi = 0, pi
    {ANGLE_PHI, true, 0xff00ff00u},         // green: the meridian across the view, phi = +-pi/2
    {ANGLE_TWO_THETA, false, 0xffff0000u},  // light blue: the equator (2 theta also marks the poles)
};
constexpr double LINE_SIN2 = 0.01;

__device__ __forceinline__ uint32_t band_colour(double theta, double phi, int flag) {
    if (flag != GR_FLAG_ESCAPE) return BLACK;
    double sc[2][2];
    sincos_def(phi, sc[ANGLE_PHI][0], sc[ANGLE_PHI][1]);
    sincos_def(2.0 * theta, sc[ANGLE_TWO_THETA][0], sc[ANGLE_TWO_THETA][1]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = sc[LINES[k].angle][LINES[k].cosine ? 1 : 0];
        if (v * v < LINE_SIN2) return LINES[k].rgba;
    }
    return SKY;
}

// Equirectangular sky texture (tw x th, row 0 at theta = 0, column 0 at
// phi = 0), bilinear filtering at the end direction: theta brought into
// [0, pi] (mod 2 pi, reflected above pi with phi turned by pi), texel
// coordinates x = frac(phi / 2 pi) tw - 1/2 and y = theta / pi th - 1/2,
// columns wrapping, rows clamped; per channel a = fma(fx, c10 - c00, c00),
// b = fma(fx, c11 - c01, c01), c = fma(fy, b - a, a), byte floor(c + 1/2).
__device__ __forceinline__ uint32_t texture_colour(double theta, double phi, int flag,
                                                   const uint32_t* __restrict__ tex, int tw,
                                                   int th) {
    if (flag != GR_FLAG_ESCAPE) return BLACK;
    const double two_pi = 4.0 * PI2_HI, pi = 2.0 * PI2_HI;
    double t = theta - two_pi * floor(theta / two_pi);
    double p = phi;
    if (t > pi) {
        t = two_pi - t;
        p = p + pi;
    }
    double u = p / two_pi;
    u = u - floor(u);
    const double x = u * (double)tw - 0.5, y = (t / pi) * (double)th - 0.5;
    const double xf = floor(x), yf = floor(y);
    const double fx = x - xf, fy = y - yf;
    int64_t i0 = (int64_t)xf % tw;
    if (i0 < 0) i0 += tw;
    const int64_t i1 = i0 + 1 == tw ? 0 : i0 + 1;
    const int64_t j = (int64_t)yf;
    const int64_t j0 = j < 0 ? 0 : (j > th - 1 ? th - 1 : j);
    const int64_t j1 = j + 1 < 0 ? 0 : (j + 1 > th - 1 ? th - 1 : j + 1);
    const uint32_t q00 = tex[j0 * tw + i0], q10 = tex[j0 * tw + i1];
    const uint32_t q01 = tex[j1 * tw + i0], q11 = tex[j1 * tw + i1];
    uint32_t out = 0;
#pragma unroll
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

// tau = |t|: escaped rays with tau < t_max from dark blue to cyan,
// level = floor(255 tau / t_max), dimmed to 7/8 on every other band of width
// `band` (band > 0); rays that did not escape and tau >= t_max cyan; invalid
// rays black.
__device__ __forceinline__ uint32_t time_colour(double t, int flag, double t_max, double band) {
    if (flag == GR_FLAG_INVALID) return BLACK;
    if (flag != GR_FLAG_ESCAPE) return CYAN;
    const double tau = fabs(t);
    const double u = tau / t_max;
    if (!(u < 1.0)) return CYAN;
    uint32_t level = (uint32_t)(u * 255.0);
    if (band > 0.0 && (((int64_t)(tau / band)) & 1)) level = (level * 7u) / 8u;
    const uint32_t blue = 64u + (level * 191u) / 255u;
    return 0xff000000u | (blue << 16) | (level << 8);
}

struct Tex {
    const uint32_t* p;
    int w, h;
};

template <int MODE>
__device__ __forceinline__ uint32_t colour(double t, double th, double ph, int f, double t_max,
                                           double band, const Tex& tx) {
    if (MODE == 0) return band_colour(th, ph, f);
    if (MODE == 2) return texture_colour(th, ph, f, tx.p, tx.w, tx.h);
    return time_colour(t, f, t_max, band);
}

// One pixel per thread and pass (any alignment).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) shade_kernel(const T* __restrict__ t,
                                                    const T* __restrict__ th,
                                                    const T* __restrict__ ph,
                                                    const int8_t* __restrict__ flag, int64_t n,
                                                    double t_max, double band, Tex tx,
                                                    uint32_t* __restrict__ rgba) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        rgba[k] = colour<MODE>(MODE == 1 ? (double)t[k] : 0.0, MODE != 1 ? (double)th[k] : 0.0,
                               MODE != 1 ? (double)ph[k] : 0.0, flag[k], t_max, band, tx);
    }
}

// Binary32 inputs, four pixels per thread and pass with 16-byte loads and
// stores (all arrays 16-byte aligned, the flags 4-byte); the last n % 4
// pixels by the first threads.
template <int MODE>
__global__ void __launch_bounds__(256) shade_kernel_x4(const float* __restrict__ t,
                                                       const float* __restrict__ th,
                                                       const float* __restrict__ ph,
                                                       const int8_t* __restrict__ flag,
                                                       int64_t n, double t_max, double band,
                                                       Tex tx, uint32_t* __restrict__ rgba) {
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t q = g; q < n4; q += stride) {
        const char4 f = reinterpret_cast<const char4*>(flag)[q];
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
        if (MODE != 1) {
            a = reinterpret_cast<const float4*>(th)[q];
            b = reinterpret_cast<const float4*>(ph)[q];
        } else {
            a = reinterpret_cast<const float4*>(t)[q];
        }
        uint4 c;
        c.x = colour<MODE>(a.x, a.x, b.x, f.x, t_max, band, tx);
        c.y = colour<MODE>(a.y, a.y, b.y, f.y, t_max, band, tx);
        c.z = colour<MODE>(a.z, a.z, b.z, f.z, t_max, band, tx);
        c.w = colour<MODE>(a.w, a.w, b.w, f.w, t_max, band, tx);
        reinterpret_cast<uint4*>(rgba)[q] = c;
    }
    const int64_t k = 4 * n4 + g;
    if (k < n)
        rgba[k] = colour<MODE>(MODE == 1 ? (double)t[k] : 0.0, MODE != 1 ? (double)th[k] : 0.0,
                               MODE != 1 ? (double)ph[k] : 0.0, flag[k], t_max, band, tx);
}

bool aligned(const void* p, uintptr_t a) { return p == nullptr || (uintptr_t)p % a == 0; }

template <typename T, int MODE>
hipError_t launch_mode(const OutPtrs& o, int64_t n, double t_max, double band, const Tex& tx,
                       uint32_t* rgba, hipStream_t s) {
    const T* t = reinterpret_cast<const T*>(o.t);
    const T* th = reinterpret_cast<const T*>(o.th);
    const T* ph = reinterpret_cast<const T*>(o.ph);
    if constexpr (sizeof(T) == 4) {
        const bool vec = aligned(MODE == 1 ? (const void*)t : (const void*)th, 16) &&
                         aligned(MODE != 1 ? (const void*)ph : nullptr, 16) &&
                         aligned(o.flag, 4) && aligned(rgba, 16);
        if (vec) {
            const unsigned grid = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>((n / 4 + 255) / 256, 1 << 16));
            hipLaunchKernelGGL((shade_kernel_x4<MODE>), dim3(grid), dim3(256), 0, s, t, th, ph,
                               o.flag, n, t_max, band, tx, rgba);
            return hipGetLastError();
        }
    }
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL((shade_kernel<T, MODE>), dim3(grid), dim3(256), 0, s, t, th, ph, o.flag,
                       n, t_max, band, tx, rgba);
    return hipGetLastError();
}

template <typename T>
hipError_t launch(int mode, const OutPtrs& o, int64_t n, double t_max, double band,
                  const Tex& tx, uint32_t* rgba, hipStream_t s) {
    if (mode == 0) return launch_mode<T, 0>(o, n, t_max, band, tx, rgba, s);
    if (mode == 2) return launch_mode<T, 2>(o, n, t_max, band, tx, rgba, s);
    return launch_mode<T, 1>(o, n, t_max, band, tx, rgba, s);
}

}  // namespace

hipError_t launch_shade(int mode, const OutPtrs& o, bool f32, int64_t n, double t_max,
                        double band, const uint32_t* texture, int tex_w, int tex_h,
                        uint32_t* rgba, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const Tex tx{texture, tex_w, tex_h};
    return f32 ? launch<float>(mode, o, n, t_max, band, tx, rgba, s)
               : launch<double>(mode, o, n, t_max, band, tx, rgba, s);
}

}  // namespace gr
