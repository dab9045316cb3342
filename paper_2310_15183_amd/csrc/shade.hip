// Shading of traced frames: the background bands of the appendix listing's
// colour kernel and the exit-time map (arXiv 2310.15183, Sec. 4, the
// exit-time figures).  Streaming kernels: one pixel per thread, grid-stride,
// reading only the arrays the mode needs.  The decisions are taken in
// binary64 with the tracer's sin/cos, so colours are reproducible bit for bit.
//
// Colours are 32-bit words with bytes R, G, B, A in memory.

#include "internal.h"

namespace gr {
namespace {

constexpr uint32_t BLACK = 0xff000000u, CYAN = 0xffffff00u;

// Escaped rays: red where sin^2(phi) < 0.01, else green where
// cos^2(phi) < 0.01, else blue where sin^2(2 theta) < 0.01, else dark blue;
// all other rays black.
__device__ __forceinline__ uint32_t band_colour(double theta, double phi, int flag) {
    if (flag != GR_FLAG_ESCAPE) return BLACK;
    double sp, cp, s2t, c2t;
    sincos_def(phi, sp, cp);
    sincos_def(2.0 * theta, s2t, c2t);
    if (sp * sp < 0.01) return 0xff0000ffu;
    if (cp * cp < 0.01) return 0xff00ff00u;
    if (s2t * s2t < 0.01) return 0xffff0000u;
    return 0xff3c0000u;
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

template <int MODE>
__device__ __forceinline__ uint32_t colour(double t, double th, double ph, int f, double t_max,
                                           double band) {
    return MODE == 0 ? band_colour(th, ph, f) : time_colour(t, f, t_max, band);
}

// One pixel per thread and pass (any alignment).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) shade_kernel(const T* __restrict__ t,
                                                    const T* __restrict__ th,
                                                    const T* __restrict__ ph,
                                                    const int8_t* __restrict__ flag, int64_t n,
                                                    double t_max, double band,
                                                    uint32_t* __restrict__ rgba) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        rgba[k] = colour<MODE>(MODE == 1 ? (double)t[k] : 0.0, MODE == 0 ? (double)th[k] : 0.0,
                               MODE == 0 ? (double)ph[k] : 0.0, flag[k], t_max, band);
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
                                                       uint32_t* __restrict__ rgba) {
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t q = g; q < n4; q += stride) {
        const char4 f = reinterpret_cast<const char4*>(flag)[q];
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
        if (MODE == 0) {
            a = reinterpret_cast<const float4*>(th)[q];
            b = reinterpret_cast<const float4*>(ph)[q];
        } else {
            a = reinterpret_cast<const float4*>(t)[q];
        }
        uint4 c;
        c.x = colour<MODE>(a.x, a.x, b.x, f.x, t_max, band);
        c.y = colour<MODE>(a.y, a.y, b.y, f.y, t_max, band);
        c.z = colour<MODE>(a.z, a.z, b.z, f.z, t_max, band);
        c.w = colour<MODE>(a.w, a.w, b.w, f.w, t_max, band);
        reinterpret_cast<uint4*>(rgba)[q] = c;
    }
    const int64_t k = 4 * n4 + g;
    if (k < n)
        rgba[k] = colour<MODE>(MODE == 1 ? (double)t[k] : 0.0, MODE == 0 ? (double)th[k] : 0.0,
                               MODE == 0 ? (double)ph[k] : 0.0, flag[k], t_max, band);
}

bool aligned(const void* p, uintptr_t a) { return p == nullptr || (uintptr_t)p % a == 0; }

template <typename T>
hipError_t launch(int mode, const OutPtrs& o, int64_t n, double t_max, double band,
                  uint32_t* rgba, hipStream_t s) {
    const T* t = reinterpret_cast<const T*>(o.t);
    const T* th = reinterpret_cast<const T*>(o.th);
    const T* ph = reinterpret_cast<const T*>(o.ph);
    if constexpr (sizeof(T) == 4) {
        const bool vec = aligned(mode == 1 ? (const void*)t : (const void*)th, 16) &&
                         aligned(mode == 0 ? (const void*)ph : nullptr, 16) &&
                         aligned(o.flag, 4) && aligned(rgba, 16);
        if (vec) {
            const unsigned grid = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>((n / 4 + 255) / 256, 1 << 16));
            if (mode == 0)
                hipLaunchKernelGGL((shade_kernel_x4<0>), dim3(grid), dim3(256), 0, s, t, th, ph,
                                   o.flag, n, t_max, band, rgba);
            else
                hipLaunchKernelGGL((shade_kernel_x4<1>), dim3(grid), dim3(256), 0, s, t, th, ph,
                                   o.flag, n, t_max, band, rgba);
            return hipGetLastError();
        }
    }
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16);
    if (mode == 0)
        hipLaunchKernelGGL((shade_kernel<T, 0>), dim3(grid), dim3(256), 0, s, t, th, ph, o.flag,
                           n, t_max, band, rgba);
    else
        hipLaunchKernelGGL((shade_kernel<T, 1>), dim3(grid), dim3(256), 0, s, t, th, ph, o.flag,
                           n, t_max, band, rgba);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_shade(int mode, const OutPtrs& o, bool f32, int64_t n, double t_max,
                        double band, uint32_t* rgba, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return f32 ? launch<float>(mode, o, n, t_max, band, rgba, s)
               : launch<double>(mode, o, n, t_max, band, rgba, s);
}

}  // namespace gr
