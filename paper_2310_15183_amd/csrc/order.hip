// Queue order of a frame for the persistent tracers: near-critical rays,
// the longest, first, so that the queue does not end on them.  Host wrapper
// and the key kernel; the sort is hipCUB's radix sort.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace gr {
namespace {

// key[k] = |b - b_crit| of pixel k's camera ray, with E = -p_t, L = p_phi and
// Carter's constant Q = p_theta^2 + cos^2(theta0) (L^2/sin^2(theta0) - a^2 E^2).
__global__ void order_keys_kernel(const Hole H, const Camera C, double b_crit, int64_t n,
                                  double s2, double c2, float* __restrict__ key,
                                  int32_t* __restrict__ val) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double pt, pr, pth, pph;
    camera_ray(C, k % C.W, k / C.W, pt, pr, pth, pph);
    const double E = -pt, L = pph;
    const double Q = fma(pth, pth, c2 * (L * L / s2 - H.a2 * E * E));
    const double b = sqrt(fmax(Q + L * L, 0.0)) / fabs(E);
    key[k] = (float)fabs(b - b_crit);
    val[k] = (int32_t)k;
}

}  // namespace

size_t frame_order_temp(int64_t npix) {
    size_t bytes = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const float*)nullptr, (float*)nullptr,
                                       (const int32_t*)nullptr, (int32_t*)nullptr, (int)npix);
    return bytes;
}

hipError_t frame_order(const Hole& H, const Camera& C, double b_crit, int64_t npix, float* keys,
                       int32_t* vals, void* temp, size_t temp_bytes, hipStream_t s) {
    double sn, cs;
    sincos_def(C.th0, sn, cs);
    const unsigned grid = (unsigned)((npix + 255) / 256);
    hipLaunchKernelGGL(order_keys_kernel, dim3(grid), dim3(256), 0, s, H, C, b_crit, npix,
                       sn * sn, cs * cs, keys, vals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys + npix, vals,
                                              vals + npix, (int)npix, 0, 32, s);
}

}  // namespace gr
