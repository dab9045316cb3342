// Queue order of a frame for the persistent tracers: near-critical rays,
// the longest, first, so that the queue does not end on them.  A counting
// sort on a logarithmic bucket of the key: the key kernel counts each pixel
// into its bucket (one atomic per pixel, which also gives the pixel its rank
// among the bucket's pixels), one workgroup turns the counts into bucket
// offsets, and a scatter kernel writes each pixel id at offset + rank.
// Pixels of one bucket come out in no fixed order; the tracers' results do
// not depend on the order.
#include "internal.h"

namespace gr {
namespace {

// Bucket of a key k >= 0: the top 15 bits of its binary32 pattern (sign
// bit 0, 8 exponent bits, the leading 6 mantissa bits), which increase with
// k: buckets 1/64 of an octave wide.  NaN keys go last.
constexpr int ORDER_BITS = 15;
constexpr int NBUCKET = 1 << ORDER_BITS;
constexpr int SCAN_THREADS = 1024;

__device__ __forceinline__ uint32_t bucket_of(float key) {
    if (!(key >= 0.0f)) return NBUCKET - 1;
    return __float_as_uint(key) >> (32 - ORDER_BITS);
}

__global__ void order_clear_kernel(uint32_t* __restrict__ count) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < NBUCKET; b += gridDim.x * blockDim.x)
        count[b] = 0u;
}

// Pixel k's key |b - b_crit| of its camera ray (E = -p_t, L = p_phi and
// Carter's constant Q = p_theta^2 + cos^2(theta0) (L^2/sin^2(theta0) -
// a^2 E^2)), its bucket (into bkt) and its rank within the bucket (into rank).
__global__ void order_count_kernel(const Hole H, const Camera C, double b_crit, int64_t n,
                                   double s2, double c2, uint32_t* __restrict__ count,
                                   uint32_t* __restrict__ bkt, uint32_t* __restrict__ rank) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double pt, pr, pth, pph;
    camera_ray(C, k % C.W, k / C.W, pt, pr, pth, pph);
    const double E = -pt, L = pph;
    const double Q = fma(pth, pth, c2 * (L * L / s2 - H.a2 * E * E));
    const double b = sqrt(fmax(Q + L * L, 0.0)) / fabs(E);
    const uint32_t q = bucket_of((float)fabs(b - b_crit));
    bkt[k] = q;
    rank[k] = atomicAdd(&count[q], 1u);
}

// Exclusive prefix sum of the NBUCKET counts in place, by one workgroup:
// each thread sums a contiguous run, the run totals are scanned in LDS, and
// each thread rewrites its run as offsets.
__global__ void __launch_bounds__(SCAN_THREADS) order_scan_kernel(uint32_t* __restrict__ count) {
    constexpr int RUN = NBUCKET / SCAN_THREADS;
    __shared__ uint32_t part[SCAN_THREADS];
    const int t = threadIdx.x;
    uint32_t* run = count + t * RUN;
    uint32_t sum = 0;
    for (int i = 0; i < RUN; ++i) sum += run[i];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < SCAN_THREADS; d <<= 1) {          // inclusive Hillis-Steele scan
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t off = part[t] - sum;                          // exclusive start of this run
    for (int i = 0; i < RUN; ++i) {
        const uint32_t c = run[i];
        run[i] = off;
        off += c;
    }
}

__global__ void order_scatter_kernel(int64_t n, const uint32_t* __restrict__ offset,
                                     const uint32_t* __restrict__ bkt,
                                     const uint32_t* __restrict__ rank,
                                     int32_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    out[offset[bkt[k]] + rank[k]] = (int32_t)k;
}

}  // namespace

size_t frame_order_temp(int64_t) { return (size_t)NBUCKET * sizeof(uint32_t); }

hipError_t frame_order(const Hole& H, const Camera& C, double b_crit, int64_t npix, float* keys,
                       int32_t* vals, void* temp, size_t temp_bytes, hipStream_t s) {
    if (npix <= 0) return hipSuccess;
    if (npix > INT32_MAX || temp_bytes < frame_order_temp(npix)) return hipErrorInvalidValue;
    double sn, cs;
    sincos_def(C.th0, sn, cs);
    uint32_t* count = (uint32_t*)temp;
    uint32_t* bkt = (uint32_t*)keys;            // keys: 2 x npix floats of room
    uint32_t* rank = (uint32_t*)vals;           // vals: the first npix entries
    const unsigned grid = (unsigned)((npix + 255) / 256);
    hipLaunchKernelGGL(order_clear_kernel, dim3(NBUCKET / 256), dim3(256), 0, s, count);
    hipLaunchKernelGGL(order_count_kernel, dim3(grid), dim3(256), 0, s, H, C, b_crit, npix,
                       sn * sn, cs * cs, count, bkt, rank);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, count);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(grid), dim3(256), 0, s, npix, count, bkt, rank,
                       vals + npix);
    return hipGetLastError();
}

}  // namespace gr
