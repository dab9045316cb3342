// FP64 geodesic tracer for the Manko-Novikov spacetime (arXiv 2310.15183,
// Sec. 2.2.3): the same Hamiltonian RK4 as the Kerr-Newman tracer (Sec. 2.1,
// Sec. 3.1.2, Sec. 3.3), with the metric's three evaluations per stage done
// in full (mn_inverse_metric).  One lane per ray over 8x8 pixel tiles.
//
// Two launches per frame.  Rays still running after `cap` steps are parked
// (their state written to a compact list, one atomic per wave) and the second
// launch continues all of them together: a frame's few trapped rays, which
// run to the step limit, then start at the same time instead of whenever
// their tiles come up, and share waves densely.  A ray's steps are the same
// in either launch, so the results are those of one uninterrupted loop.
//
// This translation unit must be compiled with -ffp-contract=off.

#include <climits>

#include "internal.h"
#include "step_fp64.h"

namespace gr {
namespace {

using namespace detail;

struct MnArgs {
    FrameArgs f;
    MnHole mn;
    Parked park;
};

template <int METHOD, bool DISK>
__device__ __forceinline__ int run(const MnArgs& X, Ray& y, int& s, int f, int cap) {
    while (f == RUNNING && s < cap) {
        const double nu = mn_step<METHOD>(X.mn, X.f.in, y);
        ++s;
        f = exit_flag<DISK>(X.f.in, X.f.r_esc, y, nu, s);
    }
    return f;
}

template <typename T, int METHOD, bool DISK>
__global__ void __launch_bounds__(256) trace_mn_static(const MnArgs X) {
    const FrameArgs& A = X.f;
    const Parked& P = X.park;
    int64_t k, pix;
    if (!static_ray(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, k, pix)) return;
    Ray y;
    start_ray(A.cam, pix, y);
    int s = 0;
    int f = run<METHOD, DISK>(X, y, s, start_flag(A.in, y), P.cap > 0 ? P.cap : INT_MAX);
    // park the rays still running (every active lane takes part in the ballot)
    const int64_t slot = take_ids(f == RUNNING, P.count);
    if (slot >= 0 && slot < P.capacity) {
        P.y[slot] = y.t;
        P.y[P.capacity + slot] = y.r;
        P.y[2 * P.capacity + slot] = y.th;
        P.y[3 * P.capacity + slot] = y.ph;
        P.y[4 * P.capacity + slot] = y.pr;
        P.y[5 * P.capacity + slot] = y.pth;
        P.steps[slot] = s;
        P.pix[slot] = pix;
        return;
    }
    f = run<METHOD, DISK>(X, y, s, f, INT_MAX);    // no room left: finish here
    write_ray<T>(A.out, k, y, f, s);
}

// Second launch: the parked rays (their number is read from the device),
// resident waves striding over the list.
template <typename T, int METHOD, bool DISK>
__global__ void __launch_bounds__(256) trace_mn_resume(const MnArgs X) {
    const FrameArgs& A = X.f;
    const Parked& P = X.park;
    const unsigned long long parked = *P.count;
    const int64_t n = parked < (unsigned long long)P.capacity ? (int64_t)parked : P.capacity;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        const int64_t pix = P.pix[q];
        Ray y;
        start_ray(A.cam, pix, y);                 // p_t, p_phi and their products
        y.t = P.y[q];
        y.r = P.y[P.capacity + q];
        y.th = P.y[2 * P.capacity + q];
        y.ph = P.y[3 * P.capacity + q];
        y.pr = P.y[4 * P.capacity + q];
        y.pth = P.y[5 * P.capacity + q];
        int s = P.steps[q];
        const int f = run<METHOD, DISK>(X, y, s, RUNNING, INT_MAX);
        write_ray<T>(A.out, pix, y, f, s);
    }
}

}  // namespace

template <int METHOD, bool DISK>
static hipError_t launch_mn(const MnArgs& X, bool f32_out, const LaunchShape& L,
                            const LaunchShape& L2, hipStream_t s) {
    if (X.park.cap > 0) {
        const hipError_t e = launch_reset_counter(X.park.count, s);
        if (e != hipSuccess) return e;
    }
    if (f32_out)
        hipLaunchKernelGGL((trace_mn_static<float, METHOD, DISK>), dim3(L.grid), dim3(L.block), 0,
                           s, X);
    else
        hipLaunchKernelGGL((trace_mn_static<double, METHOD, DISK>), dim3(L.grid), dim3(L.block), 0,
                           s, X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || X.park.cap <= 0) return e;
    if (f32_out)
        hipLaunchKernelGGL((trace_mn_resume<float, METHOD, DISK>), dim3(L2.grid), dim3(L2.block),
                           0, s, X);
    else
        hipLaunchKernelGGL((trace_mn_resume<double, METHOD, DISK>), dim3(L2.grid), dim3(L2.block),
                           0, s, X);
    return hipGetLastError();
}

template <int METHOD>
static hipError_t launch_mn_disk(const MnArgs& X, bool f32_out, bool disk, const LaunchShape& L,
                                 const LaunchShape& L2, hipStream_t s) {
    return disk ? launch_mn<METHOD, true>(X, f32_out, L, L2, s)
                : launch_mn<METHOD, false>(X, f32_out, L, L2, s);
}

hipError_t launch_trace_mn(const FrameArgs& A, const MnHole& K, bool f32_out, int method,
                           bool disk, const LaunchShape& L, const Parked& park,
                           const LaunchShape& L2, hipStream_t s) {
    MnArgs X;
    X.f = A;
    X.mn = K;
    X.park = park;
    if (method == M_EULER) return launch_mn_disk<M_EULER>(X, f32_out, disk, L, L2, s);
    if (method == M_RK4_TIME) return launch_mn_disk<M_RK4_TIME>(X, f32_out, disk, L, L2, s);
    return launch_mn_disk<M_RK4>(X, f32_out, disk, L, L2, s);
}

int occupancy_trace_mn_resume(int block) {
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
               &n, trace_mn_resume<float, M_RK4, false>, block, 0) == hipSuccess
               ? n
               : 0;
}

}  // namespace gr
