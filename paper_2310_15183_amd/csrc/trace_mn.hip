// FP64 geodesic tracer for the Manko-Novikov spacetime (arXiv 2310.15183,
// Sec. 2.2.3): the same Hamiltonian RK4 as the Kerr-Newman tracer (Sec. 2.1,
// Sec. 3.1.2, Sec. 3.3), with the metric's three evaluations per stage done
// in full (mn_inverse_metric).  One lane per ray over 8x8 pixel tiles.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "internal.h"
#include "step_fp64.h"

namespace gr {
namespace {

using namespace detail;

struct MnArgs {
    FrameArgs f;
    MnHole mn;
};

template <typename T, bool EULER, bool DISK>
__global__ void __launch_bounds__(256) trace_mn_static(const MnArgs X) {
    const FrameArgs& A = X.f;
    int64_t k, pix;
    if (!static_ray(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, k, pix)) return;
    Ray y;
    start_ray(A.cam, pix, y);
    int s = 0;
    int f = start_flag(A.in, y);
    while (f == RUNNING) {
        const double nu = mn_step<EULER>(X.mn, A.in, y);
        ++s;
        f = exit_flag<DISK>(A.in, A.r_esc, y, nu, s);
    }
    write_ray<T>(A.out, k, y, f, s);
}

}  // namespace

template <bool EULER, bool DISK>
static hipError_t launch_mn(const MnArgs& X, bool f32_out, const LaunchShape& L, hipStream_t s) {
    if (f32_out)
        hipLaunchKernelGGL((trace_mn_static<float, EULER, DISK>), dim3(L.grid), dim3(L.block), 0,
                           s, X);
    else
        hipLaunchKernelGGL((trace_mn_static<double, EULER, DISK>), dim3(L.grid), dim3(L.block), 0,
                           s, X);
    return hipGetLastError();
}

hipError_t launch_trace_mn(const FrameArgs& A, const MnHole& K, bool f32_out, bool euler,
                           bool disk, const LaunchShape& L, hipStream_t s) {
    MnArgs X;
    X.f = A;
    X.mn = K;
    if (euler && disk) return launch_mn<true, true>(X, f32_out, L, s);
    if (euler) return launch_mn<true, false>(X, f32_out, L, s);
    if (disk) return launch_mn<false, true>(X, f32_out, L, s);
    return launch_mn<false, false>(X, f32_out, L, s);
}

}  // namespace gr
