// Device checks of the binary64 tracer's building blocks, off the tracing
// path: the correctly rounded reciprocal and quotient that the Kerr-Newman
// step forms from the hardware reciprocal estimate (step_fp64.h), evaluated
// on caller-supplied operands so that they can be compared with IEEE
// division.  Host code and one kernel.
#include "grtrace.h"
#include "step_fp64.h"

namespace gr {
namespace {

__global__ void __launch_bounds__(256) division_kernel(const double* __restrict__ a,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ q,
                                                       double* __restrict__ r, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double xi = x[i];
        q[i] = detail::div_rn(a[i], xi);
        r[i] = detail::rcp_rn(xi);
    }
}

}  // namespace
}  // namespace gr

extern "C" int gr_check_division(const double* a, const double* x, double* q, double* r,
                                 int64_t n, void* hip_stream) {
    if (n < 0) return GR_EINVAL;
    if (n == 0) return GR_OK;
    if (!a || !x || !q || !r) return GR_EINVAL;
    const int64_t blocks = (n + 255) / 256;
    const int grid = (int)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(gr::division_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream,
                       a, x, q, r, n);
    return hipGetLastError() == hipSuccess ? GR_OK : GR_EDEVICE;
}
