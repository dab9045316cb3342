// Redshift of the light of the ring (arXiv 2310.15183, Sec. 3.3.3): per ray
// that stopped in the ring, the circular orbit of the ring's matter at the
// ray's end point and the ratio of the frequencies it and the camera's
// observer measure.  Streaming kernel, one ray per thread, grid-stride.
//
// This translation unit must be compiled with -ffp-contract=off.

#include "internal.h"

namespace gr {
namespace {

// Inverse metric at (r, theta) of the Kerr-Newman hole or (MN) the
// Manko-Novikov spacetime, sin/cos from their definition.
template <bool MN>
__device__ __forceinline__ InvMetric metric_at(const Hole& H, const MnHole& K, double r,
                                               double th) {
    double s, c;
    sincos_def(th, s, c);
    if constexpr (MN) {
        return mn_inverse_metric<IeeeDiv>(K, r, c, s * s);
    } else {
        return inverse_metric(H, radial_terms(H, r), theta_terms_s(H, s));
    }
}

// z of one ray ending at (r, th) with conserved p_t, p_phi: the ring's orbit
// (s_t = -1, s_phi the root of s_phi^2 d g^{phph} - 2 s_phi d g^{tph}
// + d g^{tt} = 0 with the larger dphi/dt, d = forward difference in r),
// normalised to g^{mu nu} s s = -1; z = p_mu S^mu / nu_o.  NaN without a
// timelike circular orbit.
template <bool MN>
__device__ __forceinline__ double ring_redshift(const Hole& H, const MnHole& K, double eps,
                                                double nu_o, double r, double th, double pt,
                                                double pph) {
    const InvMetric g = metric_at<MN>(H, K, r, th);
    const InvMetric gr = metric_at<MN>(H, K, r + eps, th);
    const double dtt = gr.tt - g.tt, dtp = gr.tp - g.tp, dpp = gr.pp - g.pp;
    const double disc = dtp * dtp - dpp * dtt;
    if (!(disc >= 0.0) || dpp == 0.0) return NAN;
    const double sq = sqrt(disc);
    const double x1 = (dtp + sq) / dpp, x2 = (dtp - sq) / dpp;
    const double w1 = fma(g.pp, x1, -g.tp) / fma(g.tp, x1, -g.tt);
    const double w2 = fma(g.pp, x2, -g.tp) / fma(g.tp, x2, -g.tt);
    const double x = (w1 >= w2) ? x1 : x2;
    const double norm = fma(g.pp * x, x, fma(-2.0 * g.tp, x, g.tt));
    if (!(norm < 0.0)) return NAN;
    const double k = 1.0 / sqrt(-norm);
    const double st = -k, sp = x * k;
    const double St = fma(g.tt, st, g.tp * sp);
    const double Sp = fma(g.tp, st, g.pp * sp);
    return fma(pt, St, pph * Sp) / nu_o;
}

template <typename T, bool MN>
__global__ void __launch_bounds__(256) redshift_kernel(const Hole H, const MnHole K, double eps,
                                                       double nu_o, const T* __restrict__ r,
                                                       const T* __restrict__ th,
                                                       const T* __restrict__ pt,
                                                       const T* __restrict__ pph,
                                                       const int8_t* __restrict__ flag,
                                                       int64_t n, T* __restrict__ z) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        double v = NAN;
        if (flag[k] == GR_FLAG_DISK)
            v = ring_redshift<MN>(H, K, eps, nu_o, (double)r[k], (double)th[k], (double)pt[k],
                                  (double)pph[k]);
        z[k] = (T)v;
    }
}

template <typename T>
hipError_t launch(const Hole& H, const MnHole& K, bool mn, double eps, double nu_o,
                  const OutPtrs& o, int64_t n, void* z, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16);
    const T* r = reinterpret_cast<const T*>(o.r);
    const T* th = reinterpret_cast<const T*>(o.th);
    const T* pt = reinterpret_cast<const T*>(o.pt);
    const T* pph = reinterpret_cast<const T*>(o.pph);
    T* zz = reinterpret_cast<T*>(z);
    if (mn)
        hipLaunchKernelGGL((redshift_kernel<T, true>), dim3(grid), dim3(256), 0, s, H, K, eps,
                           nu_o, r, th, pt, pph, o.flag, n, zz);
    else
        hipLaunchKernelGGL((redshift_kernel<T, false>), dim3(grid), dim3(256), 0, s, H, K, eps,
                           nu_o, r, th, pt, pph, o.flag, n, zz);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_redshift(const Hole& H, const MnHole& K, bool mn, const Integrator& in,
                           double nu_o, const OutPtrs& o, bool f32, int64_t n, void* z,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return f32 ? launch<float>(H, K, mn, in.eps, nu_o, o, n, z, s)
               : launch<double>(H, K, mn, in.eps, nu_o, o, n, z, s);
}

}  // namespace gr
