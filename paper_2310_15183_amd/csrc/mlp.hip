// Surrogate network kernels for gfx950: bfloat16 products on MFMA with
// binary32 accumulation, SiLU, loss, Adam, and the per-ray features, targets
// and fallback selection of the surrogate frame.
//
// Network: 7 inputs -> 4 hidden layers of 256 (SiLU) -> 4 outputs (escape
// logit and a correction d of the end sky direction relative to the
// straight-line (flat space) direction).  Padded device shapes: the input
// width 7 is padded to 32 and the output width 4 to 32, so every product has
// K a multiple of 32.
#include "internal.h"
#include "mlp_internal.h"

namespace gr {
namespace mlp {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf8;

constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;   // LDS rows padded to 40

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// C[M x N] = A[M x K] B[K x N]; A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn].
// 256 threads: the workgroup computes a 64x64 tile, each wave a 32x32 block
// as 2x2 MFMA 16x16x32 tiles.  K must be a multiple of 32; rows >= M and
// columns >= N are neither read nor written.  With gridDim.z = splits > 1
// (EPI_F32 only) workgroup z sums k in [z kc, (z + 1) kc) and writes its
// partial tile to part[z][M][N]; splitk_reduce_kernel adds the partials in
// order of z.  Each thread stages 8 values of A and 8 of B per k-step with one
// 16-byte load when they are contiguous and inside the matrix.
__global__ void __launch_bounds__(256) gemm_kernel(const GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 As[TM][LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[TN][LDK];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * TM;
    const int64_t n0 = (int64_t)blockIdx.y * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t kbeg = (int64_t)blockIdx.z * g.kc;
    const int64_t kend = kbeg + g.kc < g.K ? kbeg + g.kc : g.K;

    for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
        // ---- stage A (64 x 32) and B (32 x 64) into LDS, rows = m / n, k contiguous
        if (g.sak == 1) {
            const int m = tid >> 2, kk = (tid & 3) * 8;
            const int64_t gm = m0 + m;
            bf8 v;
            if (gm < g.M) v = *reinterpret_cast<const bf8*>(g.A + gm * g.sam + k0 + kk);
            else for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
            *reinterpret_cast<bf8*>(&As[m][kk]) = v;
        } else {
            const int kk = tid >> 3, m = (tid & 7) * 8;
            const int64_t gm = m0 + m;
            if (g.sam == 1 && gm + 8 <= g.M) {
                const bf8 v = *reinterpret_cast<const bf8*>(g.A + gm + (k0 + kk) * g.sak);
                for (int j = 0; j < 8; ++j) As[m + j][kk] = v[j];
            } else {
                for (int j = 0; j < 8; ++j)
                    As[m + j][kk] = gm + j < g.M ? g.A[(gm + j) * g.sam + (k0 + kk) * g.sak]
                                                 : (__bf16)0.0f;
            }
        }
        if (g.sbk == 1) {
            const int n = tid >> 2, kk = (tid & 3) * 8;
            const int64_t gn = n0 + n;
            bf8 v;
            if (gn < g.N) v = *reinterpret_cast<const bf8*>(g.B + (k0 + kk) + gn * g.sbn);
            else for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
            *reinterpret_cast<bf8*>(&Bs[n][kk]) = v;
        } else {
            const int kk = tid >> 3, n = (tid & 7) * 8;
            const int64_t gn = n0 + n;
            if (g.sbn == 1 && gn + 8 <= g.N) {
                const bf8 v = *reinterpret_cast<const bf8*>(g.B + (k0 + kk) * g.sbk + gn);
                for (int j = 0; j < 8; ++j) Bs[n + j][kk] = v[j];
            } else {
                for (int j = 0; j < 8; ++j)
                    Bs[n + j][kk] = gn + j < g.N ? g.B[(k0 + kk) * g.sbk + (gn + j) * g.sbn]
                                                 : (__bf16)0.0f;
            }
        }
        __syncthreads();
        bf8 a[2], b[2];
        const int r = lane & 15, kq = (lane >> 4) * 8;
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf8*>(&As[wm + 16 * i + r][kq]);
        for (int i = 0; i < 2; ++i) b[i] = *reinterpret_cast<const bf8*>(&Bs[wn + 16 * i + r][kq]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }

    // ---- epilogue: lane holds rows 4*(lane/16)+e (e = 0..3), column lane%16 of each tile
    float* outf = g.outf;
    int64_t sof = g.sof;
    if (gridDim.z > 1) {
        outf = g.part + (int64_t)blockIdx.z * g.M * g.N;
        sof = g.N;
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int64_t col = n0 + wn + 16 * j + (lane & 15);
            if (col >= g.N) continue;
            const float bias = g.bias ? g.bias[col] : 0.0f;
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                if (row >= g.M) continue;
                const float v = acc[i][j][e];
                switch (g.epi) {
                    case EPI_F32:
                        outf[row * sof + col] = v;
                        break;
                    case EPI_BIAS_F32:
                        g.outf[row * g.sof + col] = v + bias;
                        break;
                    case EPI_BIAS_SILU: {
                        const float z = v + bias;
                        if (g.zout) g.zout[row * g.szo + col] = z;
                        g.outh[row * g.soh + col] = (__bf16)(z * sigmoid_hw(z));
                        break;
                    }
                    case EPI_SILU_GRAD: {
                        const float z = g.zin[row * g.szi + col];
                        const float s = sigmoid_hw(z);
                        g.outh[row * g.soh + col] = (__bf16)(v * (s * (1.0f + z * (1.0f - s))));
                        break;
                    }
                }
            }
        }
}

// out[m * sof + n] = sum over z (in order) of part[z][m][n].
__global__ void splitk_reduce_kernel(const float* __restrict__ part, int splits, int64_t M,
                                     int64_t N, float* __restrict__ out, int64_t sof) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * N) return;
    float s = part[idx];
    for (int z = 1; z < splits; ++z) s += part[(int64_t)z * M * N + idx];
    out[(idx / N) * sof + idx % N] = s;
}

// Packed binary32 parameters -> padded bfloat16 weights in both orientations,
// padded binary32 biases, and the weights as MFMA A fragments of W^T: the
// 16 x 32 block (output features 16 ft.., inputs 32 ks..) is 64 lanes x 8
// values, lane l holding feature 16 ft + l % 16 at inputs 32 ks + 8 (l / 16) + j,
// stored at frag[((ft * (in_pad / 32) + ks) * 64 + l) * 8 + j] (16 contiguous
// bytes per lane, 1 KiB per block).
__global__ void pack_kernel(const float* __restrict__ params, Layer L, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    // idx runs over out_pad x in_pad of this layer
    const int n = (int)(idx / L.in_pad), k = (int)(idx % L.in_pad);   // n: out, k: in
    const bool inside = n < L.out && k < L.in;
    const __bf16 w = inside ? (__bf16)params[L.w_off + (int64_t)k * L.out + n] : (__bf16)0.0f;
    L.wf[(int64_t)n * L.in_pad + k] = w;       // forward: B(k=in, n=out)
    L.wb[(int64_t)k * L.out_pad + n] = w;      // backward: B(k=out, n=in)
    if (k == 0) L.bias[n] = n < L.out ? params[L.b_off + n] : 0.0f;
    if (n < 16 * L.ftiles) {
        const int ft = n >> 4, ks = k >> 5, lane = (n & 15) + 16 * ((k & 31) >> 3);
        L.frag[(((int64_t)ft * (L.in_pad >> 5) + ks) * 64 + lane) * 8 + (k & 7)] = w;
    }
}

// Inputs n x 7 binary32 (optionally gathered through rows[], each in
// [0, n_src); others read as zeros) -> n x 32 bfloat16.
__global__ void input_kernel(const float* __restrict__ x, const int32_t* __restrict__ rows,
                             int64_t n, int64_t n_src, __bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t src = rows ? (int64_t)rows[i] : i;
    const bool ok = src >= 0 && src < n_src;
    for (int c = 0; c < IN_PAD; ++c)
        out[i * IN_PAD + c] = (ok && c < IN) ? (__bf16)x[src * IN + c] : (__bf16)0.0f;
}

// Loss terms and output gradient (see the network description):
//   l_i = softplus(y0) - esc y0 + lam w sum_c huber(y[c] - d[c]),  L = sum l_i / n
// huber(e) = e^2 for |e| <= delta, 2 delta |e| - delta^2 beyond; the direction
// weight w is esc for rows whose target |d| <= dmax and 0 otherwise.
// dy is written as bfloat16 n x 32 (zero beyond column 3); per-block partial
// sums of l_i go to partial[blockIdx.x] (reduced by reduce_kernel).
__global__ void loss_kernel(const float* __restrict__ y, const float* __restrict__ target,
                            const int32_t* __restrict__ rows, int64_t n, int64_t n_src, float lam,
                            float delta, float dmax, float inv_n, __bf16* __restrict__ dy,
                            double* __restrict__ partial) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double li = 0.0;
    if (i < n) {
        const int64_t src = rows ? (int64_t)rows[i] : i;
        const bool ok = src >= 0 && src < n_src;
        const float zero4[OUT] = {0.f, 0.f, 0.f, 0.f};
        const float* t = ok ? target + src * OUT : zero4;
        const float* yi = y + i * OUT_PAD;
        const float esc = t[0];
        const float d2 = (t[1] * t[1] + t[2] * t[2]) + t[3] * t[3];
        const float wd = d2 <= dmax * dmax ? esc : 0.0f;
        const float y0 = yi[0];
        const float sp = fmaxf(y0, 0.0f) + log1pf(expf(-fabsf(y0)));
        float hub = 0.0f;
        for (int c = 1; c < OUT; ++c) {
            const float e = yi[c] - t[c], a = fabsf(e);
            hub += a <= delta ? e * e : 2.0f * delta * a - delta * delta;
        }
        li = (double)(sp - esc * y0 + lam * wd * hub);
        dy[i * OUT_PAD + 0] = (__bf16)((sigmoidf_(y0) - esc) * inv_n);
        for (int c = 1; c < OUT; ++c) {
            const float e = yi[c] - t[c];
            const float ge = fabsf(e) <= delta ? 2.0f * e : copysignf(2.0f * delta, e);
            dy[i * OUT_PAD + c] = (__bf16)(lam * wd * ge * inv_n);
        }
        for (int c = OUT; c < OUT_PAD; ++c) dy[i * OUT_PAD + c] = (__bf16)0.0f;
    }
    red[threadIdx.x] = li;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void reduce_kernel(const double* __restrict__ partial, int64_t n, float inv_n,
                              float* __restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(red[0] * (double)inv_n);
}

// db[c] = sum over rows of dz[r][c] (bfloat16 rows of width ld), c < ncols,
// in two passes: COLSUM_CHUNKS row ranges into part[chunk][c], then the
// chunks in order.
__global__ void colsum_partial_kernel(const __bf16* __restrict__ dz, int64_t nrows, int ld,
                                      int ncols, float* __restrict__ part) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int grp = threadIdx.x >> 6;
    const int64_t per = (nrows + COLSUM_CHUNKS - 1) / COLSUM_CHUNKS;
    const int64_t r0 = (int64_t)blockIdx.y * per;
    const int64_t r1 = r0 + per < nrows ? r0 + per : nrows;
    float s = 0.0f;
    if (c < ncols)
        for (int64_t r = r0 + grp; r < r1; r += 4) s += (float)dz[r * ld + c];
    red[grp][threadIdx.x & 63] = s;
    __syncthreads();
    if (grp == 0 && c < ncols)
        part[(int64_t)blockIdx.y * ncols + c] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void colsum_final_kernel(const float* __restrict__ part, int ncols,
                                    float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    float s = 0.0f;
    for (int k = 0; k < COLSUM_CHUNKS; ++k) s += part[k * ncols + c];
    out[c] = s;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Output rows n x 32 binary32 -> n x 4.
__global__ void output_kernel(const float* __restrict__ y, int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < OUT; ++c) out[i * OUT + c] = y[i * OUT_PAD + c];
}

}  // namespace

int splitk_count(int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
    int64_t splits = (256 + tiles - 1) / tiles;
    const int64_t max_splits = K / 128 > 1 ? K / 128 : 1;     // at least 128 k per split
    if (splits > max_splits) splits = max_splits;
    if (splits > SPLITK_MAX) splits = SPLITK_MAX;
    return (int)(splits > 1 ? splits : 1);
}

hipError_t gemm(const GemmArgs& g0, hipStream_t s) {
    if (g0.M <= 0 || g0.N <= 0) return hipSuccess;
    // the 16-byte staging loads need 8-value aligned strides and operands
    if (g0.K % TK || g0.sam % 8 && g0.sam != 1 || g0.sak % 8 && g0.sak != 1 ||
        g0.sbk % 8 && g0.sbk != 1 || g0.sbn % 8 && g0.sbn != 1 ||
        (reinterpret_cast<uintptr_t>(g0.A) | reinterpret_cast<uintptr_t>(g0.B)) & 15)
        return hipErrorInvalidValue;
    GemmArgs g = g0;
    int splits = 1;
    if (g.epi == EPI_F32 && g.part) splits = splitk_count(g.M, g.N, g.K);
    g.kc = splits > 1 ? (((g.K + splits - 1) / splits + TK - 1) / TK) * TK : g.K;
    const dim3 grid((unsigned)((g.M + TM - 1) / TM), (unsigned)((g.N + TN - 1) / TN),
                    (unsigned)splits);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, g);
    if (splits > 1) {
        const int64_t n = g.M * g.N;
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           s, g.part, splits, g.M, g.N, g.outf, g.sof);
    }
    return hipGetLastError();
}

hipError_t pack(const float* params, const Layer& L, hipStream_t s) {
    const int64_t total = (int64_t)L.out_pad * L.in_pad;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       params, L, total);
    return hipGetLastError();
}

hipError_t inputs(const float* x, const int32_t* rows, int64_t n, int64_t n_src, __bf16* out,
                  hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(input_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, rows,
                       n, n_src, out);
    return hipGetLastError();
}

hipError_t loss(const float* y, const float* target, const int32_t* rows, int64_t n,
                int64_t n_src, float lam, float delta, float dmax, __bf16* dy, double* partial,
                float* loss_out, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    const float inv_n = 1.0f / (float)n;
    hipLaunchKernelGGL(loss_kernel, dim3(blocks), dim3(256), 0, s, y, target, rows, n, n_src, lam,
                       delta, dmax, inv_n, dy, partial);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, partial, (int64_t)blocks, inv_n,
                       loss_out);
    return hipGetLastError();
}

hipError_t colsum(const __bf16* dz, int64_t nrows, int ld, int ncols, float* part, float* out,
                  hipStream_t s) {
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((unsigned)((ncols + 63) / 64), COLSUM_CHUNKS),
                       dim3(256), 0, s, dz, nrows, ld, ncols, part);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s,
                       part, ncols, out);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v,
                       n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t outputs(const float* y, int64_t n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(output_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, n,
                       out);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace gr
