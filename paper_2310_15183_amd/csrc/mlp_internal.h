// Internal interface of the surrogate-network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gr {
namespace mlp {

constexpr int IN = 7, IN_PAD = 32, HID = 256, OUT = 4, OUT_PAD = 32, NLAYER = 5;
constexpr int COLSUM_CHUNKS = 64;   // row ranges of the bias-gradient sums
constexpr int SPLITK_MAX = 64;      // k splits of a weight-gradient product

enum { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_SILU = 2, EPI_SILU_GRAD = 3 };

// Logistic function of the network's SiLU layers, 1 / (1 + 2^(-z log2 e)),
// on the hardware base-2 exponential and reciprocal (about 1 ulp each; the
// activations are rounded to bfloat16 afterwards).  Every kernel that applies
// or differentiates SiLU uses this one definition, so that the fused frame
// kernel reproduces the layer-by-layer forward pass bit for bit.  Saturates
// to 0 and 1 for large |z|.
__device__ __forceinline__ float sigmoid_hw(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * -1.44269504f));
}

// C = A B with strided bfloat16 operands and a fused epilogue (see mlp.hip).
struct GemmArgs {
    const __bf16* A;
    int64_t sam, sak;
    const __bf16* B;
    int64_t sbk, sbn;
    int64_t M, N, K;          // K a multiple of 32
    int epi;
    const float* bias;        // EPI_BIAS_*: bias[n]
    float* outf;              // EPI_F32 / EPI_BIAS_F32 output
    int64_t sof;
    __bf16* outh;             // EPI_BIAS_SILU / EPI_SILU_GRAD output
    int64_t soh;
    float* zout;              // EPI_BIAS_SILU: pre-activation (may be null)
    int64_t szo;
    const float* zin;         // EPI_SILU_GRAD: pre-activation of the layer below
    int64_t szi;
    float* part;              // EPI_F32: split-k partials (splitk_count(M, N, K) x M x N), or null
    int64_t kc;               // set by gemm(): k per split
};

// One layer's parameters: offsets into the packed binary32 vector (W in x out
// row-major, then b) and its padded device copies.
struct Layer {
    int in, out, in_pad, out_pad;
    int64_t w_off, b_off;
    __bf16* wf;     // out_pad x in_pad: forward operand B(k=in, n=out) at wf[n*in_pad + k]
    __bf16* wb;     // in_pad x out_pad: backward operand B(k=out, n=in) at wb[n*out_pad + k]
    float* bias;    // out_pad
    __bf16* frag;   // MFMA A-operand fragments of W^T (see frag_pack in mlp.hip)
    int ftiles;     // 16-row tiles of output features: ceil(out / 16)
};

// Read-only view of a packed network for kernels outside mlp.hip.
struct NetView {
    const __bf16* frag[NLAYER];
    const float* bias[NLAYER];
};

hipError_t gemm(const GemmArgs& g, hipStream_t s);
// k splits gemm() uses for an EPI_F32 product with a partial buffer.
int splitk_count(int64_t M, int64_t N, int64_t K);
hipError_t pack(const float* params, const Layer& L, hipStream_t s);
// Elements of Layer::frag for ftiles output tiles and padded input width in_pad.
inline int64_t frag_elems(int ftiles, int in_pad) { return (int64_t)ftiles * (in_pad / 32) * 64 * 8; }
hipError_t inputs(const float* x, const int32_t* rows, int64_t n, int64_t n_src, __bf16* out,
                  hipStream_t s);
hipError_t loss(const float* y, const float* target, const int32_t* rows, int64_t n,
                int64_t n_src, float lam, float delta, float dmax, __bf16* dy, double* partial,
                float* loss_out, hipStream_t s);
// part: COLSUM_CHUNKS x ncols scratch.
hipError_t colsum(const __bf16* dz, int64_t nrows, int ld, int ncols, float* part, float* out,
                  hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t outputs(const float* y, int64_t n, float* out, hipStream_t s);

}  // namespace mlp
}  // namespace gr
