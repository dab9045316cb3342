// C-ABI entry points of the surrogate network (gr_mlp_*): parameters, Adam
// state and activation workspace on the device; forward, loss and gradient,
// and the optimiser step, all on the kernels of mlp.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "grtrace.h"
#include "internal.h"
#include "mlp_internal.h"

using namespace gr::mlp;

struct gr_mlp {
    int device;
    int64_t max_batch;
    int64_t nparam;
    int64_t step;               // Adam steps taken
    float* params;              // packed binary32 master copy
    float* m;
    float* v;
    Layer layer[NLAYER];
    // workspace, max_batch rows
    __bf16* X;                  // max_batch x IN_PAD
    __bf16* H[NLAYER - 1];      // layer outputs (inputs of the next layer), x HID
    float* Z[NLAYER - 1];       // pre-activations, x HID
    float* Y;                   // max_batch x OUT_PAD
    __bf16* dY;                 // max_batch x OUT_PAD
    __bf16* dZ[2];              // ping-pong, x HID
    double* partial;            // loss partial sums
    float* kpart;               // split-k partials of the weight gradients
    float* colpart;             // partial bias-gradient sums
    float* loss;                // device scalar (when the caller passes none)
};

namespace {

const int SIZES[NLAYER + 1] = {IN, HID, HID, HID, HID, OUT};

int64_t count_params() {
    int64_t n = 0;
    for (int l = 0; l < NLAYER; ++l) n += (int64_t)SIZES[l] * SIZES[l + 1] + SIZES[l + 1];
    return n;
}

struct Guard {
    int prev = -1;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~Guard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

template <typename T>
bool dalloc(T** p, int64_t n) {
    return hipMalloc((void**)p, (size_t)n * sizeof(T)) == hipSuccess;
}

void free_all(gr_mlp* m) {
    hipFree(m->params);
    hipFree(m->m);
    hipFree(m->v);
    for (int l = 0; l < NLAYER; ++l) {
        hipFree(m->layer[l].wf);
        hipFree(m->layer[l].wb);
        hipFree(m->layer[l].bias);
        hipFree(m->layer[l].frag);
    }
    hipFree(m->X);
    for (int l = 0; l < NLAYER - 1; ++l) {
        hipFree(m->H[l]);
        hipFree(m->Z[l]);
    }
    hipFree(m->Y);
    hipFree(m->dY);
    hipFree(m->dZ[0]);
    hipFree(m->dZ[1]);
    hipFree(m->partial);
    hipFree(m->kpart);
    hipFree(m->colpart);
    hipFree(m->loss);
}

hipError_t repack(gr_mlp* m, hipStream_t s) {
    for (int l = 0; l < NLAYER; ++l) {
        hipError_t e = pack(m->params, m->layer[l], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Forward pass over n <= max_batch rows already in m->X; keep pre-activations
// when training.
hipError_t forward_rows(gr_mlp* m, int64_t n, bool keep, hipStream_t s) {
    for (int l = 0; l < NLAYER; ++l) {
        const Layer& L = m->layer[l];
        GemmArgs g;
        memset(&g, 0, sizeof g);
        if (l == 0) {
            g.A = m->X;
            g.sam = IN_PAD;
        } else {
            g.A = m->H[l - 1];
            g.sam = HID;
        }
        g.sak = 1;
        g.B = L.wf;
        g.sbk = 1;
        g.sbn = L.in_pad;
        g.M = n;
        g.N = L.out;
        g.K = L.in_pad;
        g.bias = L.bias;
        if (l < NLAYER - 1) {
            g.epi = EPI_BIAS_SILU;
            g.outh = m->H[l];
            g.soh = HID;
            g.zout = keep ? m->Z[l] : nullptr;
            g.szo = HID;
        } else {
            g.epi = EPI_BIAS_F32;
            g.outf = m->Y;
            g.sof = OUT_PAD;
        }
        hipError_t e = gemm(g, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int64_t gr_mlp_num_params(void) { return count_params(); }

int gr_mlp_create(gr_mlp** out, int device, int64_t max_batch) {
    if (!out) return GR_EINVAL;
    *out = nullptr;
    if (max_batch < 32 || max_batch > ((int64_t)1 << 28)) return GR_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return GR_EDEVICE;
    if (device < 0 || device >= ndev) return GR_EINVAL;
    Guard guard(device);
    gr_mlp* m = new (std::nothrow) gr_mlp;
    if (!m) return GR_ENOMEM;
    memset(m, 0, sizeof *m);
    m->device = device;
    m->max_batch = max_batch;
    m->nparam = count_params();
    bool ok = dalloc(&m->params, m->nparam) && dalloc(&m->m, m->nparam) &&
              dalloc(&m->v, m->nparam);
    int64_t off = 0;
    for (int l = 0; l < NLAYER && ok; ++l) {
        Layer& L = m->layer[l];
        L.in = SIZES[l];
        L.out = SIZES[l + 1];
        L.in_pad = l == 0 ? IN_PAD : HID;
        L.out_pad = l == NLAYER - 1 ? OUT_PAD : HID;
        L.w_off = off;
        off += (int64_t)L.in * L.out;
        L.b_off = off;
        off += L.out;
        L.ftiles = (L.out + 15) / 16;
        ok = dalloc(&L.wf, (int64_t)L.in_pad * L.out_pad) &&
             dalloc(&L.wb, (int64_t)L.in_pad * L.out_pad) && dalloc(&L.bias, L.out_pad) &&
             dalloc(&L.frag, frag_elems(L.ftiles, L.in_pad));
    }
    ok = ok && dalloc(&m->X, max_batch * IN_PAD);
    for (int l = 0; l < NLAYER - 1 && ok; ++l)
        ok = dalloc(&m->H[l], max_batch * HID) && dalloc(&m->Z[l], max_batch * HID);
    ok = ok && dalloc(&m->Y, max_batch * OUT_PAD) && dalloc(&m->dY, max_batch * OUT_PAD) &&
         dalloc(&m->dZ[0], max_batch * HID) && dalloc(&m->dZ[1], max_batch * HID) &&
         dalloc(&m->partial, max_batch / 256 + 2) && dalloc(&m->loss, 4) &&
         dalloc(&m->kpart, (int64_t)SPLITK_MAX * HID * HID) &&
         dalloc(&m->colpart, (int64_t)COLSUM_CHUNKS * HID);
    if (!ok) {
        free_all(m);
        delete m;
        return GR_ENOMEM;
    }
    *out = m;
    return GR_OK;
}

int gr_mlp_destroy(gr_mlp* m) {
    if (!m) return GR_OK;
    Guard guard(m->device);
    free_all(m);
    delete m;
    return GR_OK;
}

int gr_mlp_set_params(gr_mlp* m, const float* host_params) {
    if (!m || !host_params) return GR_EINVAL;
    Guard guard(m->device);
    if (hipMemcpy(m->params, host_params, m->nparam * sizeof(float), hipMemcpyHostToDevice) !=
        hipSuccess)
        return GR_EDEVICE;
    if (hipMemset(m->m, 0, m->nparam * sizeof(float)) != hipSuccess ||
        hipMemset(m->v, 0, m->nparam * sizeof(float)) != hipSuccess)
        return GR_EDEVICE;
    m->step = 0;
    if (repack(m, nullptr) != hipSuccess) return GR_EDEVICE;
    return hipDeviceSynchronize() == hipSuccess ? GR_OK : GR_EDEVICE;
}

int gr_mlp_get_params(const gr_mlp* m, float* host_params) {
    if (!m || !host_params) return GR_EINVAL;
    Guard guard(m->device);
    if (hipDeviceSynchronize() != hipSuccess) return GR_EDEVICE;
    return hipMemcpy(host_params, m->params, m->nparam * sizeof(float), hipMemcpyDeviceToHost) ==
                   hipSuccess
               ? GR_OK
               : GR_EDEVICE;
}

int gr_mlp_init(gr_mlp* m, uint64_t seed) {
    if (!m) return GR_EINVAL;
    // He-uniform weights (bound sqrt(6/fan_in)) from SplitMix64, zero biases
    std::vector<float> p(m->nparam, 0.0f);
    uint64_t st = seed;
    auto next = [&st]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int l = 0; l < NLAYER; ++l) {
        const Layer& L = m->layer[l];
        const double bound = sqrt(6.0 / L.in);
        for (int64_t i = 0; i < (int64_t)L.in * L.out; ++i) {
            const double u = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
            p[L.w_off + i] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    return gr_mlp_set_params(m, p.data());
}

int gr_mlp_forward(gr_mlp* m, const float* x, int64_t n, float* y, void* stream) {
    if (!m || n < 0 || (n > 0 && (!x || !y))) return GR_EINVAL;
    Guard guard(m->device);
    hipStream_t s = (hipStream_t)stream;
    for (int64_t r0 = 0; r0 < n; r0 += m->max_batch) {
        const int64_t nb = n - r0 < m->max_batch ? n - r0 : m->max_batch;
        if (inputs(x + r0 * IN, nullptr, nb, nb, m->X, s) != hipSuccess) return GR_EDEVICE;
        if (forward_rows(m, nb, false, s) != hipSuccess) return GR_EDEVICE;
        if (outputs(m->Y, nb, y + r0 * OUT, s) != hipSuccess) return GR_EDEVICE;
    }
    return GR_OK;
}

int gr_mlp_loss_grad(gr_mlp* m, const float* x, const float* target, const int32_t* rows,
                     int64_t n, int64_t n_src, float lam, float delta, float dmax, float* loss,
                     float* grad, void* stream) {
    if (!m || !x || !target || !grad) return GR_EINVAL;
    if (n < 32 || n > m->max_batch || n % 32) return GR_EINVAL;
    if (!rows) n_src = n;
    if (n_src < 1 || !(lam >= 0.0f) || !(delta > 0.0f) || !(dmax >= 0.0f)) return GR_EINVAL;
    Guard guard(m->device);
    hipStream_t s = (hipStream_t)stream;
    if (inputs(x, rows, n, n_src, m->X, s) != hipSuccess) return GR_EDEVICE;
    if (forward_rows(m, n, true, s) != hipSuccess) return GR_EDEVICE;
    if (gr::mlp::loss(m->Y, target, rows, n, n_src, lam, delta, dmax, m->dY, m->partial,
                      loss ? loss : m->loss, s) != hipSuccess)
        return GR_EDEVICE;
    // backward, last layer first
    const __bf16* dz = m->dY;
    int64_t ldz = OUT_PAD;
    int pp = 0;
    for (int l = NLAYER - 1; l >= 0; --l) {
        const Layer& L = m->layer[l];
        const __bf16* hin = l == 0 ? m->X : m->H[l - 1];
        const int64_t ldh = l == 0 ? IN_PAD : HID;
        GemmArgs g;
        memset(&g, 0, sizeof g);
        g.A = hin;                  // A(m = in feature, k = row) = hin[k*ldh + m]
        g.sam = 1;
        g.sak = ldh;
        g.B = dz;                   // B(k = row, n = out) = dz[k*ldz + n]
        g.sbk = ldz;
        g.sbn = 1;
        g.M = L.in;
        g.N = L.out;
        g.K = n;
        g.epi = EPI_F32;
        g.outf = grad + L.w_off;
        g.sof = L.out;
        g.part = m->kpart;
        if (gemm(g, s) != hipSuccess) return GR_EDEVICE;
        if (colsum(dz, n, (int)ldz, L.out, m->colpart, grad + L.b_off, s) != hipSuccess)
            return GR_EDEVICE;
        if (l == 0) break;
        memset(&g, 0, sizeof g);
        g.A = dz;                   // dH = dz W^T, then times SiLU'(z of layer l-1)
        g.sam = ldz;
        g.sak = 1;
        g.B = L.wb;
        g.sbk = 1;
        g.sbn = L.out_pad;
        g.M = n;
        g.N = L.in;
        g.K = L.out_pad;
        g.epi = EPI_SILU_GRAD;
        g.zin = m->Z[l - 1];
        g.szi = HID;
        g.outh = m->dZ[pp];
        g.soh = HID;
        if (gemm(g, s) != hipSuccess) return GR_EDEVICE;
        dz = m->dZ[pp];
        ldz = HID;
        pp ^= 1;
    }
    return GR_OK;
}

int gr_mlp_adam_step(gr_mlp* m, const float* grad, float lr, float beta1, float beta2, float eps,
                     void* stream) {
    if (!m || !grad) return GR_EINVAL;
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps >= 0.0f))
        return GR_EINVAL;
    Guard guard(m->device);
    hipStream_t s = (hipStream_t)stream;
    m->step += 1;
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)m->step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)m->step)));
    if (adam(m->params, grad, m->m, m->v, m->nparam, lr, beta1, beta2, eps, c1, c2, s) !=
        hipSuccess)
        return GR_EDEVICE;
    return repack(m, s) == hipSuccess ? GR_OK : GR_EDEVICE;
}

int64_t gr_mlp_steps(const gr_mlp* m) { return m ? m->step : -1; }

}  // extern "C"

int gr_mlp_device_of(const gr_mlp* m) { return m ? m->device : -1; }

NetView gr_mlp_view(const gr_mlp* m) {
    NetView v;
    for (int l = 0; l < NLAYER; ++l) {
        v.frag[l] = m->layer[l].frag;
        v.bias[l] = m->layer[l].bias;
    }
    return v;
}
