// C-ABI entry points of libgrtrace: argument validation, context, launch
// shape, batch tables, autotuning and dispatch to the kernels.  Host code.
#include <math.h>

#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "grtrace.h"
#include "internal.h"
#include "surrogate_internal.h"

int gr_mlp_device_of(const gr_mlp* m);
gr::mlp::NetView gr_mlp_view(const gr_mlp* m);

struct gr_ctx {
    int device;
    gr_integrator integ;
    gr_launch launch;                 // user or autotuned shape (block == 0: default)
    unsigned long long* counter;      // work counter (device)
    int num_cu;
    char arch[64];
    gr::BatchInstance* table;         // batch instance table (device)
    int64_t* firsts;                  // batch prefix offsets (device)
    int64_t table_cap;                // instances the device table holds
    // surrogate-frame workspace (grown on demand)
    int64_t sw_cap;                   // pixels it holds
    float* sw_logit;                  // cap escape logits
    int32_t* sw_list;                 // fallback pixel list
    unsigned long long* sw_count;
    double* sw_out[7];                // re-traced theta, phi, r, p_t, p_r, p_theta, p_phi
    int8_t* sw_flag;                  // re-traced flags
    // frame queue order (grown on demand)
    int64_t ord_cap;                  // pixels it holds
    float* ord_keys;                  // 2 x cap
    int32_t* ord_vals;                // 2 x cap
    void* ord_temp;
    size_t ord_temp_bytes;
    // rays parked between the two launches of a Manko-Novikov frame (grown on demand)
    int64_t pk_cap;                   // rays it holds
    double* pk_y;                     // 6 x cap: t, r, theta, phi, p_r, p_theta
    int32_t* pk_steps;
    int64_t* pk_pix;
    unsigned long long* pk_count;
    unsigned char* scratch;           // this device's copy of `scratch` (device address)
};

// Device memory of gr_trace_batch_noalloc: the work counter, the prefix
// offsets and the instance table of at most GR_NOALLOC_MAX_INSTANCES
// instances, in one fixed array per device (the library holds it until the
// process ends).  Host code never passes `scratch` itself to the device: its
// name is a host-side stand-in, and each device's address comes from
// hipGetSymbolAddress (scratch_address below).
namespace {
constexpr size_t kScratchAlign = 256;
constexpr size_t round_up(size_t x) { return (x + kScratchAlign - 1) / kScratchAlign * kScratchAlign; }
constexpr size_t kScratchFirsts = kScratchAlign;     // [0, 256): the work counter
constexpr size_t kScratchTable =
    kScratchFirsts + round_up(2 * (GR_NOALLOC_MAX_INSTANCES + 1) * sizeof(int64_t));
constexpr size_t kScratchBytes =
    kScratchTable + round_up(GR_NOALLOC_MAX_INSTANCES * sizeof(gr::BatchInstance));
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
hipError_t scratch_address(int device, unsigned char** out) {
    static std::mutex mu;
    static std::vector<unsigned char*> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= addr.size()) addr.resize(device + 1, nullptr);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (unsigned char*)p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace

namespace {

thread_local char g_last_error[256] = "";

int device_error(hipError_t e, const char* where) {
    snprintf(g_last_error, sizeof g_last_error, "%s: %s", where, hipGetErrorString(e));
    return GR_EDEVICE;
}

bool finite(double x) { return isfinite(x) != 0; }

int check_integrator(const gr_integrator* in) {
    if (!in) return GR_EINVAL;
    if (!(finite(in->dt) && in->dt > 0.0)) return GR_EINVAL;
    if (!(finite(in->fd_eps) && in->fd_eps > 0.0)) return GR_EINVAL;
    if (!(in->horizon_norm > 0.0) || isnan(in->horizon_norm)) return GR_EINVAL;
    if (!(finite(in->escape_factor) && in->escape_factor > 1.0)) return GR_EINVAL;
    if (in->max_steps < 0) return GR_EINVAL;
    if (in->precision != GR_FP64 && in->precision != GR_MIXED) return GR_EINVAL;
    if (in->method != GR_RK4 && in->method != GR_EULER && in->method != GR_RK4_TIME)
        return GR_EINVAL;
    if (in->method != GR_RK4 && in->precision != GR_FP64) return GR_EUNSUPPORTED;
    if (in->disk_half_angle != 0.0) {
        if (!(in->disk_half_angle > 0.0 && in->disk_half_angle < M_PI / 2)) return GR_EINVAL;
        if (!(finite(in->disk_r_in) && finite(in->disk_r_out) && in->disk_r_in >= 0.0 &&
              in->disk_r_in < in->disk_r_out))
            return GR_EINVAL;
        if (in->precision != GR_FP64) return GR_EUNSUPPORTED;
    }
    return GR_OK;
}

bool has_disk(const gr_integrator& in) { return in.disk_half_angle > 0.0; }

// Flat space (M = Q = 0, any a: oblate spheroidal coordinates) has no horizon.
bool is_flat(const gr_metric* m) { return m->M == 0.0 && m->Q == 0.0; }

double horizon(const gr_metric* m) {
    if (is_flat(m)) return 0.0;
    return m->M + sqrt(m->M * m->M - m->a * m->a - m->Q * m->Q);
}

int check_metric(const gr_metric* m) {
    if (!m) return GR_EINVAL;
    if (!(finite(m->M) && finite(m->a) && finite(m->Q))) return GR_EINVAL;
    if (m->M < 0.0) return GR_EINVAL;
    if (is_flat(m)) return GR_OK;
    if (m->a * m->a + m->Q * m->Q > m->M * m->M) return GR_EINVAL;   // naked singularity
    return GR_OK;
}

int check_camera(const gr_metric* m, const gr_camera* c) {
    if (!c) return GR_EINVAL;
    if (!(finite(c->r0) && finite(c->theta0) && finite(c->phi0) && finite(c->fov)))
        return GR_EINVAL;
    if (!(c->r0 > horizon(m))) return GR_EINVAL;
    if (!(c->theta0 > 0.0 && c->theta0 < M_PI)) return GR_EINVAL;
    if (!(c->fov > 0.0 && c->fov < M_PI)) return GR_EINVAL;
    if (c->width < 1 || c->height < 1) return GR_EINVAL;
    if ((int64_t)c->width * (int64_t)c->height > ((int64_t)1 << 40)) return GR_EINVAL;
    return GR_OK;
}

int check_output(const gr_output* o) {
    if (!o || !o->flag) return GR_EINVAL;
    if (o->dtype != GR_F64 && o->dtype != GR_F32) return GR_EINVAL;
    return GR_OK;
}

// The context's launch shape, else the default for frames or batches: frames
// one ray per lane over 8x8 pixel tiles in workgroups of 64 (neighbouring
// pixels take nearly the same number of steps, so a wave's lanes stay busy
// without refill, and the step needs fewer registers); batches refill in
// workgroups of 256, instances with the longest rays first.
gr_launch effective_launch(const gr_ctx* ctx, bool batch = false) {
    gr_launch l = ctx->launch;
    if (l.block == 0) {
        l.waves_per_simd = 0;
        if (batch) {
            l.block = 256;
            l.refill = 1;
            l.order = 1;
        } else {
            l.block = 64;
            l.refill = 0;
            l.order = 0;
        }
    }
    return l;
}

// Grid for a persistent launch of `nray` rays with `per_cu_max` resident
// workgroups per CU.
gr::LaunchShape resident_shape(const gr_ctx* ctx, const gr_launch& l, int per_cu_max,
                               int64_t nray) {
    gr::LaunchShape L;
    L.block = l.block;
    L.refill = 1;
    int per_cu = std::max(1, per_cu_max);
    if (l.waves_per_simd > 0) {
        const int waves_per_block = L.block / 64;
        const int want = std::max(1, (l.waves_per_simd * 4) / waves_per_block);
        per_cu = std::min(per_cu, want);
    }
    const int64_t blocks_needed = (nray + L.block - 1) / L.block;
    const int64_t resident = (int64_t)per_cu * ctx->num_cu;
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>(resident, blocks_needed));
    return L;
}

// Grid of a frame launch: persistent, or (no refill) one lane per ray with
// whole 8x8 pixel tiles per wave when the frame has no pixel list.
gr::LaunchShape frame_shape(const gr_ctx* ctx, const gr::FrameArgs& A, bool f32_out) {
    const gr_launch l = effective_launch(ctx);
    const bool mixed = ctx->integ.precision == GR_MIXED;
    const int64_t nray = A.nray;
    int64_t lanes = nray;
    if (!A.pixels) lanes = 64 * (((int64_t)A.cam.W + 7) / 8) * (((int64_t)A.cam.H + 7) / 8);
    const int64_t blocks = (lanes + l.block - 1) / l.block;
    if (!l.refill && blocks <= INT32_MAX) {    // larger grids take the persistent form
        gr::LaunchShape L;
        L.block = l.block;
        L.refill = 0;
        L.grid = (int)std::max<int64_t>(1, blocks);
        return L;
    }
    return resident_shape(ctx, l,
                          mixed ? gr::occupancy_trace_mixed(l.block, f32_out)
                                : gr::occupancy_trace_fp64(l.block, f32_out),
                          nray);
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

gr::Integrator device_integrator(const gr_integrator& in) {
    gr::Integrator I;
    I.dt = in.dt;
    I.eps = in.fd_eps;
    I.inv_eps = 1.0 / in.fd_eps;
    gr::sincos_def(in.fd_eps, I.sin_eps, I.cos_eps);
    I.scale = -0.5 * (1.0 / in.fd_eps);
    I.hnorm = in.horizon_norm;
    I.esc_factor = in.escape_factor;
    I.disk_r_in = in.disk_r_in;
    I.disk_r_out = in.disk_r_out;
    I.disk_dth = in.disk_half_angle;
    I.max_steps = in.max_steps;
    return I;
}

gr::OutPtrs out_ptrs(const gr_output* o) {
    gr::OutPtrs p;
    p.t = o->t;
    p.r = o->r;
    p.th = o->theta;
    p.ph = o->phi;
    p.pt = o->p_t;
    p.pr = o->p_r;
    p.pth = o->p_theta;
    p.pph = o->p_phi;
    p.flag = o->flag;
    p.steps = o->steps;
    return p;
}

gr::FrameArgs frame_args(const gr_ctx* ctx, const gr_metric* m, const gr_camera* c,
                         const gr_output* o, const int32_t* pixels, int64_t nray) {
    gr::FrameArgs A;
    memset(&A, 0, sizeof A);
    A.hole = gr::make_hole(m->M, m->a, m->Q);
    A.cam = gr::make_camera(A.hole, c->r0, c->theta0, c->phi0, c->fov, c->width, c->height);
    A.in = device_integrator(ctx->integ);
    A.r_esc = ctx->integ.escape_factor * c->r0;
    A.nray = nray;
    A.pixels = pixels;
    A.out = out_ptrs(o);
    return A;
}

int64_t instance_rays(const gr_instance* I) {
    return I->n_pixels < 0 ? (int64_t)I->camera.width * I->camera.height : I->n_pixels;
}

int validate_batch(const gr_ctx* ctx, const gr_instance* inst, int32_t n) {
    if (!ctx || !inst || n < 1) return GR_EINVAL;
    if (ctx->integ.method != GR_RK4 || has_disk(ctx->integ)) return GR_EUNSUPPORTED;
    for (int32_t k = 0; k < n; ++k) {
        const gr_instance* I = &inst[k];
        int rc = check_metric(&I->metric);
        if (!rc) rc = check_camera(&I->metric, &I->camera);
        if (rc) return rc;
        if (I->n_pixels < -1) return GR_EINVAL;
        if (instance_rays(I) == 0) continue;
        rc = check_output(&I->out);
        if (rc) return rc;
        if (I->n_pixels > 0 && !I->pixels) return GR_EINVAL;
    }
    if (ctx->integ.precision != GR_FP64) return GR_EUNSUPPORTED;
    return GR_OK;
}

// Build and upload the instance table; returns the total ray count in *total.
// Critical impact parameter of the Reissner-Nordstrom hole with the same M
// and Q (photon sphere r_ph = (3M + sqrt(9M^2 - 8Q^2))/2): the centre of the
// ring of longest rays (queue order; the surrogate's impact rule).
double critical_impact(const gr_metric* m) {
    if (!(m->M > 0.0)) return 0.0;
    const double M = m->M, Q2 = m->Q * m->Q;
    const double rph = 0.5 * (3.0 * M + sqrt(std::max(9.0 * M * M - 8.0 * Q2, 0.0)));
    const double f = 1.0 - 2.0 * M / rph + Q2 / (rph * rph);
    return f > 0.0 ? rph / sqrt(f) : 0.0;
}

// Constants of the surrogate's features and Reissner-Nordstrom baseline.
gr::SurConst sur_constants(const gr_metric* m, const gr_camera* c, double r_esc) {
    gr::SurConst S;
    memset(&S, 0, sizeof S);
    const double M = m->M, Q2 = m->Q * m->Q, Mn = M > 0.0 ? M : 1.0;
    S.feat[0] = (float)(m->a / Mn);
    S.feat[1] = (float)(fabs(m->Q) / Mn);
    S.feat[2] = (float)c->theta0;
    S.feat[3] = (float)(c->r0 / (50.0 * Mn));
    S.feat[4] = (float)c->fov;
    S.st = sin(c->theta0);
    S.ct = cos(c->theta0);
    S.sp = sin(c->phi0);
    S.cp = cos(c->phi0);
    S.r0 = c->r0;
    S.R = r_esc;
    S.u0 = 1.0 / c->r0;
    S.u1 = 1.0 / r_esc;
    S.M = M;
    S.Q2 = Q2;
    const double f0 = 1.0 - (2.0 * M - Q2 / c->r0) / c->r0;
    S.bscale = f0 > 0.0 ? c->r0 / sqrt(f0) : 0.0;
    const double bc = critical_impact(m);
    S.inv_bc = bc > 0.0 ? 1.0 / bc : 0.0;
    if (M > 0.0)
        S.uph = Q2 > 0.0 ? (3.0 * M - sqrt(std::max(9.0 * M * M - 8.0 * Q2, 0.0))) / (4.0 * Q2)
                         : 1.0 / (3.0 * M);
    return S;
}

gr::BatchInstance batch_instance(const gr_ctx* ctx, const gr_instance* I) {
    gr::BatchInstance B;
    memset(&B, 0, sizeof B);
    B.hole = gr::make_hole(I->metric.M, I->metric.a, I->metric.Q);
    B.cam = gr::make_camera(B.hole, I->camera.r0, I->camera.theta0, I->camera.phi0,
                            I->camera.fov, I->camera.width, I->camera.height);
    B.r_esc = ctx->integ.escape_factor * I->camera.r0;
    B.pixels = I->n_pixels < 0 ? nullptr : I->pixels;
    B.out = out_ptrs(&I->out);
    B.f32 = I->out.dtype == GR_F32;
    B.sur = sur_constants(&I->metric, &I->camera, B.r_esc);
    return B;
}

// Device table capacity for m instances (m + 1 prefix offsets).
int reserve_table(gr_ctx* ctx, int64_t m) {
    if (m <= ctx->table_cap) return GR_OK;
    const int64_t cap = std::max<int64_t>(m, 2 * ctx->table_cap);
    gr::BatchInstance* t = nullptr;
    int64_t* f = nullptr;
    if (hipMalloc(&t, cap * sizeof(gr::BatchInstance)) != hipSuccess) return GR_ENOMEM;
    if (hipMalloc(&f, 2 * (cap + 1) * sizeof(int64_t)) != hipSuccess) {
        hipFree(t);
        return GR_ENOMEM;
    }
    // the old table may still be read by queued work on another stream the
    // caller synchronises; free after the device is idle for this context
    hipDeviceSynchronize();
    hipFree(ctx->table);
    hipFree(ctx->firsts);
    ctx->table = t;
    ctx->firsts = f;
    ctx->table_cap = cap;
    return GR_OK;
}

// Device buffers of a batch: instance table, prefix offsets, work counter.
struct BatchBuffers {
    gr::BatchInstance* table;
    int64_t* firsts;
    unsigned long long* counter;
};

// Non-empty instances of a batch.
int64_t nonempty_instances(const gr_instance* inst, int32_t n) {
    int64_t m = 0;
    for (int32_t k = 0; k < n; ++k) m += instance_rays(&inst[k]) > 0;
    return m;
}

// dst == nullptr: the context's table, grown with hipMalloc as needed.
// Otherwise dst must hold the batch (the caller checked its size).
int upload_batch(gr_ctx* ctx, const gr_instance* inst, int32_t n, int order,
                 hipStream_t s, int32_t* ninst, int64_t* total, int64_t* waves = nullptr,
                 const BatchBuffers* dst = nullptr) {
    std::vector<int32_t> idx;
    for (int32_t k = 0; k < n; ++k)
        if (instance_rays(&inst[k]) > 0) idx.push_back(k);
    if (order == 1) {
        // longest expected rays first: path length grows with the escape radius
        std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) {
            return inst[x].camera.r0 > inst[y].camera.r0;
        });
    }
    const int64_t m = (int64_t)idx.size();
    std::vector<gr::BatchInstance> tab(m);
    // ray offsets, then wave offsets (8x8 tiles of a frame, 64 list entries)
    std::vector<int64_t> firsts(2 * (m + 1), 0);
    int64_t* wf = firsts.data() + m + 1;
    for (int64_t q = 0; q < m; ++q) {
        const gr_instance* I = &inst[idx[q]];
        tab[q] = batch_instance(ctx, I);
        const int64_t n = instance_rays(I);
        firsts[q + 1] = firsts[q] + n;
        const int64_t nw = I->n_pixels < 0 ? ((int64_t)I->camera.width + 7) / 8 *
                                                 (((int64_t)I->camera.height + 7) / 8)
                                           : (n + 63) / 64;
        wf[q + 1] = wf[q] + nw;
    }
    *ninst = (int32_t)m;
    *total = firsts[m];
    if (waves) *waves = wf[m];
    if (m == 0) return GR_OK;
    gr::BatchInstance* table = dst ? dst->table : nullptr;
    int64_t* dfirsts = dst ? dst->firsts : nullptr;
    if (!dst) {
        int rc = reserve_table(ctx, m);
        if (rc) return rc;
        table = ctx->table;
        dfirsts = ctx->firsts;
    }
    // pageable sources: the copies are staged before hipMemcpyAsync returns
    hipError_t e = hipMemcpyAsync(table, tab.data(), m * sizeof(gr::BatchInstance),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dfirsts, firsts.data(), 2 * (m + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_error(e, "batch table upload");
    return GR_OK;
}

int run_batch(gr_ctx* ctx, const gr_instance* inst, int32_t n, const gr_launch& l,
              hipStream_t s, const BatchBuffers* dst = nullptr) {
    int32_t ninst = 0;
    int64_t total = 0, waves = 0;
    int rc = upload_batch(ctx, inst, n, l.order, s, &ninst, &total, &waves, dst);
    if (rc) return rc;
    if (total == 0) return GR_OK;
    const BatchBuffers buf = dst ? *dst : BatchBuffers{ctx->table, ctx->firsts, ctx->counter};
    gr::BatchArgs B;
    memset(&B, 0, sizeof B);
    B.in = device_integrator(ctx->integ);
    B.inst = buf.table;
    B.firsts = buf.firsts;
    B.wfirsts = buf.firsts + ninst + 1;
    B.ninst = ninst;
    B.total = total;
    gr::LaunchShape L;
    const int64_t blocks = (64 * waves + l.block - 1) / l.block;
    if (!l.refill && blocks <= INT32_MAX) {
        L.block = l.block;
        L.refill = 0;
        L.grid = (int)blocks;
    } else {
        L = resident_shape(ctx, l, gr::occupancy_trace_fp64_batch(l.block), total);
    }
    hipError_t e = gr::launch_trace_fp64_batch(B, L, buf.counter, s);
    if (e != hipSuccess) return device_error(e, "trace_fp64_batch launch");
    return GR_OK;
}

// ---------------------------------------------------------------- autotune cache
// One JSON object per line:
// {"key": "...", "block": B, "waves_per_simd": W, "refill": R, "order": O, "ms": T}
std::string cache_key(const gr_ctx* ctx, int64_t total, int32_t ninst) {
    int lg = 0;
    while (((int64_t)1 << (lg + 1)) <= total) ++lg;
    int ln = 0;
    while ((1 << (ln + 1)) <= ninst) ++ln;
    char buf[160];
    snprintf(buf, sizeof buf, "%s/trace_fp64_batch/rays2^%d/inst2^%d", ctx->arch, lg, ln);
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, gr_launch* out) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        const std::string pat = "\"key\": \"" + key + "\"";
        if (!strstr(line, pat.c_str())) continue;
        gr_launch l;
        const char* p;
        if ((p = strstr(line, "\"block\": ")) && sscanf(p, "\"block\": %d", &l.block) == 1 &&
            (p = strstr(line, "\"waves_per_simd\": ")) &&
            sscanf(p, "\"waves_per_simd\": %d", &l.waves_per_simd) == 1 &&
            (p = strstr(line, "\"order\": ")) && sscanf(p, "\"order\": %d", &l.order) == 1) {
            l.refill = 1;
            if ((p = strstr(line, "\"refill\": ")) && sscanf(p, "\"refill\": %d", &l.refill) == 1 &&
                l.refill != 0)
                l.refill = 1;
            *out = l;      // the last matching line wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_append(const char* path, const std::string& key, const gr_launch& l, double ms) {
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"key\": \"%s\", \"block\": %d, \"waves_per_simd\": %d, \"refill\": %d, "
            "\"order\": %d, \"ms\": %.3f}\n",
            key.c_str(), l.block, l.waves_per_simd, l.refill, l.order, ms);
    fclose(f);
}

int check_instance_geometry(const gr_instance* inst, int32_t n) {
    if (!inst || n < 1) return GR_EINVAL;
    for (int32_t k = 0; k < n; ++k) {
        const gr_instance* I = &inst[k];
        int rc = check_metric(&I->metric);
        if (!rc) rc = check_camera(&I->metric, &I->camera);
        if (rc) return rc;
        if (I->n_pixels < -1) return GR_EINVAL;
        if (I->n_pixels > 0 && !I->pixels) return GR_EINVAL;
    }
    return GR_OK;
}

void free_surrogate_ws(gr_ctx* c) {
    hipFree(c->sw_logit);
    hipFree(c->sw_list);
    hipFree(c->sw_count);
    for (int k = 0; k < 7; ++k) hipFree(c->sw_out[k]);
    hipFree(c->sw_flag);
    c->sw_logit = nullptr;
    c->sw_list = nullptr;
    c->sw_count = nullptr;
    for (int k = 0; k < 7; ++k) c->sw_out[k] = nullptr;
    c->sw_flag = nullptr;
    c->sw_cap = 0;
}

void free_order_ws(gr_ctx* c) {
    hipFree(c->ord_keys);
    hipFree(c->ord_vals);
    hipFree(c->ord_temp);
    c->ord_keys = nullptr;
    c->ord_vals = nullptr;
    c->ord_temp = nullptr;
    c->ord_cap = 0;
    c->ord_temp_bytes = 0;
}

int grow_order_ws(gr_ctx* c, int64_t n) {
    if (n <= c->ord_cap) return GR_OK;
    hipDeviceSynchronize();
    free_order_ws(c);
    const size_t tb = gr::frame_order_temp(n);
    bool ok = hipMalloc(&c->ord_keys, 2 * n * sizeof(float)) == hipSuccess &&
              hipMalloc(&c->ord_vals, 2 * n * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&c->ord_temp, tb > 0 ? tb : 1) == hipSuccess;
    if (!ok) {
        free_order_ws(c);
        return GR_ENOMEM;
    }
    c->ord_cap = n;
    c->ord_temp_bytes = tb;
    return GR_OK;
}

void free_park_ws(gr_ctx* c) {
    hipFree(c->pk_y);
    hipFree(c->pk_steps);
    hipFree(c->pk_pix);
    hipFree(c->pk_count);
    c->pk_y = nullptr;
    c->pk_steps = nullptr;
    c->pk_pix = nullptr;
    c->pk_count = nullptr;
    c->pk_cap = 0;
}

// Room for n parked rays (at most PARK_MAX; rays past it finish in the first launch).
constexpr int64_t PARK_MAX = (int64_t)1 << 22;

int grow_park_ws(gr_ctx* c, int64_t n) {
    n = std::min(n, PARK_MAX);
    if (n <= c->pk_cap) return GR_OK;
    hipDeviceSynchronize();
    free_park_ws(c);
    bool ok = hipMalloc(&c->pk_y, 6 * n * sizeof(double)) == hipSuccess &&
              hipMalloc(&c->pk_steps, n * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&c->pk_pix, n * sizeof(int64_t)) == hipSuccess &&
              hipMalloc(&c->pk_count, sizeof(unsigned long long)) == hipSuccess;
    if (!ok) {
        free_park_ws(c);
        return GR_ENOMEM;
    }
    c->pk_cap = n;
    return GR_OK;
}

int grow_surrogate_ws(gr_ctx* c, int64_t n) {
    if (n <= c->sw_cap) return GR_OK;
    hipDeviceSynchronize();
    free_surrogate_ws(c);
    bool ok = hipMalloc(&c->sw_logit, n * sizeof(float)) == hipSuccess &&
              hipMalloc(&c->sw_list, n * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&c->sw_count, sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&c->sw_flag, n) == hipSuccess;
    for (int k = 0; k < 7 && ok; ++k) ok = hipMalloc(&c->sw_out[k], n * sizeof(double)) == hipSuccess;
    if (!ok) {
        free_surrogate_ws(c);
        return GR_ENOMEM;
    }
    c->sw_cap = n;
    return GR_OK;
}

// Validation of a Manko-Novikov spacetime and a camera outside its horizon.
int check_mn(const gr_metric_mn* m, const gr_camera* c, gr::MnHole* K) {
    if (!m || !c) return GR_EINVAL;
    if (!(std::isfinite(m->M) && std::isfinite(m->S) && std::isfinite(m->q))) return GR_EINVAL;
    if (!(m->M > 0.0) || m->S == 0.0 || !(fabs(m->S) < m->M * m->M)) return GR_EINVAL;
    *K = gr::make_mn_hole(m->M, m->S, m->q);
    if (!(K->k > 0.0 && std::isfinite(K->beta))) return GR_EINVAL;
    if (!(std::isfinite(c->r0) && std::isfinite(c->theta0) && std::isfinite(c->phi0) &&
          std::isfinite(c->fov)))
        return GR_EINVAL;
    if (!(c->r0 > m->M + K->k)) return GR_EINVAL;
    if (!(c->theta0 > 0.0 && c->theta0 < M_PI) || !(c->fov > 0.0 && c->fov < M_PI))
        return GR_EINVAL;
    if (c->width < 1 || c->height < 1 ||
        (int64_t)c->width * (int64_t)c->height > ((int64_t)1 << 40))
        return GR_EINVAL;
    return GR_OK;
}

int redshift_common(gr_ctx* ctx, const gr::Hole& H, const gr::MnHole& K, bool mn, double nu_o,
                    const gr_output* out, int64_t n, void* z, void* hip_stream) {
    int rc = check_output(out);
    if (rc) return rc;
    if (!z || n < 0 || !out->r || !out->theta || !out->p_t || !out->p_phi) return GR_EINVAL;
    DeviceGuard guard(ctx->device);
    const hipError_t e = gr::launch_redshift(H, K, mn, device_integrator(ctx->integ), nu_o,
                                             out_ptrs(out), out->dtype == GR_F32, n, z,
                                             (hipStream_t)hip_stream);
    if (e != hipSuccess) return device_error(e, "redshift launch");
    return GR_OK;
}

}  // namespace

extern "C" {

int gr_trace_init(gr_ctx** ctx, int device, const gr_integrator* integ) {
    if (!ctx) return GR_EINVAL;
    *ctx = nullptr;
    int rc = check_integrator(integ);
    if (rc) return rc;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return device_error(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return GR_EINVAL;
    DeviceGuard guard(device);
    gr_ctx* c = new (std::nothrow) gr_ctx;
    if (!c) return GR_ENOMEM;
    memset(c, 0, sizeof *c);
    c->device = device;
    c->integ = *integ;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return device_error(e, "hipGetDeviceProperties");
    }
    c->num_cu = prop.multiProcessorCount;
    snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    for (char* p = c->arch; *p; ++p)
        if (*p == ':') *p = '\0';      // drop feature suffixes such as ":sramecc+"
    e = scratch_address(device, &c->scratch);
    if (e != hipSuccess) {
        delete c;
        return device_error(e, "hipGetSymbolAddress(scratch)");
    }
    e = hipMalloc(&c->counter, sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete c;
        device_error(e, "hipMalloc");
        return GR_ENOMEM;
    }
    *ctx = c;
    return GR_OK;
}

int gr_trace_set_integrator(gr_ctx* ctx, const gr_integrator* integ) {
    if (!ctx) return GR_EINVAL;
    const int rc = check_integrator(integ);
    if (rc) return rc;
    ctx->integ = *integ;
    return GR_OK;
}

int gr_trace_set_launch(gr_ctx* ctx, const gr_launch* l) {
    if (!ctx) return GR_EINVAL;
    if (!l) {
        memset(&ctx->launch, 0, sizeof ctx->launch);
        return GR_OK;
    }
    if (l->block != 64 && l->block != 128 && l->block != 256) return GR_EINVAL;
    if (l->waves_per_simd < 0 || l->waves_per_simd > 8) return GR_EINVAL;
    if (l->refill != 0 && l->refill != 1) return GR_EINVAL;
    if (l->order < 0 || l->order > 2) return GR_EINVAL;
    ctx->launch = *l;
    return GR_OK;
}

int gr_trace_get_launch(const gr_ctx* ctx, gr_launch* l) {
    if (!ctx || !l) return GR_EINVAL;
    *l = effective_launch(ctx);
    return GR_OK;
}

int gr_trace_frame(gr_ctx* ctx, const gr_metric* m, const gr_camera* c, const gr_output* out,
                   void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    int rc = check_metric(m);
    if (!rc) rc = check_camera(m, c);
    if (!rc) rc = check_output(out);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    const int64_t nray = (int64_t)c->width * c->height;
    const bool f32 = out->dtype == GR_F32;
    gr::FrameArgs A = frame_args(ctx, m, c, out, nullptr, nray);
    hipError_t e;
    const gr_launch l0 = effective_launch(ctx);
    if (l0.refill && l0.order == 2 && nray >= 4096) {
        // near-critical rays first (results do not depend on the order)
        rc = grow_order_ws(ctx, nray);
        if (rc) return rc;
        e = gr::frame_order(A.hole, A.cam, critical_impact(m), nray, ctx->ord_keys,
                            ctx->ord_vals, ctx->ord_temp, ctx->ord_temp_bytes,
                            (hipStream_t)hip_stream);
        if (e != hipSuccess) return device_error(e, "frame order");
        A.order = ctx->ord_vals + nray;
    }
    if (ctx->integ.precision == GR_MIXED) {
        const gr::LaunchShape L = frame_shape(ctx, A, f32);
        e = gr::launch_trace_mixed(A, horizon(m), f32, L, ctx->counter,
                                   (hipStream_t)hip_stream);
        if (e != hipSuccess) return device_error(e, "trace_mixed launch");
        return GR_OK;
    }
    gr::LaunchShape L = frame_shape(ctx, A, f32);
    const int method = ctx->integ.method;
    const bool disk = has_disk(ctx->integ);
    if ((method != GR_RK4 || disk) && L.refill) {
        // the other methods and the ring exist in the one-ray-per-lane kernel only
        const int64_t tiles = ((int64_t)c->width + 7) / 8 * (((int64_t)c->height + 7) / 8);
        if (tiles > INT32_MAX) return GR_EUNSUPPORTED;
        L.block = 64;
        L.refill = 0;
        L.grid = (int)tiles;
    }
    e = gr::launch_trace_fp64(A, f32, method, disk, L, ctx->counter, (hipStream_t)hip_stream);
    if (e != hipSuccess) return device_error(e, "trace_fp64 launch");
    return GR_OK;
}

int gr_trace_frame_mn(gr_ctx* ctx, const gr_metric_mn* m, const gr_camera* c,
                      const gr_output* out, void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    gr::MnHole K;
    int rc = check_mn(m, c, &K);
    if (rc) return rc;
    rc = check_output(out);
    if (rc) return rc;
    if (ctx->integ.precision != GR_FP64) return GR_EUNSUPPORTED;
    DeviceGuard guard(ctx->device);
    const int64_t nray = (int64_t)c->width * c->height;
    gr::FrameArgs A;
    memset(&A, 0, sizeof A);
    A.cam = gr::make_camera_mn(K, c->r0, c->theta0, c->phi0, c->fov, c->width, c->height);
    A.in = device_integrator(ctx->integ);
    A.r_esc = ctx->integ.escape_factor * c->r0;
    A.nray = nray;
    A.out = out_ptrs(out);
    gr::LaunchShape L;
    L.block = 64;
    L.refill = 0;
    const int64_t blocks = ((int64_t)c->width + 7) / 8 * (((int64_t)c->height + 7) / 8);
    if (blocks > INT32_MAX) return GR_EINVAL;
    L.grid = (int)blocks;
    // Park the rays still running after a quarter of the step limit and
    // continue them together in a second launch (without the workspace, one
    // launch does everything).
    gr::Parked park;
    memset(&park, 0, sizeof park);
    gr::LaunchShape L2 = L;
    const int32_t cap = ctx->integ.max_steps >= 4096 ? ctx->integ.max_steps / 4 : 0;
    if (cap > 0 && grow_park_ws(ctx, nray) == GR_OK) {
        park.y = ctx->pk_y;
        park.steps = ctx->pk_steps;
        park.pix = ctx->pk_pix;
        park.count = ctx->pk_count;
        park.capacity = std::min(nray, ctx->pk_cap);
        park.cap = cap;
        const int64_t resident =
            (int64_t)std::max(1, gr::occupancy_trace_mn_resume(64)) * ctx->num_cu;
        L2.grid = (int)std::max<int64_t>(1, std::min(resident, (park.capacity + 63) / 64));
    }
    const hipError_t e = gr::launch_trace_mn(A, K, out->dtype == GR_F32,
                                             ctx->integ.method, has_disk(ctx->integ), L, park,
                                             L2,
                                             (hipStream_t)hip_stream);
    if (e != hipSuccess) return device_error(e, "trace_mn launch");
    return GR_OK;
}

int gr_redshift(gr_ctx* ctx, const gr_metric* m, const gr_camera* c, const gr_output* out,
                int64_t n, void* z, void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    int rc = check_metric(m);
    if (!rc) rc = check_camera(m, c);
    if (rc) return rc;
    const gr::Hole H = gr::make_hole(m->M, m->a, m->Q);
    const gr::InvMetric g0 =
        gr::inverse_metric(H, gr::radial_terms(H, c->r0), gr::theta_terms(H, c->theta0));
    gr::MnHole K;
    memset(&K, 0, sizeof K);
    return redshift_common(ctx, H, K, false, sqrt(-1.0 / g0.tt), out, n, z, hip_stream);
}

int gr_redshift_mn(gr_ctx* ctx, const gr_metric_mn* m, const gr_camera* c, const gr_output* out,
                   int64_t n, void* z, void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    gr::MnHole K;
    const int rc = check_mn(m, c, &K);
    if (rc) return rc;
    double s, co;
    gr::sincos_def(c->theta0, s, co);
    const gr::InvMetric g0 = gr::mn_inverse_metric<gr::IeeeDiv>(K, c->r0, co, s * s);
    gr::Hole H;
    memset(&H, 0, sizeof H);
    return redshift_common(ctx, H, K, true, sqrt(-1.0 / g0.tt), out, n, z, hip_stream);
}

int gr_shade_frame(const gr_shade* sh, const gr_output* out, int64_t n, uint32_t* rgba,
                   void* hip_stream) {
    if (!sh || !rgba || n < 0) return GR_EINVAL;
    int rc = check_output(out);
    if (rc) return rc;
    if (sh->mode == GR_SHADE_BANDS) {
        if (!out->theta || !out->phi) return GR_EINVAL;
    } else if (sh->mode == GR_SHADE_TIME) {
        if (!out->t || !(sh->t_max > 0.0) || !(sh->band >= 0.0) || !std::isfinite(sh->band))
            return GR_EINVAL;
    } else if (sh->mode == GR_SHADE_TEXTURE) {
        if (!out->theta || !out->phi || !sh->texture || sh->tex_width < 1 || sh->tex_height < 1)
            return GR_EINVAL;
    } else {
        return GR_EINVAL;
    }
    const hipError_t e = gr::launch_shade(sh->mode, out_ptrs(out), out->dtype == GR_F32, n,
                                          sh->t_max, sh->band, sh->texture, sh->tex_width,
                                          sh->tex_height, rgba, (hipStream_t)hip_stream);
    if (e != hipSuccess) return device_error(e, "shade launch");
    return GR_OK;
}

int gr_trace_batch(gr_ctx* ctx, const gr_instance* inst, int32_t n, void* hip_stream) {
    const int rc = validate_batch(ctx, inst, n);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    return run_batch(ctx, inst, n, effective_launch(ctx, true), (hipStream_t)hip_stream);
}

int gr_trace_batch_noalloc(gr_ctx* ctx, const gr_instance* inst, int32_t n, void* hip_stream) {
    const int rc = validate_batch(ctx, inst, n);
    if (rc) return rc;
    const int64_t m = nonempty_instances(inst, n);
    if (m > GR_NOALLOC_MAX_INSTANCES) {
        snprintf(g_last_error, sizeof g_last_error,
                 "gr_trace_batch_noalloc: %lld instances with rays exceed the maximum of %d",
                 (long long)m, GR_NOALLOC_MAX_INSTANCES);
        return GR_EINVAL;
    }
    DeviceGuard guard(ctx->device);
    const BatchBuffers dst{(gr::BatchInstance*)(ctx->scratch + kScratchTable),
                           (int64_t*)(ctx->scratch + kScratchFirsts),
                           (unsigned long long*)ctx->scratch};
    return run_batch(ctx, inst, n, effective_launch(ctx, true), (hipStream_t)hip_stream, &dst);
}

int gr_trace_autotune(gr_ctx* ctx, const gr_instance* inst, int32_t n, int32_t trial_steps,
                      const char* cache_path, gr_launch* best, void* hip_stream) {
    int rc = validate_batch(ctx, inst, n);
    if (rc) return rc;
    if (trial_steps < 0) return GR_EINVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    int64_t total = 0;
    int32_t ninst = 0;
    for (int32_t k = 0; k < n; ++k) {
        total += instance_rays(&inst[k]);
        ninst += instance_rays(&inst[k]) > 0;
    }
    const std::string key = cache_key(ctx, total, ninst);
    gr_launch win;
    bool have = cache_path && cache_lookup(cache_path, key, &win);
    if (!have) {
        const gr_integrator full = ctx->integ;
        if (trial_steps > 0 && trial_steps < full.max_steps) ctx->integ.max_steps = trial_steps;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            ctx->integ = full;
            return device_error(hipGetLastError(), "hipEventCreate");
        }
        double best_ms = 1e300;
        const int blocks[3] = {64, 128, 256};
        const int waves[2] = {2, 0};
        // persistent shapes, then one ray per lane (waves_per_simd does not apply)
        for (int refill = 1; refill >= 0 && !rc; --refill)
        for (int order = 0; order <= 1 && !rc; ++order)
            for (int b = 0; b < 3 && !rc; ++b)
                for (int w = 0; w < (refill ? 2 : 1) && !rc; ++w) {
                    gr_launch l;
                    l.block = blocks[b];
                    l.waves_per_simd = refill ? waves[w] : 0;
                    l.refill = refill;
                    l.order = order;
                    hipEventRecord(e0, s);
                    rc = run_batch(ctx, inst, n, l, s);
                    hipEventRecord(e1, s);
                    if (rc) break;
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        rc = device_error(hipGetLastError(), "autotune trial");
                        break;
                    }
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    if (ms < best_ms) {
                        best_ms = ms;
                        win = l;
                    }
                }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        ctx->integ = full;
        if (rc) return rc;
        if (cache_path) cache_append(cache_path, key, win, best_ms);
    }
    ctx->launch = win;
    if (best) *best = win;
    return run_batch(ctx, inst, n, win, s);
}

int gr_surrogate_inputs(gr_ctx* ctx, const gr_instance* inst, int32_t n, float* x,
                        float* u_flat, void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    int rc = check_instance_geometry(inst, n);
    if (rc) return rc;
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) total += instance_rays(&inst[k]);
    if (total > 0 && (!x || !u_flat)) return GR_EINVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t ninst = 0;
    rc = upload_batch(ctx, inst, n, 0, s, &ninst, &total);
    if (rc || total == 0) return rc;
    hipError_t e = gr::sur::inputs(ctx->table, ctx->firsts, ninst, total, x, u_flat, s);
    return e == hipSuccess ? GR_OK : device_error(e, "surrogate inputs");
}

int gr_surrogate_targets(gr_ctx* ctx, const gr_instance* inst, int32_t n, const float* u_flat,
                         float* target, void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    int rc = check_instance_geometry(inst, n);
    if (rc) return rc;
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) {
        const gr_instance* I = &inst[k];
        total += instance_rays(I);
        if (instance_rays(I) == 0) continue;
        const gr_output& o = I->out;
        if (check_output(&o) || !o.theta || !o.phi || !o.r || !o.p_t || !o.p_r || !o.p_theta ||
            !o.p_phi)
            return GR_EINVAL;
    }
    if (total > 0 && (!u_flat || !target)) return GR_EINVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t ninst = 0;
    rc = upload_batch(ctx, inst, n, 0, s, &ninst, &total);
    if (rc || total == 0) return rc;
    hipError_t e = gr::sur::targets(ctx->table, ctx->firsts, ninst, total, u_flat, target, s);
    return e == hipSuccess ? GR_OK : device_error(e, "surrogate targets");
}

int gr_surrogate_frame(gr_ctx* ctx, gr_mlp* mlp, const gr_metric* m, const gr_camera* c,
                       const gr_fallback* rule, int8_t* flag, float* dir, int8_t* fallback,
                       int64_t* n_fallback, void* hip_stream) {
    if (!ctx || !mlp || !rule || !flag || !dir || !fallback) return GR_EINVAL;
    int rc = check_metric(m);
    if (!rc) rc = check_camera(m, c);
    if (rc) return rc;
    const float logit_min = rule->logit_min, max_gain = rule->max_gain;
    const int32_t edge_px = rule->edge_px;
    if (!(logit_min >= 0.0f) || edge_px < 0 || edge_px > 16) return GR_EINVAL;
    if (!(max_gain >= 0.0f && max_gain <= 1e6f)) return GR_EINVAL;
    if (!(rule->min_impact >= 0.0f && rule->min_impact <= 1e3f)) return GR_EINVAL;
    // a turn of max_gain pixel widths (fov / width) as a chord of unit vectors
    const double turn = std::min((double)max_gain * (c->fov / c->width), M_PI);
    const float chord = max_gain > 0.0f ? (float)(2.0 * sin(0.5 * turn)) : 0.0f;
    if (ctx->integ.precision != GR_FP64 || ctx->integ.method != GR_RK4 || has_disk(ctx->integ))
        return GR_EUNSUPPORTED;
    if (gr_mlp_device_of(mlp) != ctx->device) return GR_EINVAL;
    const int64_t npix = (int64_t)c->width * c->height;
    if (npix > ((int64_t)1 << 31) - 1) return GR_EINVAL;
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    rc = grow_surrogate_ws(ctx, npix);
    if (rc) return rc;
    // 1. inputs, network, class and direction of every pixel in one launch
    gr_instance frame;
    memset(&frame, 0, sizeof frame);
    frame.metric = *m;
    frame.camera = *c;
    frame.n_pixels = -1;
    const gr::BatchInstance I = batch_instance(ctx, &frame);
    hipError_t e = gr::sur::frame_net(I, npix, gr_mlp_view(mlp), rule->min_impact, flag, dir,
                                      ctx->sw_logit, s);
    if (e != hipSuccess) return device_error(e, "surrogate network");
    // 2. pixels to re-trace: small logits and class edges
    e = gr::sur::fallback(ctx->sw_logit, flag, dir, c->width, c->height, logit_min, edge_px,
                          chord * chord, fallback, ctx->sw_list, ctx->sw_count, s);
    if (e != hipSuccess) return device_error(e, "surrogate fallback selection");
    // 3. re-trace the fallback pixels with the binary64 tracer and merge, with
    // the count left on the device: nothing here waits for the GPU
    gr_instance fb = frame;
    fb.pixels = ctx->sw_list;
    fb.n_pixels = npix;                       // upper bound; the kernels read the count
    fb.out.theta = ctx->sw_out[0];
    fb.out.phi = ctx->sw_out[1];
    fb.out.r = ctx->sw_out[2];
    fb.out.p_t = ctx->sw_out[3];
    fb.out.p_r = ctx->sw_out[4];
    fb.out.p_theta = ctx->sw_out[5];
    fb.out.p_phi = ctx->sw_out[6];
    fb.out.flag = ctx->sw_flag;
    fb.out.dtype = GR_F64;
    rc = reserve_table(ctx, 1);
    if (rc) return rc;
    const gr::BatchInstance B = batch_instance(ctx, &fb);
    e = hipMemcpyAsync(ctx->table, &B, sizeof B, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = gr::sur::set_firsts(ctx->sw_count, ctx->firsts, s);
    if (e != hipSuccess) return device_error(e, "fallback table");
    gr::BatchArgs A;
    memset(&A, 0, sizeof A);
    A.in = device_integrator(ctx->integ);
    A.inst = ctx->table;
    A.firsts = ctx->firsts;
    A.ninst = 1;
    A.total = npix;
    const gr_launch l = effective_launch(ctx, true);
    const gr::LaunchShape L =
        resident_shape(ctx, l, gr::occupancy_trace_fp64_batch(l.block), npix);
    e = gr::launch_trace_fp64_batch(A, L, ctx->counter, s);
    if (e != hipSuccess) return device_error(e, "fallback trace launch");
    e = gr::sur::merge(ctx->table, ctx->sw_list, ctx->sw_count, npix, flag, dir, s);
    if (e != hipSuccess) return device_error(e, "fallback merge");
    if (n_fallback) {
        unsigned long long count = 0;
        e = hipMemcpyAsync(&count, ctx->sw_count, sizeof count, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_error(e, "fallback count");
        *n_fallback = (int64_t)count;
    }
    return GR_OK;
}

int gr_trace_destroy(gr_ctx* ctx) {
    if (!ctx) return GR_OK;
    DeviceGuard guard(ctx->device);
    free_surrogate_ws(ctx);
    free_order_ws(ctx);
    free_park_ws(ctx);
    hipFree(ctx->counter);
    hipFree(ctx->table);
    hipFree(ctx->firsts);
    delete ctx;
    return GR_OK;
}

const char* gr_trace_strerror(int code) {
    switch (code) {
        case GR_OK: return "success";
        case GR_EINVAL: return "invalid argument";
        case GR_ENOMEM: return "out of device memory";
        case GR_EDEVICE: return "HIP runtime error";
        case GR_EUNSUPPORTED: return "unsupported request";
        default: return "unknown error code";
    }
}

const char* gr_trace_last_device_error(void) { return g_last_error; }

int gr_trace_validate(const gr_metric* m, const gr_camera* c, const gr_integrator* integ,
                      const gr_output* out) {
    int rc = check_metric(m);
    if (!rc) rc = check_camera(m, c);
    if (!rc) rc = check_output(out);
    if (!rc && integ) rc = check_integrator(integ);
    return rc;
}

double gr_horizon_radius(const gr_metric* m) {
    if (!m) return NAN;
    return horizon(m);
}

}  // extern "C"
