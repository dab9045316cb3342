// C-ABI entry points of libgrtrace: argument validation, context, launch
// shape and dispatch to the kernels.  Host code only.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "grtrace.h"
#include "internal.h"

struct gr_ctx {
    int device;
    gr_integrator integ;
    gr_launch launch;          // user override (block == 0: none)
    unsigned long long* counter;
    int num_cu;
};

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
    return GR_OK;
}

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

// Resident-grid launch shape for `nray` rays.
gr::LaunchShape shape_for(const gr_ctx* ctx, int64_t nray, bool f32_out) {
    gr::LaunchShape L;
    gr_launch l = ctx->launch;
    if (l.block == 0) {
        l.block = 256;
        l.waves_per_simd = 0;
        l.refill = 1;
    }
    L.block = l.block;
    L.refill = l.refill;
    const int64_t blocks_needed = (nray + L.block - 1) / L.block;
    if (!L.refill) {
        L.grid = (int)std::max<int64_t>(1, blocks_needed);
        return L;
    }
    int per_cu = gr::occupancy_trace_fp64(L.block, f32_out);
    if (per_cu < 1) per_cu = 1;
    if (l.waves_per_simd > 0) {
        const int waves_per_block = L.block / 64;
        const int want = std::max(1, (l.waves_per_simd * 4) / waves_per_block);
        per_cu = std::min(per_cu, want);
    }
    const int64_t resident = (int64_t)per_cu * ctx->num_cu;
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>(resident, blocks_needed));
    return L;
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

gr::FrameArgs frame_args(const gr_ctx* ctx, const gr_metric* m, const gr_camera* c,
                         const gr_output* o, const int32_t* pixels, int64_t nray) {
    gr::FrameArgs A;
    memset(&A, 0, sizeof A);
    A.hole = gr::make_hole(m->M, m->a, m->Q);
    A.cam = gr::make_camera(A.hole, c->r0, c->theta0, c->phi0, c->fov, c->width, c->height);
    A.in.dt = ctx->integ.dt;
    A.in.eps = ctx->integ.fd_eps;
    A.in.inv_eps = 1.0 / ctx->integ.fd_eps;
    A.in.hnorm = ctx->integ.horizon_norm;
    A.in.esc_factor = ctx->integ.escape_factor;
    A.in.max_steps = ctx->integ.max_steps;
    A.r_esc = ctx->integ.escape_factor * c->r0;
    A.nray = nray;
    A.pixels = pixels;
    A.out.t = o->t;
    A.out.r = o->r;
    A.out.th = o->theta;
    A.out.ph = o->phi;
    A.out.pt = o->p_t;
    A.out.pr = o->p_r;
    A.out.pth = o->p_theta;
    A.out.pph = o->p_phi;
    A.out.flag = o->flag;
    A.out.steps = o->steps;
    return A;
}

int launch_frame(gr_ctx* ctx, const gr_metric* m, const gr_camera* c, const gr_output* o,
                 const int32_t* pixels, int64_t nray, hipStream_t s) {
    if (nray == 0) return GR_OK;
    const bool f32 = o->dtype == GR_F32;
    const gr::FrameArgs A = frame_args(ctx, m, c, o, pixels, nray);
    const gr::LaunchShape L = shape_for(ctx, nray, f32);
    hipError_t e = gr::launch_trace_fp64(A, f32, L, ctx->counter, s);
    if (e != hipSuccess) return device_error(e, "trace_fp64 launch");
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
    e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) {
        delete c;
        return device_error(e, "hipDeviceGetAttribute");
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
    ctx->launch = *l;
    return GR_OK;
}

int gr_trace_get_launch(const gr_ctx* ctx, gr_launch* l) {
    if (!ctx || !l) return GR_EINVAL;
    if (ctx->launch.block) {
        *l = ctx->launch;
    } else {
        l->block = 256;
        l->waves_per_simd = 0;
        l->refill = 1;
    }
    return GR_OK;
}

int gr_trace_frame(gr_ctx* ctx, const gr_metric* m, const gr_camera* c, const gr_output* out,
                   void* hip_stream) {
    if (!ctx) return GR_EINVAL;
    int rc = check_metric(m);
    if (!rc) rc = check_camera(m, c);
    if (!rc) rc = check_output(out);
    if (rc) return rc;
    if (ctx->integ.precision != GR_FP64) return GR_EUNSUPPORTED;
    DeviceGuard guard(ctx->device);
    return launch_frame(ctx, m, c, out, nullptr, (int64_t)c->width * c->height,
                        (hipStream_t)hip_stream);
}

static int64_t instance_rays(const gr_instance* I) {
    return I->n_pixels < 0 ? (int64_t)I->camera.width * I->camera.height : I->n_pixels;
}

int gr_trace_batch(gr_ctx* ctx, const gr_instance* inst, int32_t n, void* hip_stream) {
    if (!ctx || !inst || n < 1) return GR_EINVAL;
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
    DeviceGuard guard(ctx->device);
    for (int32_t k = 0; k < n; ++k) {
        const gr_instance* I = &inst[k];
        const int64_t nray = instance_rays(I);
        if (nray == 0) continue;
        const int32_t* pix = I->n_pixels < 0 ? nullptr : I->pixels;
        const int rc = launch_frame(ctx, &I->metric, &I->camera, &I->out, pix, nray,
                                    (hipStream_t)hip_stream);
        if (rc) return rc;
    }
    return GR_OK;
}

int gr_trace_destroy(gr_ctx* ctx) {
    if (!ctx) return GR_OK;
    DeviceGuard guard(ctx->device);
    hipFree(ctx->counter);
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
