/*
 * grtrace: backward ray tracing of null geodesics around a Kerr-Newman black
 * hole on AMD Instinct MI355X (gfx950), C ABI.
 *
 * Method (arXiv 2310.15183, "Graphical Processing of Geodesic Propagation in
 * Python"): every pixel of a pinhole camera launches one ray; the ray follows
 * Hamilton's equations for H = 1/2 g^{mu nu}(r,theta) p_mu p_nu (Sec. 2.1,
 * eq. hamGeodesic, with the factor 1/2 of Appendix A) in Boyer-Lindquist
 * coordinates (Sec. 2.2.2; the charge Q enters through
 * Delta = r^2 - 2Mr + a^2 + Q^2), integrated by classical RK4 (Sec. 3.1.2)
 * whose step h = dt / |dt/dtau| is fixed from the first stage so that
 * coordinate time advances by about dt per step (appendix listing).  The
 * metric derivatives d_r g and d_theta g are forward differences of step
 * fd_eps (listing; Sec. 3.3.3 explains the choice: any metric works).  A ray
 * stops on escape (r > escape_factor * r0, Sec. 3.3.2 "Propagation"), at the
 * horizon (|dt/dtau| > horizon_norm: the coordinate-time step collapses), on
 * a non-finite state, or after max_steps updates.  The camera is the one of
 * Sec. 3.3.1 "Initial positions": directions in the camera's local frame,
 * dt/dtau from the null condition, then scaled so that dt/dtau = -1.
 *
 * Conventions shared by every call:
 *   - All pointers to per-ray data are DEVICE pointers, caller-owned, with
 *     room for one entry per traced ray (W*H for a whole frame, or n_pixels
 *     for a pixel list).  Entry k belongs to pixel k (whole frame, row-major
 *     j*W + i, row 0 at the top) or to pixels[k] (pixel list).
 *   - Calls are asynchronous on the HIP stream passed in (NULL = the null
 *     stream); outputs are valid once that stream has completed.  A context
 *     holds a small device work counter and must not be used by two calls
 *     that may run concurrently (two host threads, or two streams).
 *   - Return values: GR_OK (0) or a negative error code.  Arguments are
 *     validated on the host before anything is launched; on error nothing is
 *     launched and no output is touched.  Device errors reported by the HIP
 *     runtime come back as GR_EDEVICE (see gr_trace_last_device_error).
 *   - Flags written per ray: GR_FLAG_TIMEOUT (0, step limit), GR_FLAG_ESCAPE
 *     (1), GR_FLAG_HORIZON (2), GR_FLAG_INVALID (3, non-finite state),
 *     GR_FLAG_DISK (4, stopped in the ring of gr_integrator).  After each
 *     update the ring is tested first, then escape, then horizon.
 *   - GR_FP64 results are a deterministic function of the inputs: they do not
 *     depend on the launch configuration, the stream, or which other pixels
 *     are traced in the same call.
 */
#ifndef GRTRACE_H
#define GRTRACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GR_OK = 0,
    GR_EINVAL = -1,        /* an argument is out of range or a required pointer is NULL */
    GR_ENOMEM = -2,        /* device allocation for the context failed */
    GR_EDEVICE = -3,       /* the HIP runtime reported an error */
    GR_EUNSUPPORTED = -4   /* valid request this build does not support */
};

enum {
    GR_FLAG_TIMEOUT = 0,
    GR_FLAG_ESCAPE = 1,
    GR_FLAG_HORIZON = 2,
    GR_FLAG_INVALID = 3,
    GR_FLAG_DISK = 4
};

/* Integrator precision.
 * GR_FP64: binary64 throughout; results are reproducible bit for bit.
 * GR_MIXED (gr_trace_frame only): binary32 RK4 stages (stage points,
 *   right-hand sides, contraction, the RK4 combination; t and phi from
 *   binary64 sums of g^tt, g^tphi, g^phph); binary64 metric
 *   evaluations and forward differences (sin at theta+eps by angle
 *   addition, reciprocals by v_rcp_f64 and two Newton steps); whole binary64
 *   steps while r < 1.2 r_+ or |p_r| < 1e-3, back to binary32 stages once
 *   r > 1.25 r_+ and |p_r| > 2e-3.  The state itself stays binary64: each
 *   step's binary32 increment is added to it in binary64, because rounding
 *   theta and phi to binary32 at every step alone random-walks the end angles
 *   by ~5e-6 rad over 1e4 steps, a twentieth of the 1e-4 rad accuracy target
 *   before any other error.  Accuracy is stated against GR_FP64, not bit for
 *   bit. */
enum { GR_FP64 = 0, GR_MIXED = 1 };

/* Element type of the floating-point outputs. */
enum { GR_F64 = 0, GR_F32 = 1 };

/* Kerr-Newman black hole, geometric units G = c = 1: mass M >= 0, spin
 * length a = J/M (|a| < M for a black hole; a > 0 rotates toward +phi) and
 * charge Q.  Requires a^2 + Q^2 <= M^2, except M = Q = 0 with any a, which
 * is flat space in oblate spheroidal coordinates (no horizon).  Q = 0 is Kerr,
 * a = Q = 0 Schwarzschild. */
typedef struct {
    double M, a, Q;
} gr_metric;

/* Manko-Novikov spacetime with a mass quadrupole (arXiv 2310.15183,
 * Sec. 2.2.3): mass M > 0, spin S (angular momentum; a = S/M) with
 * 0 < |S| < M^2 (S = 0 is excluded, as in the paper: the construction divides
 * by it), and quadrupole deviation q from Kerr (mass quadrupole
 * -S^2/M - q M^3; q = 0 is Kerr, q < 0 prolate, q > 0 oblate).  The horizon
 * sits at r = M + k, k = sqrt(M^2 - (S/M)^2). */
typedef struct {
    double M, S, q;
} gr_metric_mn;

/* Static pinhole camera at Boyer-Lindquist (r0, theta0, phi0) looking toward
 * the hole.  fov is the full horizontal field of view in radians, pixels are
 * square, image right is +phi and image up is -theta.  Requires
 * r0 > r_+ = M + sqrt(M^2 - a^2 - Q^2), 0 < theta0 < pi, 0 < fov < pi,
 * width >= 1, height >= 1. */
typedef struct {
    double r0, theta0, phi0, fov;
    int32_t width, height;
} gr_camera;

/* Integration method (arXiv 2310.15183, Sec. 3.1).
 * GR_RK4: classical Runge-Kutta with the step h = dt / |dt/dtau| fixed from
 *   the first stage (Sec. 3.1.2, as in the appendix listing).
 * GR_EULER: explicit Euler, x += h f(x) with the same h (Sec. 3.1.1); first
 *   order, for the accuracy/cost comparison of Sec. "Resolution and
 *   Calculation Speed".
 * GR_RK4_TIME: classical Runge-Kutta with coordinate time as the parameter,
 *   each stage reparametrised: every stage's derivative is divided by that
 *   stage's own |dt/dtau|, the stage points are x + dt/2 k1, x + dt/2 k2,
 *   x + dt k3, so each step advances t by exactly dt (fourth order in dt).
 * GR_EULER and GR_RK4_TIME: binary64 frames only (gr_trace_frame,
 *   gr_trace_frame_mn): batches, the surrogate and GR_MIXED return
 *   GR_EUNSUPPORTED. */
enum { GR_RK4 = 0, GR_EULER = 1, GR_RK4_TIME = 2 };

/* Integrator settings.  dt > 0 is the coordinate-time step, fd_eps > 0 the
 * forward-difference step, horizon_norm > 0 the |dt/dtau| at which a ray is
 * declared captured, escape_factor > 1 the escape radius in units of r0,
 * max_steps >= 0 the step limit (0 returns the initial state), precision
 * GR_FP64 or GR_MIXED, method GR_RK4, GR_EULER or GR_RK4_TIME.
 * Suggested: 0.01, 1e-8, 1e4, 1.5, 20000, GR_FP64, GR_RK4. */
typedef struct {
    double dt, fd_eps, horizon_norm, escape_factor;
    int32_t max_steps;
    int32_t precision;
    int32_t method;
    /* Solid ring around the equator (Sec. 3.3.2: objects are volumes a ray
     * stops in; Fig. KerrDisk): a ray whose step ends with
     * disk_r_in <= r <= disk_r_out and |theta - pi/2| <= disk_half_angle
     * stops with GR_FLAG_DISK.  Off when disk_half_angle == 0; otherwise
     * 0 <= disk_r_in < disk_r_out and 0 < disk_half_angle < pi/2.  Binary64
     * frames only (batches, the surrogate and GR_MIXED: GR_EUNSUPPORTED). */
    double disk_r_in, disk_r_out, disk_half_angle;
} gr_integrator;

/* Per-ray outputs (device pointers).  The eight floating-point arrays hold
 * the state after the last update, elements of type dtype (GR_F64 or
 * GR_F32, rounded to nearest); any of them may be NULL (not written).  p_t
 * and p_phi are constant along a ray (t and phi derivatives of the metric
 * vanish).  flag (int8) is required; steps (int32, number of updates taken)
 * may be NULL. */
typedef struct {
    void *t, *r, *theta, *phi;
    void *p_t, *p_r, *p_theta, *p_phi;
    int8_t *flag;
    int32_t *steps;
    int32_t dtype;
} gr_output;

/* One image of a batch: its black hole, camera and outputs.  n_pixels = -1
 * traces all width*height pixels (pixels is ignored); n_pixels >= 0 traces
 * the n_pixels entries of the device list pixels (indices j*width + i, any
 * order, repeats allowed, each in [0, width*height)).  An instance with no
 * rays (n_pixels = 0) may leave pixels and every output pointer NULL. */
typedef struct {
    gr_metric metric;
    gr_camera camera;
    gr_output out;
    const int32_t *pixels;
    int64_t n_pixels;
} gr_instance;

typedef struct gr_ctx gr_ctx;

/* Launch shape of the tracing kernels (results never depend on it).
 * block: threads per workgroup (64, 128 or 256); waves_per_simd: target
 * residency used to size the persistent grid (1..8, 0 = as many as fit);
 * refill: 1 = lanes that finish take the next ray from the work queue,
 * 0 = each lane traces one ray and the grid covers every ray (one 8x8 pixel
 * tile of a frame, or 64 entries of a pixel list, per wave); order: 0 = rays
 * are queued in the order given;
 * 1 = batches queue the instances with the longest expected rays (largest
 * escape radius) first, which shortens the tail; 2 = as 1, and frames of at
 * least 4096 pixels traced with refill queue their pixels sorted by how close
 * the camera ray's impact parameter sqrt(Carter Q + L_z^2)/E is to the
 * critical one (16 bytes per pixel of context workspace).  Without refill a
 * frame is traced one ray per lane over 8x8 pixel tiles, one tile per wave.
 * Until a shape is set, frames use {64, 0, 0, 0} (neighbouring pixels take
 * nearly the same number of steps, so waves stay full without refill) and
 * batches {256, 0, 1, 1}, the fastest measured for each. */
typedef struct {
    int32_t block;
    int32_t waves_per_simd;
    int32_t refill;
    int32_t order;
} gr_launch;

/* Create a context on HIP device `device` with the given integrator.
 * Allocates a few bytes of device memory (work counter).  *ctx is set to
 * NULL on error.  Errors: GR_EINVAL (ctx NULL, integrator out of range),
 * GR_ENOMEM, GR_EDEVICE. */
int gr_trace_init(gr_ctx **ctx, int device, const gr_integrator *integ);

/* Trace every pixel of one frame with the context's integrator (GR_FP64 or
 * GR_MIXED).  Errors: GR_EINVAL (validation above, NULL ctx/m/c/out or
 * out->flag), GR_EDEVICE (launch failed). */
int gr_trace_frame(gr_ctx *ctx, const gr_metric *m, const gr_camera *c,
                   const gr_output *out, void *hip_stream);

/* gr_trace_frame for a Manko-Novikov spacetime (Sec. 2.2.3; the inverse
 * components of the appendix listing's metricAtPoint): the same camera
 * (orthonormal scale factors from the metric at the camera), integrator and
 * exits, the metric evaluated in full at the three points of every stage
 * (its exponentials from their series definition, so results are
 * reproducible bit for bit).  One ray per lane over 8x8 pixel tiles whatever
 * the context's launch shape.  With a step limit of 4096 or more, rays still
 * running after a quarter of it are parked in context workspace (60 bytes per
 * pixel, at most 2^22 pixels, grown with hipMalloc on first need) and a
 * second launch on the same stream continues them all together; the results
 * are those of one uninterrupted integration.  If the workspace cannot be
 * allocated, one launch does everything.  The camera needs r0 > M + k.
 * Errors: GR_EINVAL (validation, NULL arguments, a frame of more than
 * 2^31 - 1 tiles), GR_EUNSUPPORTED (a GR_MIXED context), GR_EDEVICE. */
int gr_trace_frame_mn(gr_ctx *ctx, const gr_metric_mn *m, const gr_camera *c,
                      const gr_output *out, void *hip_stream);

/* Redshift z = lambda_O / lambda_S of the light of the ring (Sec. 3.3.3) for
 * n traced rays: the ring's matter moves on circular orbits (p_r = p_theta =
 * 0, dp/dtau = 0; with s_t = -1, s_phi solves s_phi^2 d_r g^{phph}
 * - 2 s_phi d_r g^{tph} + d_r g^{tt} = 0, d_r by the context's forward
 * difference; the root turning faster toward +phi; normalised to
 * g^{mu nu} s s = -1), and the camera's locally non-rotating observer
 * receives the ray: z = (p_t S^t + p_phi S^phi) / sqrt(-1/g^{tt}(camera))
 * with S^mu = g^{mu nu} s_nu at the ray's end.  Rays without GR_FLAG_DISK,
 * and rings inside the photon orbit (no timelike circular orbit), get NaN.
 * Reads r, theta, p_t, p_phi and flag of `out` (traced with camera c; the
 * dtype of out), writes z[n] (device, the same dtype).  Errors: GR_EINVAL
 * (NULL arguments, a needed array missing, n < 0, invalid metric/camera),
 * GR_EDEVICE. */
int gr_redshift(gr_ctx *ctx, const gr_metric *m, const gr_camera *c, const gr_output *out,
                int64_t n, void *z, void *hip_stream);

/* gr_redshift for a Manko-Novikov spacetime. */
int gr_redshift_mn(gr_ctx *ctx, const gr_metric_mn *m, const gr_camera *c,
                   const gr_output *out, int64_t n, void *z, void *hip_stream);

/* Shading of traced rays into 32-bit colours (bytes R, G, B, A in memory),
 * the figures of arXiv 2310.15183, Sec. 4.
 * GR_SHADE_BANDS (the exit-position figures, "perspective" and "flat
 *   space"): an escaped ray shows a dark-blue sky with three lines on it,
 *   each a narrow interval of one Boyer-Lindquist angle of its end position,
 *   drawn where the squared sine of the offset from the line is < 0.01, in
 *   this precedence: red, the meridian through the camera (phi = 0, pi: a
 *   vertical line through the hole); green, the meridian across the view
 *   (phi = +-pi/2: a circle around the hole); light blue, the equator (the
 *   interval in 2 theta also covers the poles).  Other rays black.  Reads
 *   theta, phi, flag.
 * GR_SHADE_TIME (the exit-time figures): tau = |t| at the end; escaped rays
 *   with tau < t_max shade from dark blue to cyan with
 *   level = floor(255 tau / t_max), dimmed to 7/8 on every other band of
 *   width `band` when band > 0; rays that did not escape, and tau >= t_max,
 *   are cyan; invalid rays black.  Reads t, flag.
 * GR_SHADE_TEXTURE (the textured figures, bilinear texture filtering): an
 *   escaped ray shows an equirectangular sky texture (tex_width x
 *   tex_height device words, row-major, row 0 at theta = 0, column 0 at
 *   phi = 0) at its end direction, filtered bilinearly: theta brought into
 *   [0, pi] (mod 2 pi; above pi reflected with phi turned by pi), texel
 *   (i, j) centred at phi = 2 pi (i + 1/2)/tex_width, theta = pi (j + 1/2)
 *   /tex_height, columns wrapping around in phi, rows clamped at the poles;
 *   each byte is the bilinear interpolation of the four nearest texels'
 *   bytes, rounded half up.  Other rays black.  Reads theta, phi, flag.
 * Decisions are taken in binary64 with the tracer's sin/cos. */
enum { GR_SHADE_BANDS = 0, GR_SHADE_TIME = 1, GR_SHADE_TEXTURE = 2 };

typedef struct {
    int32_t mode;
    double t_max;               /* GR_SHADE_TIME: > 0 */
    double band;                /* GR_SHADE_TIME: >= 0, 0 = no banding */
    const uint32_t *texture;    /* GR_SHADE_TEXTURE: device texels, caller-owned */
    int32_t tex_width, tex_height;  /* GR_SHADE_TEXTURE: >= 1 */
} gr_shade;

/* Colour n rays held in `out` (device arrays of a traced frame or batch
 * instance, binary64 or binary32) into rgba[n] (device), asynchronously on
 * the stream.  Errors: GR_EINVAL (NULL arguments, n < 0, a needed output
 * array missing, t_max <= 0 or band < 0 for GR_SHADE_TIME, no texture or a
 * texture side < 1 for GR_SHADE_TEXTURE), GR_EDEVICE. */
int gr_shade_frame(const gr_shade *shade, const gr_output *out, int64_t n, uint32_t *rgba,
                   void *hip_stream);

/* Trace n >= 1 instances (possibly different black holes, cameras and image
 * sizes) in one persistent launch fed by one work queue (GR_FP64 only:
 * GR_EUNSUPPORTED for GR_MIXED).  The instance table
 * (416 bytes per instance) is copied to device memory owned by the
 * context, which grows it with hipMalloc when a larger batch arrives.  Same
 * errors as gr_trace_frame (GR_ENOMEM if the table cannot grow); an error in
 * any instance rejects the whole call. */
int gr_trace_batch(gr_ctx *ctx, const gr_instance *inst, int32_t n, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * trace as gr_trace_batch, with the same arguments, validation and results
 * bit for bit, but the instance table, prefix offsets and work counter live
 * in one fixed array per device (GR_NOALLOC_MAX_INSTANCES instances, about
 * 200 KB) that the library holds until the process ends, instead of context
 * memory grown with hipMalloc.  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call); copies the table from host memory with
 * hipMemcpyAsync and clears the counter with a kernel, on the stream.  Every
 * call on one device shares that device's array and overwrites it: two calls
 * that may overlap on one device (two streams, two host threads, two
 * contexts) race and must be serialised by the caller.  Errors: those of
 * gr_trace_batch, except that the table never grows: more than
 * GR_NOALLOC_MAX_INSTANCES instances with rays give GR_EINVAL (the text of
 * gr_trace_last_device_error names the limit) and launch nothing. */
#define GR_NOALLOC_MAX_INSTANCES 512
int gr_trace_batch_noalloc(gr_ctx *ctx, const gr_instance *inst, int32_t n, void *hip_stream);

/* Replace the integrator settings of a context (same validation as init). */
int gr_trace_set_integrator(gr_ctx *ctx, const gr_integrator *integ);

/* Override (or with launch == NULL restore) the launch shape. */
int gr_trace_set_launch(gr_ctx *ctx, const gr_launch *launch);

/* Launch shape the next frame call will use (batches: see gr_launch). */
int gr_trace_get_launch(const gr_ctx *ctx, gr_launch *launch);

/* Pick the launch shape for a batch by measurement, store it in the context
 * and trace the batch with it.  Candidate shapes (persistent: block
 * 64/128/256 and residency 2 or as many as fit; one ray per lane: block
 * 64/128/256; both queue orders) are timed on the batch with the
 * step limit lowered to trial_steps (0 = no lowering); every candidate gives
 * identical results, so the outputs hold the final full run, made with the
 * winner.  If cache_path is non-NULL, a winner recorded there for the same
 * device architecture and batch size class is reused without trials, and a
 * new winner is appended.  *best (may be NULL) receives the shape.  Blocks
 * the calling thread until the stream has finished the trials.  Errors: those
 * of gr_trace_batch, GR_EINVAL for trial_steps < 0. */
int gr_trace_autotune(gr_ctx *ctx, const gr_instance *inst, int32_t n, int32_t trial_steps,
                      const char *cache_path, gr_launch *best, void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Learned surrogate (a network trained on rays the tracer itself produced).
 *
 * Network: 7 inputs -> 4 hidden layers of 256 with SiLU -> 4 outputs, with
 * bfloat16 weights and activations on the matrix cores and binary32
 * accumulation.  Inputs of a ray: pixel angles atan(x), atan(y) of its
 * image-plane coordinates, a/M, |Q|/M, theta0, r0/(50 M), fov (M taken as 1
 * for flat space).  Outputs: an escape logit and a correction d of the end
 * sky direction: the ray is predicted to escape when the logit is positive,
 * towards normalise(u_flat + d), where u_flat is the baseline direction of
 * gr_surrogate_inputs: where the camera ray would leave the escape sphere
 * r = escape_factor * r0 around the Reissner-Nordstrom hole with the same M
 * and Q (the straight line of flat space if that hole captures the ray).  Parameters are one packed binary32 vector: for each
 * layer, W (in x out, row-major) then b (out).  Loss of a batch of n rays with
 * targets (escaped, d): mean of softplus(y0) - escaped*y0 +
 * lam*escaped*sum_c huber(y[c] - d[c]), huber(e) = e^2 for |e| <= delta and
 * 2 delta |e| - delta^2 beyond.  All array arguments are device pointers
 * unless named host_*; calls are asynchronous on the stream unless stated. */
typedef struct gr_mlp gr_mlp;

/* Number of binary32 values in the packed parameter vector (200,452). */
int64_t gr_mlp_num_params(void);

/* Create a network on `device` with workspace for max_batch rows per pass
 * (32 <= max_batch <= 2^28; about 7.4 KB per row).  Parameters start unset:
 * call gr_mlp_init or gr_mlp_set_params.  Errors: GR_EINVAL, GR_ENOMEM. */
int gr_mlp_create(gr_mlp **mlp, int device, int64_t max_batch);
int gr_mlp_destroy(gr_mlp *mlp);

/* He-uniform weights (bound sqrt(6/fan_in), SplitMix64 stream from seed),
 * zero biases; resets the optimiser.  Synchronous. */
int gr_mlp_init(gr_mlp *mlp, uint64_t seed);

/* Copy the packed parameters from / to host memory (gr_mlp_num_params
 * floats); set resets the optimiser.  Synchronous. */
int gr_mlp_set_params(gr_mlp *mlp, const float *host_params);
int gr_mlp_get_params(const gr_mlp *mlp, float *host_params);

/* y (n x 4) = network(x (n x 7)), in chunks of max_batch rows. */
int gr_mlp_forward(gr_mlp *mlp, const float *x, int64_t n, float *y, void *hip_stream);

/* Loss (written to *loss, a device float; may be NULL) and its gradient
 * (grad, gr_mlp_num_params floats, overwritten) over n rows, n a multiple of
 * 32 and <= max_batch.  rows (may be NULL) gathers row rows[i] of x (n_src x
 * 7) and target (n_src x 4); rows outside [0, n_src) read as zeros.  lam >= 0
 * weights the direction term, delta > 0 is its Huber threshold (a huge
 * delta gives the squared error), and rows whose target correction is longer
 * than dmax >= 0 take no direction loss (a huge dmax keeps every row). */
int gr_mlp_loss_grad(gr_mlp *mlp, const float *x, const float *target, const int32_t *rows,
                     int64_t n, int64_t n_src, float lam, float delta, float dmax, float *loss,
                     float *grad, void *hip_stream);

/* One Adam step (Kingma and Ba, bias-corrected) on the binary32 master
 * parameters with the given gradient; refreshes the bfloat16 copies. */
int gr_mlp_adam_step(gr_mlp *mlp, const float *grad, float lr, float beta1, float beta2,
                     float eps, void *hip_stream);

/* Adam steps taken since the last init/set. */
int64_t gr_mlp_steps(const gr_mlp *mlp);

/* Network inputs x (total x 7) and baseline directions u_flat (total x 3) of
 * the rays of a batch, enumerated like gr_trace_batch with instances in the
 * order given (frame order or pixel-list order).  The baseline is where the
 * camera ray would cross the escape sphere around the Reissner-Nordstrom hole
 * with the same M and Q (its sweep is a 1-D integral), or where the
 * straight line of flat space crosses it if that hole captures the ray.
 * Outputs of the instances are not used. */
int gr_surrogate_inputs(gr_ctx *ctx, const gr_instance *inst, int32_t n, float *x,
                        float *u_flat, void *hip_stream);

/* Training targets (total x 4: escaped 0/1, d = u - u_flat) from the traced
 * outputs of the same instances (theta, phi, r and all four momenta required,
 * binary64 or binary32); u is where the traced ray crossed the escape sphere,
 * its end state moved back along its own velocity. */
int gr_surrogate_targets(gr_ctx *ctx, const gr_instance *inst, int32_t n, const float *u_flat,
                         float *target, void *hip_stream);

/* Which pixels of a surrogate frame are re-traced with RK4 (any rule that
 * holds): |logit| < logit_min; a pixel within Chebyshev distance edge_px
 * (0..16) has the other class; (max_gain > 0) the predicted end directions of
 * the pixel and an 8-neighbour, both escaping, differ by more than max_gain
 * pixel widths (fov / width radians each), a local magnification above
 * max_gain; (min_impact > 0) the pixel is predicted to escape and its camera
 * ray's impact parameter is below min_impact times the critical one of the
 * Reissner-Nordstrom hole with the same M and Q, where the network's
 * baseline does not hold (see gr_surrogate_inputs). */
typedef struct {
    float logit_min;
    int32_t edge_px;
    float max_gain;
    float min_impact;
} gr_fallback;

/* Surrogate frame with RK4 fallback.  Every pixel gets the network's class
 * (flag: GR_FLAG_ESCAPE or GR_FLAG_HORIZON) and end direction (dir, 3 floats,
 * zero unless escaped), computed for the whole frame in one fused launch
 * (inputs, the five layers, classification) with the same bfloat16 products
 * and binary32 sums as gr_mlp_forward.  Pixels selected by rule (fallback[p]
 * = 1) are re-traced by the context's binary64 tracer and their traced flag
 * and escape-sphere direction replace the network's.  The whole frame is
 * queued on hip_stream without waiting for the GPU (the fallback count stays
 * on the device and sizes the retrace there) unless n_fallback (host) is
 * non-NULL: then the call waits for the stream and stores the count.
 * Workspace (about 65 B per pixel) is kept in the context, so frames in
 * flight at the same time need one context each; calls on one context must
 * be ordered (same stream, or synchronised).  Errors: GR_EINVAL (also for
 * networks on another device), GR_EUNSUPPORTED (context not GR_FP64),
 * GR_ENOMEM. */
int gr_surrogate_frame(gr_ctx *ctx, gr_mlp *mlp, const gr_metric *m, const gr_camera *c,
                       const gr_fallback *rule, int8_t *flag, float *dir, int8_t *fallback,
                       int64_t *n_fallback, void *hip_stream);

/* Free the context (waits for nothing: the caller synchronises its streams
 * first).  NULL is accepted. */
int gr_trace_destroy(gr_ctx *ctx);

/* Static description of an error code. */
const char *gr_trace_strerror(int code);

/* Text of the last HIP error seen by this library in the calling thread
 * ("" if none). */
const char *gr_trace_last_device_error(void);

/* Check of the binary64 step's divisions (not part of tracing): for k < n,
 * q[k] = a[k] / x[k] and r[k] = 1 / x[k] formed as the Kerr-Newman step forms
 * them (hardware reciprocal estimate, Newton-Raphson refinements, Markstein's
 * correction), so that tests can compare them with IEEE division.  Correctly
 * rounded for finite, normal operands with a normal quotient; other operands
 * give unspecified values.  Device arrays of n doubles, asynchronous on the
 * stream.  Errors: GR_EINVAL (n < 0, or a NULL array with n > 0), GR_EDEVICE
 * (launch failed). */
int gr_check_division(const double *a, const double *x, double *q, double *r, int64_t n,
                      void *hip_stream);

/* Run the host-side validation of gr_trace_frame on its arguments without a
 * device or context (integ may be NULL to skip it).  Returns GR_OK or
 * GR_EINVAL. */
int gr_trace_validate(const gr_metric *m, const gr_camera *c, const gr_integrator *integ,
                      const gr_output *out);

/* Outer event horizon r_+ = M + sqrt(M^2 - a^2 - Q^2) (host helper; 0 for
 * flat space). */
double gr_horizon_radius(const gr_metric *m);

#ifdef __cplusplus
}
#endif

#endif /* GRTRACE_H */
