/*
 * misr.h -- C ABI of libmisr.so: the SCG cost/gradient hot path of multi-image
 * super-resolution (FL-MISR, arXiv 2108.04315) on one AMD MI355X (gfx950).
 *
 * Problem statement (Sec. 3.1): K low-resolution frames y_k, each the image of
 * the unknown high-resolution image x under a known system matrix
 * A_k = D B M_k (Eq. sisr: M_k motion, B blur, D decimation), plus noise.
 * x minimises (Eq. objective, split as in Eq. reformulated)
 *
 *     J(x) = sum_k || A_k x - y_k ||_p^p  +  lambda * sum_d gamma(d) || x - S_d x ||_1
 *
 * with the bilateral total variation prior of Eq. prior, gamma(d) = alpha^(dx+dy),
 * d in [0, w-1]^2 minus the origin.  The minimiser is found with the scaled
 * conjugate gradient method the paper uses (Sec. 3.1, Algorithm 1; Moller 1993)
 * for a fixed number of passes (Algorithm 1's loop bound).
 *
 * Readings fixed by this library where the paper is silent:
 *   - M_k is a bilinear translation by (dx_k, dy_k) LR pixels = s*(dx_k, dy_k)
 *     HR pixels, zero outside the image: (M_k x)(u,v) = x~(u + s dy_k, v + s dx_k);
 *   - B is a "same" 2-D convolution with zero padding by the P x P PSF
 *     psf_1d (outer) psf_1d;
 *   - D is s x s block averaging; A_k is applied M first, then B, then D;
 *   - the L1 norms are smoothed: phi(z) = sqrt(z^2 + eps^2) - eps
 *     (eps = 0 gives |z| with sign(0) = 0);
 *   - BTV pairs (i, i + d) count only when both pixels are inside the image.
 *
 * Layouts.  Images are dense row-major, row stride = width.  x is H x W.
 * y is K contiguous frames of (H/s) x (W/s).  The gradient and all scratch
 * vectors are float32.  x and y are stored as misr_dtype (f32, f16 or bf16);
 * arithmetic is float32, and inner products and SCG scalars are float64.
 *
 * Ownership.  The caller owns every data buffer (device memory unless stated);
 * the library never frees them and keeps no pointer past the call, except for
 * server requests, whose buffers must stay valid until the request is DONE,
 * FAILED or CANCELLED.  The library owns ctx, op and server handles and frees
 * them in the matching *_destroy call.  Workspace is library-owned and cached
 * per op.
 *
 * Errors.  Every entry point returns misr_status; no C++ exception crosses the
 * ABI.  Arguments are validated on the host before any launch (MISR_E_INVAL,
 * with a message in misr_last_error()).  Work is enqueued asynchronously on the
 * given HIP stream (a hipStream_t passed as void*, NULL = default stream) unless
 * a function says it synchronises.  Calls that share an op must not overlap in
 * time on different streams (the op's workspace is shared).
 */
#ifndef MISR_H
#define MISR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MISR_OK = 0,
    MISR_E_INVAL = 1,     /* bad argument; nothing was launched */
    MISR_E_NOMEM = 2,     /* device allocation failed or HBM budget exceeded */
    MISR_E_HIP = 3,       /* a HIP runtime call failed */
    MISR_E_NUMERIC = 4,   /* non-finite cost or curvature: solve stopped early */
    MISR_E_BUSY = 5,      /* server queue full */
    MISR_E_NOTFOUND = 6,  /* unknown request id */
    MISR_E_CANCELLED = 7, /* request was cancelled */
    MISR_E_TIMEOUT = 8    /* wait timed out */
} misr_status;

typedef enum { MISR_F32 = 0, MISR_F16 = 1, MISR_BF16 = 2 } misr_dtype;

typedef struct misr_ctx misr_ctx;
typedef struct misr_op misr_op;
typedef struct misr_server misr_server;

/* Acquisition geometry (Sec. 3.1 Eq. sisr; Sec. 3.2: frames shifted by a
 * fraction of a detector pixel).  All pointers are host memory, read during
 * misr_op_create only. */
typedef struct {
    int32_t hr_h, hr_w;       /* HR image size; both divisible by scale */
    int32_t scale;            /* s >= 1: LR frame is (hr_h/s) x (hr_w/s) */
    int32_t n_frames;         /* K >= 1 */
    const double *shifts_lr;  /* [K][2] = (dx, dy) in LR pixels, |dx|,|dy| <= 1;
                                 may be NULL when warps is given */
    int32_t psf_size;         /* P, odd, 1 <= P <= 15 */
    const double *psf_1d;     /* [P] taps; the 2-D PSF is their outer product */
    const double *psf_frames; /* NULL, or [K][2][P]: frame k's own blur B_k (A_k =
                                 D B_k M_k), vertical taps then horizontal taps,
                                 B_k their outer product; overrides psf_1d */
    /* General operators (A_k = D B_k M_k with a general M_k or B_k).  When
     * either field below is set the operator runs on the general kernels:
     * FP32 images (img_dtype MISR_F32, y_u16 = 0), untiled (tile_lr = 0),
     * x_init 0 or 1 (solves, batches and served requests alike);
     * misr_interpolate is rejected.  A_k is evaluated from its factors
     * (matrix-free: the warp's six coefficients and a Q x Q blur-and-bin
     * kernel per frame, Q = s + P - 1) when every frame's warp is invertible
     * and the windows its adjoint gathers from fit the kernels' local memory
     * (warps that shrink the image by less than about 3x); otherwise, or with
     * general_ell = 1, A and its transpose are stored as sparse matrices
     * (ELL, about 2 x 8 B x (P + s + 2)^2 per LR pixel and frame of device
     * memory, built on the host at misr_op_create). */
    const double *warps;      /* NULL, or [K][6]: frame k's warp M_k samples x
                                 bilinearly at row w0 u + w1 v + w2, column
                                 w3 u + w4 v + w5 for HR pixel (u, v) (zero off
                                 the grid); overrides shifts_lr.  The shift
                                 (dx, dy) is (1, 0, s dy, 0, 1, s dx) */
    const double *psf_2d;     /* NULL, or [K][P][P]: frame k's non-separable PSF,
                                 h[a + R][b + R] weighting the sample at offset
                                 (-a, -b), R = (P - 1) / 2 (zero padding);
                                 overrides psf_1d and psf_frames */
    int32_t general_ell;      /* 1: a general operator is stored as sparse
                                 matrices even where the matrix-free kernels
                                 apply (0: matrix-free where they apply) */
} misr_geometry;

/* Objective and solver settings (Eq. objective, Eq. prior, Algorithm 1). */
typedef struct {
    double lambda_reg;   /* lambda >= 0 (default 0.01) */
    double alpha_btv;    /* alpha in (0, 1) (default 0.4) */
    double eps;          /* Charbonnier eps of the prior >= 0 (default 1e-3) */
    int32_t btv_w;       /* window w in [1, 3] (default 3) */
    int32_t data_p;      /* data norm p in {1, 2} (default 2); p = 1 is the
                            Charbonnier-smoothed L1 norm with eps_data */
    double eps_data;     /* Charbonnier eps of the L1 data term (p = 1) >= 0 */
    double scg_sigma;    /* SCG sigma > 0 (default 1e-4) */
    double scg_lambda1;  /* SCG initial scale lambda_1 > 0 (default 1e-6) */
    int32_t n_iter;      /* SCG passes >= 0, failed passes included */
    misr_dtype img_dtype;/* storage of x and y */
    int32_t tile_lr;     /* 0: solve the image whole; else split into tiles of
                            tile_lr x tile_lr LR pixels held separately in HBM
                            with a halo exchanged every pass */
    int32_t halo_lr;     /* halo width in LR pixels for tile_lr > 0 */
    int32_t x_rounding;  /* x_work = 1 with a 16-bit img_dtype: rounding of each
                            x update, 0 to nearest even (default), 1 stochastic,
                            driven by a counter-based hash of (pixel, pass) so
                            that it is reproducible */
    int32_t x_work;      /* SCG iterate with a 16-bit img_dtype: 0 (default) FP32
                            in library buffers (x is widened on entry and rounded
                            to nearest even on exit; y stays 16-bit); 1 held in
                            img_dtype itself (half the x traffic, but steps below
                            half a unit in the last place are lost, so the solve
                            stalls once steps get small) */
    int32_t x_init;      /* start point of misr_scg_solve and served requests:
                            0 the caller's x (default); 1 bicubic upsampling of
                            frame 0 (misr_upsample); 2 multi-image interpolation
                            (misr_interpolate); computed on the device into x,
                            so served requests may pass x0 = NULL */
    int32_t y_u16;       /* 0: y stored in img_dtype (default); 1: y holds the
                            detector's uint16 counts and frame values are
                            y_scale * count (the paper's 16-bit input images,
                            Sec. 4); cost/gradient, solves and served requests */
    double y_scale;      /* > 0 with y_u16 = 1 */
} misr_params;

/* One SCG pass as recorded on the device. */
typedef struct {
    double E;        /* cost after the pass */
    double E_t;      /* cost at the trial point x + alpha p */
    double delta;    /* scaled curvature used for alpha */
    double mu;       /* p . r */
    double alpha;    /* step size mu / delta */
    double Delta;    /* comparison parameter */
    double lam;      /* scale parameter after the pass */
    double pi;       /* |p|^2 of the pass's direction */
    double rr;       /* |r|^2 at the start of the pass (r = -grad J(x)) */
    int32_t success; /* 1 if the step was accepted */
    int32_t pad_;
} misr_scg_iter;

typedef struct {
    misr_scg_iter *iters; /* host array with room for `capacity` passes, or NULL */
    int32_t capacity;
    int32_t n_passes;     /* out: passes run (< n_iter only on early stop) */
    int32_t n_success;    /* out: accepted passes */
    int32_t stop;         /* out: 0 ran all passes, 1 ||r|| = 0, 2 non-finite */
    double E0;            /* out: cost at x0 */
    double E_final;       /* out: cost at the returned x */
} misr_scg_trace;

/* ------------------------------------------------------------------ setup */
/* Fills p with the defaults listed above (n_iter = 50, f32, untiled). */
void misr_params_default(misr_params *p);

/* Host-only validation (no device is touched). */
misr_status misr_geometry_check(const misr_geometry *g);
misr_status misr_params_check(const misr_params *p);

/* Thread-local description of the last error on this thread; valid until the
 * next misr_* call on the same thread. */
const char *misr_last_error(void);

/* Binds a context to HIP device `hip_device` (ordinal).  A context must outlive
 * the ops and servers created on it: misr_ctx_destroy returns MISR_E_BUSY (and
 * frees nothing) while any of them is alive. */
misr_status misr_ctx_create(int hip_device, misr_ctx **out);
misr_status misr_ctx_destroy(misr_ctx *ctx);

/* Precomputes the operator: per frame, the 1-D band weights of A_k's row and
 * column factors (A_k = C_y,k (x) C_x,k is exact because M, B and D are all
 * separable, zero padding included).  Built once and reused by every call on
 * this geometry, as the paper builds A_i once per acquisition (Sec. 3.2). */
misr_status misr_op_create(misr_ctx *ctx, const misr_geometry *g, misr_op **out);
/* Waits for the device to go idle, then frees the operator (always).  Returns
 * MISR_E_HIP if that wait reports a device error (raised by any earlier work
 * on the device), so that an asynchronous fault surfaces at the caller that
 * released the operator. */
misr_status misr_op_destroy(misr_op *op);
/* Band length L of the per-frame 1-D factors (taps per LR pixel per axis);
 * 0 for a general operator. */
int misr_op_band(const misr_op *op);
/* Entries per row of a general operator's sparse matrices: *a_w for A (per LR
 * pixel and frame), *t_w for A^T (per HR pixel); both 0 for a banded or a
 * matrix-free general operator (no stored matrices).  MISR_E_INVAL on NULL
 * arguments. */
misr_status misr_op_sparse_width(const misr_op *op, int32_t *a_w, int32_t *t_w);

/* Tile autotuner: times the trial and update passes (alternating, as in a
 * solve) of every compiled tile
 * variant of this banded operator (0: the widest tile that fits both passes;
 * 1: one about half as wide, which gives small images more workgroups; 2,
 * where it exists: variant 0 with a wider trial-pass tile, the widest the
 * trial pass's LDS alone allows) on the caller's
 * frames y and image x (device buffers, img_dtype storage; x is read only),
 * `reps` launches each with HIP events, and keeps the fastest for every
 * later call on this operator (solves, batches, operators).  *tile_h x
 * *tile_w: the chosen tile in HR pixels.  A general operator has no tiles
 * (both 0).  Synchronises with `stream`.  On an error the operator keeps the
 * variant it had.  Results do not depend on the tile shape except for the
 * summation order of the cost and inner products. */
misr_status misr_op_tune(misr_op *op, const misr_params *params, const void *y, void *x,
                         int reps, int32_t *tile_h, int32_t *tile_w, void *stream);
/* The operator's current tile shape of the update pass and the operators
 * (HR pixels; 0 x 0 for a general operator); the trial pass's tile has the
 * same height. */
misr_status misr_op_tile(const misr_op *op, int32_t *tile_h, int32_t *tile_w);
/* The operator's current tile variant (-1 for a general operator) and the
 * width of its trial-pass tile in HR pixels. */
misr_status misr_op_tile_variant(const misr_op *op, int32_t *variant, int32_t *trial_w);
/* Selects a compiled tile variant directly (as listed for misr_op_tune; 0 is
 * the default).  MISR_E_INVAL for a variant not compiled for this operator's
 * scale and band length, or for a general operator. */
misr_status misr_op_set_tile(misr_op *op, int variant);

/* --------------------------------------------------------------- operators */
/* y[k] = A_k x for every frame (Eq. sisr without noise).
 * x: device, H*W elements of dtype dt.  y: device, K*(H/s)*(W/s) of dtype dt. */
misr_status misr_forward(const misr_op *op, misr_dtype dt, const void *x, void *y,
                         void *stream);

/* x = sum_k A_k^T r_k.  r: device, K*(H/s)*(W/s) of dtype dt.  x: device, H*W
 * float32 (overwritten). */
misr_status misr_adjoint(const misr_op *op, misr_dtype dt, const void *r, float *x,
                         void *stream);

/* Multi-image interpolation, the paper's non-iterative fusion baseline
 * (Sec. 4: LR pixel values inserted at their integer HR positions).  Frame
 * k's pixel (i, j) is written to HR (s i + ty_k, s j + tx_k) with
 * t_k = round(s d_k) (halves away from zero); an HR pixel that receives
 * several samples takes their mean (frame order), one that receives none
 * frame 0's pixel (floor(u/s), floor(v/s)).  y: device, K*(H/s)*(W/s) of
 * dtype dt; x: device H*W of dtype dt (overwritten, rounded to nearest even
 * for 16-bit dtypes). */
misr_status misr_interpolate(const misr_op *op, misr_dtype dt, const void *y, void *x,
                             void *stream);

/* Bicubic upsampling of frame 0 by s (the solver's usual start point): Keys
 * cubic convolution (a = -1/2), HR pixel u at LR coordinate (u + 1/2)/s - 1/2,
 * taps clamped to the frame.  y, x as for misr_interpolate. */
misr_status misr_upsample(const misr_op *op, misr_dtype dt, const void *y, void *x,
                          void *stream);

/* J(x) and grad J(x) (Eq. objective).  x, y: device, params->img_dtype.
 * g: device float32 H*W (overwritten).  cost_dev: device double[3] receiving
 * {J, data term, lambda * prior}.  Honours params->tile_lr. */
misr_status misr_cost_grad(const misr_op *op, const misr_params *params, const void *x,
                           const void *y, float *g, double *cost_dev, void *stream);

/* misr_cost_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same J(x), grad J(x) and cost_dev {J, data term, lambda * prior}, bit
 * for bit, with no device allocation, free or host-to-device copy.  Its work
 * list, solver state and partial sums live in a fixed workspace of
 * misr_cost_grad_noalloc_max_bytes() bytes (2 MiB) in device memory of every
 * GPU the library runs on (located when a context is created on that device,
 * held until the process ends).  Banded operators (translational frames,
 * separable PSFs), untiled (params->tile_lr == 0); x and y stored as
 * params->img_dtype (x evaluated as stored).  The workspace holds 32 752
 * tiles (8192 x 8192 HR at the 48 x 96 tiles of x2 operators fits); larger
 * images return MISR_E_INVAL with the limit in misr_last_error(), before any
 * launch.  Every call on a device shares that device's workspace, and only the
 * values a call writes are read back: calls that overlap on one device (other
 * streams or threads) race; calls ordered on one stream do not. */
misr_status misr_cost_grad_noalloc(const misr_op *op, const misr_params *params, const void *x,
                                   const void *y, float *g, double *cost_dev, void *stream);
/* Bytes of the workspace of misr_cost_grad_noalloc on each device. */
size_t misr_cost_grad_noalloc_max_bytes(void);

/* SCG solve (Algorithm 1 on one GPU): params->n_iter passes from x_inout,
 * result written back to x_inout (device, params->img_dtype).  y: device.
 * trace (host, nullable): when given, the call synchronises the stream and
 * fills it.  Returns MISR_E_NUMERIC (only when trace is given; without a trace,
 * misr_scg_status reports it) if the solve stopped on a non-finite value;
 * x_inout then holds the last finite iterate. */
misr_status misr_scg_solve(const misr_op *op, const misr_params *params, const void *y,
                           void *x_inout, misr_scg_trace *trace, void *stream);

/* Outcome of the last misr_scg_solve on this operator, for callers that pass
 * no trace: Algorithm 1's output is the last iterate, and this library stops a
 * solve whose cost or curvature turns non-finite (keeping the last finite
 * iterate).  Waits for that solve: synchronises `stream`, which must be the
 * solve's stream or a stream ordered after it.  Fills summary's counters
 * (n_passes, n_success, stop, E0, E_final; summary->iters is not touched) when
 * summary is not NULL.  Returns MISR_E_NUMERIC if that solve stopped on a
 * non-finite value (stop = 2), MISR_OK otherwise; MISR_E_INVAL if no solve has
 * run on the operator.  misr_cost_grad, misr_forward and the other calls on
 * the operator do not change what it reports. */
misr_status misr_scg_status(const misr_op *op, misr_scg_trace *summary, void *stream);

/* n independent solves advanced together: every SCG pass of every projection
 * runs in the same kernel launches (one work list over all projections' tiles).
 * Per-projection state stays separate, so each result equals its solo solve.
 * ops/params/y/x/traces are host arrays of length n (traces nullable, entries
 * nullable).  Projections may differ in geometry and n_iter but must share
 * img_dtype and have tile_lr == 0. */
misr_status misr_scg_solve_batch(int n, const misr_op *const *ops,
                                 const misr_params *params, const void *const *y,
                                 void *const *x_inout, misr_scg_trace *traces, void *stream);

/* Measurement aid: times one image pass of the solve in isolation.  Prepares
 * the state of misr_scg_solve(op, params, y, x) up to the first trial point,
 * then launches pass `which` (0: fused cost+gradient at x + alpha p,
 * 1: update + curvature, 2: the two in turn, as in a solve) `reps` times on
 * the library stream between two HIP events and returns the mean duration
 * in microseconds in *avg_us (host; for 2, of one trial + update pair).
 * Both passes are idempotent at a fixed state, so repeated launches do the
 * work of one pass each.  x is left unchanged.  Synchronises the stream. */
misr_status misr_time_pass(const misr_op *op, const misr_params *params, const void *y,
                           void *x, int which, int reps, double *avg_us, void *stream);

/* ------------------------------------------------------------------ serving */
/* On-the-fly acquisition (Sec. 3.2): each rotation angle's frames arrive as a
 * request; requests are admitted while device memory allows and solved
 * together, each pass of every admitted solve in the same launches. */
typedef enum {
    MISR_REQ_QUEUED = 0,
    MISR_REQ_RUNNING = 1,
    MISR_REQ_DONE = 2,
    MISR_REQ_FAILED = 3,
    MISR_REQ_CANCELLED = 4
} misr_req_state;

typedef void (*misr_done_cb)(uint64_t id, misr_status status, void *user);

typedef struct {
    misr_geometry geom;       /* host arrays read during submit */
    misr_params params;       /* tile_lr > 0 splits a large request into tiles */
    const void *y;            /* K frames (device or host, see below) */
    const void *x0;           /* initial HR image; NULL with params.x_init > 0 */
    void *x_out;              /* result (device or host) */
    int32_t on_device;        /* 1: y, x0, x_out are device pointers; 0: host */
    misr_done_cb done_cb;     /* nullable; called from the scheduler thread */
    void *user;
} misr_request;

typedef struct {
    size_t hbm_budget_bytes;  /* cap on device memory for admitted requests */
    int32_t max_slots;        /* cap on concurrently admitted requests */
    int32_t max_queue;        /* submit returns MISR_E_BUSY beyond this */
    int32_t fail_alloc_n;     /* fault hook: the n-th slot allocation fails (0 off) */
    int32_t fill_mpx;         /* 0: admit whatever memory and slots allow (every
                                 admitted solve advances in every pass); > 0:
                                 admit in arrival order only while the admitted
                                 solves hold fewer than fill_mpx million HR
                                 pixels (a request is always admitted when none
                                 runs), so small requests are batched to fill the
                                 device and large ones keep first-come order */
    int32_t fail_list_n;      /* fault hook: the n-th work-list allocation fails
                                 (0 off); every request of that cycle then fails
                                 with MISR_E_NOMEM and none of its kernels runs */
    int32_t max_idle_ops;     /* cached operators (one per distinct geometry)
                                 that no admitted request uses are kept up to
                                 this many (0: 8), least recently used evicted
                                 first; idle ones are also evicted when a
                                 request would not fit the budget.  Evicting
                                 waits for the device (misr_op_destroy).
                                 Negative: MISR_E_INVAL */
    int32_t order;            /* 0: every admitted solve advances in every
                                 cycle (admission as fill_mpx says).  1 and 2:
                                 requests are admitted in arrival order while
                                 memory and slots allow (fill_mpx holds none
                                 back), and each cycle (about 3 ms of device
                                 time) advances the admitted solves first in
                                 the order's key, arrival order among equals,
                                 as many as fit in fill_mpx million HR pixels
                                 (at least one; fill_mpx 0: all).  1, shortest
                                 remaining work first: key HR pixels x passes
                                 left (a large request waits while smaller
                                 ones keep arriving); 2, earliest finish
                                 first: key submit time + the device time of
                                 the work left at the server's running
                                 estimate (a request that has waited long
                                 enough is no longer overtaken).  A solve left
                                 out of a cycle keeps its state on the device
                                 and resumes unchanged; results do not depend
                                 on the order.  Other values: MISR_E_INVAL */
} misr_server_config;

/* Occupancy of a server (misr_server_query). */
typedef struct {
    int32_t queued;           /* requests waiting for admission */
    int32_t running;          /* requests admitted and not yet retired */
    int32_t n_ops;            /* cached operators (one per distinct geometry) */
    int32_t n_idle_ops;       /* of those, operators no admitted request uses */
    size_t used_bytes;        /* device bytes charged against hbm_budget_bytes:
                                 the admitted requests' buffers and work-list
                                 share, and the cached operators' tables */
} misr_server_info;

typedef struct {
    double t_submit_us, t_admit_us, t_done_us;  /* host steady clock */
    int32_t n_passes, n_success;
    misr_status status;
    int32_t pad_;
    double E_final;
    size_t bytes;             /* device bytes charged to the request while it
                                 is admitted: its buffers and work-list share */
    size_t op_bytes;          /* estimate of its operator's tables, charged at
                                 admission unless the operator is cached (the
                                 cache then charges the tables' exact size) */
} misr_req_stats;

misr_status misr_server_create(misr_ctx *ctx, const misr_server_config *cfg,
                               misr_server **out);
/* Non-blocking; assigns *id. */
misr_status misr_server_submit(misr_server *s, const misr_request *req, uint64_t *id);
misr_status misr_server_poll(misr_server *s, uint64_t id, misr_req_state *state,
                             misr_req_stats *stats);
/* Blocks until the request leaves QUEUED/RUNNING or timeout_us passes (<0: forever). */
misr_status misr_server_wait(misr_server *s, uint64_t id, int64_t timeout_us);
misr_status misr_server_cancel(misr_server *s, uint64_t id);
/* Current occupancy (host-side counters; no device call). */
misr_status misr_server_query(misr_server *s, misr_server_info *out);
/* Drains every submitted request, waits for the device to go idle, then
 * frees the server (always).  Returns MISR_E_HIP if that wait reports a device
 * error. */
misr_status misr_server_destroy(misr_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MISR_H */
