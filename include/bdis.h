/*
 * bdis.h -- C ABI of the MI355X (gfx950) BDIS dense-inverse-search stereo library.
 *
 * BDIS (Song, Zhu, Lin, Ghaffari, arXiv 2205.03133) estimates per-pixel
 * disparity of a rectified stereo pair by a coarse-to-fine dense inverse
 * search (Sec. III, Fig. 1): per pyramid level, a per-patch inverse-
 * compositional 1-D Lucas-Kanade search (Eq. 1), a Bayesian window posterior
 * per patch (Eq. 5-6), and probability-weighted fusion of the overlapping
 * patches through a spatial Gaussian mixture (Eq. 9-13), with the fused map
 * initialising the next finer level.  An optional per-pixel variance follows
 * Eq. 15-18 (disparity form, without the depth Jacobian).  Also exported: a
 * float form with reverse-mode gradients (bdis_compute_f32, bdis_backward),
 * batches of pairs of mixed sizes in one call, the paper's preset that stops
 * at a coarser level and upsamples (finest_level), the depth form of Eq. 14
 * and 18 (bdis_depth), the ablation weightings of Sec. V (fusion,
 * propagate), the variance coverage check (bdis_coverage) and the 2-D
 * optical-flow form of the underlying dense inverse search (bdis_flow).
 *
 * Conventions shared by every entry point:
 *  - Image and output pointers are DEVICE pointers (HBM of the current HIP
 *    device), row-major, `pitch` in ELEMENTS, pitch >= w.  Outputs are written
 *    with pitch w (dense H x W).
 *  - Disparity is d = x_left - x_right: left pixel x matches right pixel x - d.
 *  - Every output pixel is written.  Invalid pixels (no accepted patch covers
 *    them at the finest level, or confidence below `prob_thresh`) get NaN
 *    disparity, NaN variance and confidence 0.
 *  - The caller owns inputs and outputs.  The library owns its workspace,
 *    allocated in bdis_create and released in bdis_destroy.
 *  - Compute calls are asynchronous on `stream` (a hipStream_t; NULL is the
 *    null stream) once a batch shape has been seen.  The first call with a
 *    new batch shape (pair sizes, levels and parameters) times the
 *    launch shapes of every level on `stream` (search lanes per patch and
 *    workgroup size, fusion tile height, pyramid form, and whether the
 *    coarsest level's pyramid step, search and fusion run as one workgroup
 *    per pair, and whether runs of small pyramid levels are built by one
 *    launch) and synchronises it,
 *    then records the launch sequence as a graph; a job table larger than any
 *    before synchronises the device before it is reallocated.  A context
 *    keeps at most 32 recorded sequences: recording one more destroys the
 *    least recently launched one, after synchronising the device.  The tuned
 *    choices persist in a cache file keyed by the device architecture, the
 *    library version and the level shapes (read by bdis_create, rewritten
 *    after tuning), so a later process skips the timing.  Environment: BDIS_TUNE=0 skips the timing
 *    (size-based defaults), BDIS_TUNE_CACHE=path names the cache file
 *    (default $HOME/.cache/bdis/tune.json; empty: no file), BDIS_GRAPH=0
 *    launches eagerly without graphs, BDIS_SEARCH_CONFIG=k (read by
 *    bdis_create; k = lane mapping * 4 + workgroup-size index into 64, 128,
 *    256, 512) uses search configuration k on every level without timing
 *    (bdis_create fails with BDIS_E_ARG for an invalid k); read by
 *    bdis_create, BDIS_TOP=0 / 1 keeps the coarsest level in its per-phase
 *    launches / runs it as one workgroup per pair where that fits, and
 *    BDIS_CHAIN=0 / 1 builds the pyramid one launch per level / builds runs of
 *    small levels in one launch where possible (unset: the tuner times both).
 *  - Errors are returned as bdis_status; the library never aborts.  The text
 *    of the last error of a context is available from bdis_last_error.
 *  - A context is not thread-safe: calls on one context must come from one
 *    host thread at a time.  Calls on different streams are ordered by the
 *    library, because every call reuses the context's workspace: the first
 *    change of stream drains the device once, later ones make the new stream
 *    wait for the previous call's work.
 */
#ifndef BDIS_H
#define BDIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdis_ctx bdis_ctx;

typedef enum {
  BDIS_OK = 0,
  BDIS_E_ARG = -1,      /* null pointer, parameter out of range, non-finite float input   */
  BDIS_E_SIZE = -2,     /* a processed pyramid level is smaller than the patch            */
  BDIS_E_CAPACITY = -3, /* request exceeds the limits given to bdis_create               */
  BDIS_E_HIP = -4,      /* a HIP runtime call failed (text in bdis_last_error)            */
  BDIS_E_NOMEM = -5,    /* workspace allocation failed; the context stays usable         */
  BDIS_E_STATE = -6     /* call not valid in the current state                          */
} bdis_status;

#define BDIS_MAX_LEVELS 8
#define BDIS_MAX_PATCH 16

/* Method parameters.  Defaults (bdis_params_default) follow the parameter
 * list of Sec. IV-A where the paper gives a value. */
typedef struct {
  int32_t levels;          /* L, 1..8: pyramid levels n = L-1 (coarsest) .. finest_level     */
  int32_t finest_level;    /* f, 0..L-1: finest searched level (paper: scale 2^1 -> f = 1);  */
                           /* f > 0 upsamples its maps to W x H (bilinear at x / 2^f; the    */
                           /* disparity scaled by 2^f, the variance by 4^f)                  */
  int32_t patch;           /* P, 3..16: square patch side (paper: 10)                        */
  int32_t stride;          /* S, 1..P: patch-grid stride (paper: overlap 0.55 -> S = 4)      */
  int32_t iters;           /* K, 1..256: fixed inverse-compositional iterations (paper: 12)  */
  int32_t sigma_r_dynamic; /* 1: sigma_r from the spread of the level's residuals (Sec.III-B)*/
  int32_t variance;        /* 1: per-patch (Eq. 15-17) and per-pixel (Eq. 18) variance      */
  int32_t float_pyramid;   /* 0: uint8 entry points (integer pyramid); 1: float entry points */
  float sigma_s;           /* spatial sigma of the mixture kernel, level px (paper: 4)       */
  float sigma_r;           /* fixed sigma_r (dynamic == 0) or its scale alpha_r (dynamic)   */
  float valid_ratio;       /* gamma in (0, 1]: least in-bounds fraction of an accepted patch  */
  float var_fail_sigma;    /* sigma given to a failed variance fit; <= 0 means P             */
  float var_fit_thresh;    /* largest mean squared fit residual of Eq. 17 (paper: 0.1)       */
  float prob_thresh;       /* confidence below this is invalid; 0 disables (paper: 0.15)     */
  float level_weight[BDIS_MAX_LEVELS]; /* omega_n: level n weighs omega_n / sum (Eq. 12: 2^n) */
  int32_t fusion;          /* fusion weight of a patch at a pixel: 0 mask x probability      */
                           /* (Eq. 13, default); 1 inverse squared photometric residual of   */
                           /* the pixel, floored at 1 (Eq. 2, the DIS baseline); 2 Eq. 13    */
                           /* with a uniform mask (the "no sGMM" ablation of Sec. V)         */
  int32_t propagate;       /* 1 (default): patch probability adds the parent confidence      */
                           /* (Eq. 11); 0: level term only (the "no coarse-to-fine" ablation)*/
} bdis_params;

/* One stereo pair of a batch (all pointers device pointers). */
typedef struct {
  const uint8_t* left;
  const uint8_t* right;
  int32_t w, h, pitch;
  int32_t levels;          /* pyramid depth for this pair (finest_level < levels <= params.levels); 0 means params.levels */
  float* disparity;        /* H x W, required                                             */
  float* variance;         /* H x W, or NULL                                              */
  float* confidence;       /* H x W, or NULL                                              */
} bdis_pair;

/* Fills *p with the defaults.  BDIS_E_ARG if p is NULL. */
bdis_status bdis_params_default(bdis_params* p);

/* Checks parameters on their own (no image size).  BDIS_OK or BDIS_E_ARG. */
bdis_status bdis_params_check(const bdis_params* p);

/* Creates a context for images up to max_w x max_h and batches of up to
 * max_batch pairs, allocating its device workspace on the current device.
 * The workspace holds what the coarse-to-fine pass of Sec. III / Fig. 1 keeps
 * between its steps: the pyramid of both views (one pixel of level n covers
 * 2^n x 2^n input pixels, Sec. III-B), the per-patch search results of each
 * level (Eq. 1, 5-6) and the fused maps that start the next finer level
 * (Eq. 13, Fig. 1).
 * flags: 0, or a combination of BDIS_TRAIN (the differentiable float path,
 * below) and BDIS_KEEP (intermediates for bdis_debug_dump).  On failure *out
 * is NULL.
 * Errors: BDIS_E_ARG (null out/params, bad params, max_* < 1),
 *         BDIS_E_SIZE (max_w x max_h too small for the levels and patch),
 *         BDIS_E_NOMEM, BDIS_E_HIP. */
bdis_status bdis_create(bdis_ctx** out, const bdis_params* p, int max_w, int max_h, int max_batch,
                        unsigned flags);

/* Replaces the method parameters of a context.  Parameters that size the
 * workspace (levels, patch, stride) must stay within what bdis_create sized:
 * otherwise BDIS_E_CAPACITY and the old parameters stay in force. */
bdis_status bdis_set_params(bdis_ctx* ctx, const bdis_params* p);

/* One rectified uint8 pair -> disparity (required), variance and confidence
 * (nullable): the problem the paper states in Sec. III (a rectified pair in,
 * per-pixel disparity out; coarse to fine as in Fig. 1), each level searched
 * patch by patch (Eq. 1, inverse-compositional 1-D search; Eq. 5-6 window
 * posterior) and fused (Eq. 9-13); confidence is the fused probability of
 * Eq. 13, variance the disparity form of Eq. 15-18.  variance must be NULL
 * unless params.variance is 1.
 * Errors: BDIS_E_ARG, BDIS_E_SIZE (image too small for levels/patch),
 *         BDIS_E_CAPACITY (w > max_w or h > max_h), BDIS_E_HIP. */
bdis_status bdis_compute(bdis_ctx* ctx, const uint8_t* left, const uint8_t* right, int w, int h,
                         int pitch, float* disparity, float* variance, float* confidence,
                         void* stream);

/* A batch of n pairs of possibly different sizes and pyramid depths, all in
 * one call (every level of every pair in a fixed sequence of launches): per
 * pair the same computation as bdis_compute (Sec. III, Eq. 1, 5-6, 9-13,
 * 15-18), with the same results bit for bit.
 * pairs is a HOST array of n descriptors.  Outputs as bdis_compute.
 * Errors: as bdis_compute, plus BDIS_E_CAPACITY if n > max_batch. */
bdis_status bdis_compute_batch(bdis_ctx* ctx, int n, const bdis_pair* pairs, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bdis_compute
 * of one uint8 pair without a context.  Same arguments and outputs as
 * bdis_compute, with the method parameters passed directly.  The workspace and
 * job table live in a static device array of 48 MiB that the library holds on
 * every device it runs on until the process ends; the call allocates nothing
 * (no hipMalloc, no pinned staging, no graph) and does not tune (the default
 * search configuration of each level).  Every call on a device shares that
 * device's array and leaves its contents behind (each array is rewritten
 * before it is read, so nothing needs clearing): calls that overlap on one
 * device -- on different streams or from different host threads -- race, so
 * order them on one stream.  The pass runs asynchronously on `stream`; the
 * host is never synchronised.  Errors: BDIS_E_ARG, BDIS_E_SIZE,
 * BDIS_E_CAPACITY (the pair's workspace does not fit the array: e.g. one
 * 1920 x 1080 pair at patch 8, stride 3, 6 levels fits, a 4K pair does not;
 * the message gives the bytes needed), BDIS_E_HIP.  The text of a failure is
 * read with bdis_last_error(NULL). */
bdis_status bdis_compute_static(const bdis_params* p, const uint8_t* left, const uint8_t* right, int w, int h,
                                int pitch, float* disparity, float* variance, float* confidence, void* stream);

/* ---- differentiable (float) path --------------------------------------- */

/* bdis_create flag: size the workspace for the float path and keep the state
 * its backward pass needs (iterates of every patch, fusion sums, adjoints). */
#define BDIS_TRAIN 1u
/* bdis_create flag: store every per-patch intermediate of the uint8 path for
 * bdis_debug_dump (start values, SSD(0), in-bounds ratios, Hessians and the
 * patch records of every level).  Without it the search stores only what the
 * later phases read (displacement, propagated probability, window SSD
 * differences, acceptance). */
#define BDIS_KEEP 2u

/* One float pair of a batch (device pointers, pitch in elements). */
typedef struct {
  const float* left;
  const float* right;
  int32_t w, h, pitch;
  int32_t levels;          /* 0 means params.levels                                       */
  float* disparity;
  float* variance;         /* or NULL */
  float* confidence;       /* or NULL */
} bdis_pair_f32;

/* Output gradients in, image gradients out, for one pair (device pointers,
 * dense W x H; grad_variance / grad_left / grad_right may be NULL). */
typedef struct {
  const float* grad_disparity;
  const float* grad_variance;
  float* grad_left;
  float* grad_right;
} bdis_pair_grad;

/* Float images -> outputs, as bdis_compute, through the same method with an
 * FP64 pyramid without rounding (params.float_pyramid must be 1; the context
 * must have been created with BDIS_TRAIN).  The state of the call is kept for
 * bdis_backward.  Errors: as bdis_compute, plus BDIS_E_STATE. */
bdis_status bdis_compute_f32(bdis_ctx* ctx, const float* left, const float* right, int w, int h, int pitch,
                             float* disparity, float* variance, float* confidence, void* stream);
bdis_status bdis_compute_f32_batch(bdis_ctx* ctx, int n, const bdis_pair_f32* pairs, void* stream);

/* Reverse mode through the last float-path call (the fixed-K unrolled search
 * and the Bayesian fusion of every level, then the pyramid): given
 * dL/d disparity (and dL/d variance), writes dL/d left and dL/d right (float,
 * dense W x H) and, if grad_hyper is not NULL, the DEVICE array of 2 + L
 * doubles [dL/d sigma_s, dL/d sigma_r (alpha_r when dynamic), dL/d omega_0 ..
 * dL/d omega_{L-1}], summed over the pairs of the call.  Discrete decisions
 * (unit cells, resets, acceptance, holes, variance-fit outcomes) carry no
 * gradient.  Errors: BDIS_E_STATE without a preceding float-path call,
 * BDIS_E_ARG for a batch size that differs from it. */
bdis_status bdis_backward(bdis_ctx* ctx, const float* grad_disparity, const float* grad_variance,
                          float* grad_left, float* grad_right, double* grad_hyper, void* stream);
bdis_status bdis_backward_batch(bdis_ctx* ctx, int n, const bdis_pair_grad* grads, double* grad_hyper,
                                void* stream);

/* Optical-flow form (f4): the 2-D dense inverse search that BDIS builds on
 * (Eq. 1 with u a 2-vector) between two uint8 frames i0, i1 (device, row
 * pitch `pitch`), with the context's levels, patch, stride and iterations:
 * per patch an inverse-compositional update on the 2 x 2 Hessian of the
 * Sobel-x / Sobel-y template gradients (bilinear warp, indices clamped; no
 * update when det H < 1e-3; reset to the start after a step longer than P),
 * per pixel the DIS fusion of Eq. 2.  Writes the flow (u, v), I1(x + u, y + v)
 * ~ I0(x, y), as dense float W x H maps.  Needs float_pyramid 0 and
 * finest_level 0; the probability, variance and ablation parameters are not
 * used.  Errors: BDIS_E_ARG, BDIS_E_CAPACITY, BDIS_E_SIZE, BDIS_E_HIP. */
bdis_status bdis_flow(bdis_ctx* ctx, const uint8_t* i0, const uint8_t* i1, int w, int h, int pitch, float* flow_u,
                      float* flow_v, void* stream);

/* Depth form (Eq. 14 and Eq. 18): for each pixel of a W x H disparity map (and
 * its variance), depth = fb / d and depth variance = (fb)^2 / d^4 * var, where
 * fb is focal length x baseline (depth comes out in the units of the
 * baseline when d and f are in pixels).  Pixels with d <= 0 or NaN get NaN.
 * All pointers are device pointers with row pitch `pitch` (elements) on the
 * inputs and dense W x H outputs; `variance` and `depth_variance` may be NULL
 * (together).  Asynchronous on `stream`.  Errors: BDIS_E_ARG. */
bdis_status bdis_depth(bdis_ctx* ctx, const float* disparity, const float* variance, int w, int h, int pitch,
                       float fb, float* depth, float* depth_variance, void* stream);

/* Variance coverage (the frame-wise check of Sec. V, Table 6): over the pixels of
 * a W x H map with a finite disparity, a finite non-negative variance, a finite
 * reference disparity and valid != 0 (`valid` may be NULL), counts those with
 * |d - ref| <= k sqrt(var), the comparison taken in double precision.
 * counts: DEVICE array of 2 int64 (covered, considered), overwritten.
 * disparity/variance/reference are float maps with row pitch `pitch`, valid
 * (uint8) shares it.  Asynchronous on `stream`.  Errors: BDIS_E_ARG. */
bdis_status bdis_coverage(bdis_ctx* ctx, const float* disparity, const float* variance, const float* reference,
                          const uint8_t* valid, int w, int h, int pitch, float k, long long* counts, void* stream);

/* Debug access to the intermediates of the last single-pair compute (the
 * call synchronises `stream`).  `what` selects the array (BDIS_DBG_*), bytes
 * is the capacity of host_dst; returns BDIS_E_ARG if too small.  UINIT, SSD0,
 * RHO, HESS and DENS are stored only by contexts created with BDIS_KEEP
 * (BDIS_E_STATE otherwise). */
enum {
  BDIS_DBG_LEFT = 0,    /* uint8 level image, W_n x H_n                              */
  BDIS_DBG_RIGHT = 1,   /* uint8 level image                                         */
  BDIS_DBG_UINIT = 2,   /* double per patch: initial displacement                    */
  BDIS_DBG_PIPAR = 3,   /* double per patch: probability propagated from the parent  */
  BDIS_DBG_U = 4,       /* double per patch: final displacement (= -disparity)       */
  BDIS_DBG_SSD0 = 5,    /* double per patch: window SSD at the centre                */
  BDIS_DBG_DSSD = 6,    /* double[4] per patch: SSD(d)-SSD(0), d = -1,-1/2,1/2,1     */
  BDIS_DBG_RHO = 7,     /* float per patch: in-bounds ratio                          */
  BDIS_DBG_ACC = 8,     /* int32 per patch: 1 accepted                               */
  BDIS_DBG_HESS = 9,    /* float per patch: Hessian                                  */
  BDIS_DBG_DENS = 10,   /* double[4] per patch: (u, weight pi or -1, sigma_k^2, post)*/
  BDIS_DBG_UBAR = 11,   /* double level map (levels above the finest)                */
  BDIS_DBG_QMAP = 12,   /* double level map (levels above the finest)                */
  BDIS_DBG_SCAL = 13    /* double[2]: sigma_r^2, tau of the level                    */
};
bdis_status bdis_debug_dump(bdis_ctx* ctx, int level, int what, void* host_dst, size_t bytes,
                            void* stream);

/* Per-kernel timing (for measurement): while enabled, calls launch eagerly
 * (no graph) and each timed launch carries a pair of HIP events that its
 * kernel dispatches record themselves (hipExtLaunchKernelGGL: start of the
 * first kernel, end of the last), so a span is the kernels' own execution, as
 * a profiler's kernel trace reports it.  kernel: 0 pyramid, 1 patch search,
 * 2 patch probability (launched for large levels only; small levels compute
 * it inside the fusion), 3 fusion, 4 the per-pair sigma_r reduction (large
 * levels only), 5 the backward pass (all launches of a level), 6 the coarsest
 * level run as one workgroup per pair (its pyramid step, search, level
 * scalars, records and fusion in one launch).  A phase that
 * launches nothing on a level is not counted.  bdis_timing_enable(ctx, 1)
 * clears the totals and starts recording; bdis_timing_read synchronises the
 * recorded events and returns the summed GPU time (ms) and the launch count
 * of one kernel since enabling; bdis_timing_read_level the same for one
 * pyramid level (level -1: all levels). */
enum {
  BDIS_K_PYRAMID = 0,
  BDIS_K_SEARCH = 1,
  BDIS_K_PROB = 2,
  BDIS_K_FUSE = 3,
  BDIS_K_REDUCE = 4,
  BDIS_K_BACKWARD = 5,
  BDIS_K_TOP = 6,
  BDIS_K_COUNT = 7
};
bdis_status bdis_timing_enable(bdis_ctx* ctx, int enable);
/* Host time (ms) the last bdis_compute / bdis_compute_batch call spent tuning
 * launch shapes (first call of a new batch shape without a cached choice) and
 * capturing its graph (first call of a new launch sequence); 0 when it did
 * neither.  Errors: BDIS_E_ARG. */
bdis_status bdis_setup_time(bdis_ctx* ctx, double* tune_ms, double* capture_ms);
bdis_status bdis_timing_read(bdis_ctx* ctx, int kernel, double* total_ms, long* launches);
bdis_status bdis_timing_read_level(bdis_ctx* ctx, int kernel, int level, double* total_ms, long* launches);

/* Geometry of level `level` for a w x h input: level size and patch grid. */
bdis_status bdis_level_dims(const bdis_params* p, int w, int h, int level, int* lw, int* lh,
                            int* nx, int* ny);

/* Frees the context and its workspace (synchronises the device). NULL is a no-op. */
void bdis_destroy(bdis_ctx* ctx);

/* Text of the last error on ctx (or, with ctx NULL, of the last failed
 * bdis_create or bdis_compute_static). */
const char* bdis_last_error(const bdis_ctx* ctx);

/* Library version string. */
const char* bdis_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BDIS_H */
