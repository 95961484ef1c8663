/*
 * bdis_ref.h -- plain FP64 CPU oracle of the BDIS dense-inverse-search stereo
 * hot path (Song et al., "BDIS: Bayesian Dense Inverse Searching Method for
 * Real-Time Stereo Surgical Image Matching", Sec. III, Eq. 1-18).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against; it is loaded by the test-suite, by the smoke check and by the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code,
 * header or table with the GPU library.
 *
 * All images are host pointers, row-major, `pitch` in elements (pitch >= w).
 * Outputs are caller-owned H x W double arrays (pitch = w).  Disparity uses
 * d = x_left - x_right; invalid pixels get NaN disparity / NaN variance and
 * confidence 0.
 */
#ifndef BDIS_REF_H
#define BDIS_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t levels;          /* L: levels n = L-1 (coarsest) .. finest_level                 */
  int32_t finest_level;    /* f: finest processed level, 0 <= f < L; f > 0 upsamples its maps */
  int32_t patch;           /* P: square patch side, >= 3                                    */
  int32_t stride;          /* S: patch-grid stride, 1 <= S <= P                             */
  int32_t iters;           /* K: fixed number of inverse-compositional iterations, >= 1     */
  int32_t sigma_r_dynamic; /* 1: photometric sigma from the level's residuals; 0: fixed     */
  int32_t variance;        /* 1: per-patch and per-pixel variance at the finest level      */
  int32_t float_pyramid;   /* 1: pyramid without integer rounding (used by the f64 entry)   */
  double sigma_s;          /* spatial sigma of the patch mixture kernel (level px)          */
  double sigma_r;          /* fixed sigma_r, or the scale alpha_r when dynamic              */
  double valid_ratio;      /* gamma in (0, 1]: minimum in-bounds fraction of an accepted patch */
  double var_fail_sigma;   /* sigma assigned to a failed variance fit; <= 0 means P         */
  double var_fit_thresh;   /* largest accepted mean squared fit residual (ln-p units)       */
  double prob_thresh;      /* pixels with confidence below this are invalid; 0 = off        */
  double level_weight[8];  /* omega_n; level n contributes omega_n / sum(omega)             */
  int32_t fusion;          /* fusion weight: 0 Eq. 13 (mask x probability), 1 Eq. 2 (inverse */
                           /* squared photometric residual, DIS), 2 Eq. 13 with a uniform mask */
  int32_t propagate;       /* 1: add the parent confidence Pi (Eq. 11); 0: level term only    */
} bdis_ref_params;

typedef struct bdis_ref_trace bdis_ref_trace;

enum { BDIS_REF_OK = 0, BDIS_REF_E_ARG = -1, BDIS_REF_E_SIZE = -2, BDIS_REF_E_NOMEM = -5 };

/* Per-level intermediates kept in a trace (all copied out as doubles). */
enum {
  BDIS_REF_LEFT = 0,     /* level image, left  (W_n x H_n)                      */
  BDIS_REF_RIGHT = 1,    /* level image, right (W_n x H_n)                      */
  BDIS_REF_GRAD = 2,     /* x-gradient of the left level, Sobel / 8             */
  BDIS_REF_UINIT = 3,    /* per patch: initial displacement                     */
  BDIS_REF_PIPAR = 4,    /* per patch: probability propagated from the parent   */
  BDIS_REF_U = 5,        /* per patch: final displacement u (= -disparity)      */
  BDIS_REF_SSD = 6,      /* per patch: 5 window SSDs, offsets -1,-1/2,0,1/2,1   */
  BDIS_REF_RHO = 7,      /* per patch: in-bounds ratio                          */
  BDIS_REF_ACC = 8,      /* per patch: 1 accepted, 0 rejected                   */
  BDIS_REF_POST = 9,     /* per patch: window posterior (0 if rejected)         */
  BDIS_REF_PI = 10,      /* per patch: propagated probability (0 if rejected)   */
  BDIS_REF_SIGK2 = 11,   /* per patch: variance (finest level, NaN otherwise)   */
  BDIS_REF_HESS = 12,    /* per patch: Gauss-Newton Hessian H                   */
  BDIS_REF_UBAR = 13,    /* level map: fused displacement                       */
  BDIS_REF_QMAP = 14,    /* level map: fused confidence                         */
  BDIS_REF_VALID = 15,   /* level map: 1 where at least one patch contributed   */
  BDIS_REF_ODISP = 16,   /* finest level f > 0: disparity before upsampling     */
  BDIS_REF_OVAR = 17,    /* finest level f > 0: variance before upsampling      */
  BDIS_REF_OCONF = 18,   /* finest level f > 0: confidence before upsampling    */
  BDIS_REF_FV = 19,      /* optical flow: per patch vertical displacement v     */
  BDIS_REF_VBAR = 20,    /* optical flow: level map of the fused v (UBAR: u)    */
  BDIS_REF_GY = 21       /* optical flow: y-gradient of the first frame (GRAD: x) */
};
enum { BDIS_REF_SIGMA_R2 = 0, BDIS_REF_TAU = 1, BDIS_REF_NACC = 2, BDIS_REF_GAMMA = 3 };

/* Integer path: uint8 images, integer-rounded pyramid (float_pyramid ignored). */
int bdis_ref_compute_u8(const bdis_ref_params* p, const uint8_t* left, const uint8_t* right,
                        int w, int h, int pitch, double* disparity, double* variance,
                        double* confidence, bdis_ref_trace** trace);
/* Float path: double images, pyramid without rounding. */
int bdis_ref_compute_f64(const bdis_ref_params* p, const double* left, const double* right,
                         int w, int h, int pitch, double* disparity, double* variance,
                         double* confidence, bdis_ref_trace** trace);

/* 2-D dense inverse search (DIS optical flow, the base method BDIS extends):
 * frames I0, I1 (uint8, integer pyramid), flow (u, v) with I1(x + u, y + v) ~
 * I0(x, y); levels, patch, stride and iters from p (finest_level must be 0);
 * per-patch 2-D inverse-compositional LK, fusion with the DIS weights of Eq. 2.
 * Outputs: dense W x H doubles.  The trace keeps u (U, UBAR) and v (FV, VBAR). */
int bdis_ref_flow(const bdis_ref_params* p, const uint8_t* i0, const uint8_t* i1, int w, int h, int pitch,
                  double* flow_u, double* flow_v, bdis_ref_trace** trace);

/* Level geometry: image size and patch-grid size; returns 0 or BDIS_REF_E_ARG. */
int bdis_ref_trace_dims(const bdis_ref_trace* t, int level, int* w, int* h, int* nx, int* ny);
/* Copies `what` of `level` into dst (capacity n doubles); returns the count or < 0. */
long bdis_ref_trace_get(const bdis_ref_trace* t, int level, int what, double* dst, long n);
double bdis_ref_trace_scalar(const bdis_ref_trace* t, int level, int what);
/* Hash of every discrete decision of a level (cells, resets, acceptances,
 * variance-fit outcomes, holes): equal hashes mean equal branches. */
uint64_t bdis_ref_trace_hash(const bdis_ref_trace* t, int level);
void bdis_ref_trace_free(bdis_ref_trace* t);

/* Start of the patches of a w x h level from the parent level's fused maps
 * (pw x ph): per patch k of the level's grid (row-major), uinit[k] = 2 ubar and
 * pipar[k] = qmap, both sampled bilinearly (indices clamped) at half the patch
 * centre.  The same routine the compute entry points use between levels. */
int bdis_ref_parent_init(const double* ubar, const double* qmap, int pw, int ph, int w, int h, int P, int S,
                         double* uinit, double* pipar);

/* Patch-grid origins along an axis of length n; returns the count or < 0. */
int bdis_ref_grid(int n, int patch, int stride, int* origins, int cap);

/* Spatial mixture mask M (P x P, row b, column a), as defined for the densification. */
int bdis_ref_mask(int patch, double sigma_s, double* dst);

/* Variance coverage (the frame-wise check of Sec. V, Table 6): over pixels with a
 * valid disparity, a finite variance, a finite reference and valid[i] != 0 (valid
 * may be NULL), counts those with |d - ref| <= k sqrt(var).  Writes the count
 * and the number of pixels considered. */
int bdis_ref_coverage(const double* disp, const double* var, const double* ref, const uint8_t* valid,
                      long n, double k, long* covered, long* total);

/* Depth form (Eq. 14, 18): depth = fb / d and depth variance (fb)^2 / d^4 * var
 * for d > 0 (fb = focal length x baseline, in the units wanted for depth);
 * NaN elsewhere.  `var` and `depth_var` may be NULL. */
int bdis_ref_depth(const double* disp, const double* var, long n, double fb, double* depth,
                   double* depth_var);

#ifdef __cplusplus
}
#endif
#endif
