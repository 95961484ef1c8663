/*
 * bdis_ref.c -- plain, slow, FP64 CPU oracle of the BDIS hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see bdis_ref.h).  Written for readability, not
 * speed: every step is a direct loop over the definition, sums run in
 * ascending patch index and ascending pixel index, exp is libm's, and the
 * library is compiled with -ffp-contract=off.
 *
 * Paper: Song, Zhu, Lin, Ghaffari, "BDIS: Bayesian Dense Inverse Searching
 * Method for Real-Time Stereo Surgical Image Matching" (arXiv 2205.03133).
 * The readings taken where the paper is silent are listed in the design notes
 * and repeated at each step below.
 */
#include "bdis_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NWIN 5               /* samples in the Bayesian window (Sec. IV-A parameter list) */
#define EPS_H 1e-3           /* smallest Hessian that is inverted                         */
#define EPS_SIGMA 1e-6       /* floor of the dynamic sigma_r^2                            */
#define MAX_LEVELS 8

static const double kWinOffset[NWIN] = {-1.0, -0.5, 0.0, 0.5, 1.0};

typedef struct {
  int w, h, nx, ny;
  double* left;   /* w*h */
  double* right;  /* w*h */
  double* grad;   /* w*h */
  /* per patch */
  double *uinit, *pipar, *u, *ssd, *rho, *acc, *post, *pi, *sigk2, *hess;
  /* maps */
  double *ubar, *qmap, *valid;
  double *odisp, *ovar, *oconf; /* finest level f > 0: outputs before upsampling */
  double *fv, *vbar, *gy;        /* optical flow: per patch v, level map of v, y-gradient */
  double sigma_r2, tau, nacc, gamma;
  uint64_t dhash; /* hash of every discrete decision taken on this level */
} ref_level;

struct bdis_ref_trace {
  int levels;
  ref_level lv[MAX_LEVELS];
};

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* FNV-1a over the discrete decisions (unit cells, resets, acceptances, holes,
 * variance-fit outcomes); two runs with equal hashes took the same branches,
 * so a finite difference between them measures a derivative. */
static void mix(uint64_t* h, long long v) {
  for (int b = 0; b < 8; ++b) {
    *h ^= (uint64_t)((v >> (8 * b)) & 0xff);
    *h *= 1099511628211ULL;
  }
}

/* Reflect-101 border: -1 -> 1, -2 -> 2, n -> n-2, n+1 -> n-3. */
static int reflect101(int i, int n) {
  while (i < 0 || i >= n) {
    if (i < 0) i = -i;
    if (i >= n) i = 2 * (n - 1) - i;
  }
  return i;
}

/* Bilinear sample of a w x h map at (x, y) with indices clamped to the map. */
static double bilinear(const double* m, int w, int h, double x, double y) {
  double fx0 = floor(x), fy0 = floor(y);
  double ax = x - fx0, ay = y - fy0;
  int x0 = clampi((int)fx0, 0, w - 1), x1 = clampi((int)fx0 + 1, 0, w - 1);
  int y0 = clampi((int)fy0, 0, h - 1), y1 = clampi((int)fy0 + 1, 0, h - 1);
  double top = (1.0 - ax) * m[(size_t)y0 * w + x0] + ax * m[(size_t)y0 * w + x1];
  double bot = (1.0 - ax) * m[(size_t)y1 * w + x0] + ax * m[(size_t)y1 * w + x1];
  return (1.0 - ay) * top + ay * bot;
}

/* Patch grid along one axis of a level of size n (Sec. IV-A: patch size and
 * overlap; the stride S is given directly).  Origins i*S, the last one moved
 * to n-P so the grid ends on the border; count ceil((n-P)/S)+1. */
static int grid_count(int n, int P, int S) { return (n - P + S - 1) / S + 1; }
static int grid_origin(int i, int n, int P, int S) {
  int o = i * S;
  return o < n - P ? o : n - P;
}

/* ------------------------------------------------------------------------- */
/* O1: pyramid.  One pixel of level n stands for 2^n x 2^n input pixels      */
/* (Sec. III-B).  Reading: separable binomial [1 4 6 4 1]/16 with reflect-101 */
/* borders, sampled at even pixels; integer path rounds (sum + 128) >> 8.     */
/* ------------------------------------------------------------------------- */
static const int kBinom[5] = {1, 4, 6, 4, 1};

static void pyramid_down(const double* src, int sw, int sh, double* dst, int dw, int dh,
                         int integer) {
  for (int j = 0; j < dh; ++j)
    for (int i = 0; i < dw; ++i) {
      double acc = 0.0;
      for (int b = 0; b < 5; ++b) {
        int y = reflect101(2 * j + b - 2, sh);
        for (int a = 0; a < 5; ++a) {
          int x = reflect101(2 * i + a - 2, sw);
          acc += (double)(kBinom[a] * kBinom[b]) * src[(size_t)y * sw + x];
        }
      }
      if (integer) {
        long s = (long)acc; /* exact: integer inputs, sum < 2^16 */
        dst[(size_t)j * dw + i] = (double)((s + 128) >> 8);
      } else {
        dst[(size_t)j * dw + i] = acc / 256.0;
      }
    }
}

/* ------------------------------------------------------------------------- */
/* O2: template gradient.  The Jacobian/Hessian of the inverse-compositional */
/* search live on the left patch and are computed once (Sec. III-A).          */
/* Reading: Sobel-x with reflect-101 borders, divided by 8 (intensity/px).    */
/* ------------------------------------------------------------------------- */
static void sobel_x(const double* img, int w, int h, double* g) {
  for (int y = 0; y < h; ++y) {
    int ym = reflect101(y - 1, h), yp = reflect101(y + 1, h);
    for (int x = 0; x < w; ++x) {
      int xm = reflect101(x - 1, w), xp = reflect101(x + 1, w);
      double gs = (img[(size_t)ym * w + xp] - img[(size_t)ym * w + xm]) +
                  2.0 * (img[(size_t)y * w + xp] - img[(size_t)y * w + xm]) +
                  (img[(size_t)yp * w + xp] - img[(size_t)yp * w + xm]);
      g[(size_t)y * w + x] = gs / 8.0;
    }
  }
}

/* Linear warp of one right-image row sample: position x + u, indices clamped
 * to the row (the bilinear warp of Eq. 1 with zero vertical weight). */
static double warp_sample(const double* row, int w, int x, double u) {
  double fm = floor(u);
  int m = (int)fm;
  double f = u - fm;
  double a = row[clampi(x + m, 0, w - 1)];
  double b = row[clampi(x + m + 1, 0, w - 1)];
  return (1.0 - f) * a + f * b;
}

/* Mean-normalised SSD between the left patch T and the right image warped
 * at displacement v (window term of Eq. 6, patch mean normalisation of
 * Sec. IV-A): sum_i ((I_i - mean I) - (T_i - mean T))^2, two passes. */
static double patch_ssd(const double* L, const double* R, int w, int ox, int oy, int P, double v) {
  int n = P * P;
  double sw = 0.0, st = 0.0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) {
      sw += warp_sample(R + (size_t)(oy + r) * w, w, ox + c, v);
      st += L[(size_t)(oy + r) * w + ox + c];
    }
  double mw = sw / n, mt = st / n, ssd = 0.0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) {
      double e = (warp_sample(R + (size_t)(oy + r) * w, w, ox + c, v) - mw) -
                 (L[(size_t)(oy + r) * w + ox + c] - mt);
      ssd += e * e;
    }
  return ssd;
}

/* ------------------------------------------------------------------------- */
/* O5-O8: one patch.                                                          */
/*  - Eq. 1 with the inverse-compositional roles (Sec. III-A): the residual   */
/*    is linearised on the left patch, J_i = g_i - mean(g) (mean-normalised   */
/*    template), H = sum J^2, and each of the K iterations (fixed, Sec. IV-A: */
/*    min = max iterations) takes u <- u - sum J_i (I_w,i - T_i) / H.         */
/*  - A final displacement further than P from the start is reset to the     */
/*    start (reading of the patch searching threshold, Sec. III-E).          */
/*  - Window SSDs at offsets -1, -1/2, 0, 1/2, 1 (Sec. IV-A, Eq. 5-6).        */
/*  - Accepted iff the centre has the smallest SSD (saddle / unconverged     */
/*    rejection, Sec. III-B and III-F) and the in-bounds fraction >= gamma.  */
/* ------------------------------------------------------------------------- */
static void search_patch(ref_level* lv, const bdis_ref_params* p, int k, int ox, int oy) {
  const int P = p->patch, w = lv->w, n = P * P;
  const double* L = lv->left;
  const double* R = lv->right;
  const double* G = lv->grad;
  double gbar = 0.0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) gbar += G[(size_t)(oy + r) * w + ox + c];
  gbar /= n;
  double H = 0.0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) {
      double J = G[(size_t)(oy + r) * w + ox + c] - gbar;
      H += J * J;
    }
  lv->hess[k] = H;
  const double u0 = lv->uinit[k];
  double u = u0;
  if (H >= EPS_H) {
    for (int t = 0; t < p->iters; ++t) {
      double bsum = 0.0;
      for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) {
          size_t idx = (size_t)(oy + r) * w + ox + c;
          double J = G[idx] - gbar;
          double Iw = warp_sample(R + (size_t)(oy + r) * w, w, ox + c, u);
          bsum += J * (Iw - L[idx]);
        }
      mix(&lv->dhash, (long long)floor(u));
      u = u - bsum / H;
    }
  }
  const int reset = fabs(u - u0) > (double)P;
  mix(&lv->dhash, reset);
  if (reset) u = u0;
  lv->u[k] = u;
  for (int d = 0; d < NWIN; ++d) mix(&lv->dhash, (long long)floor(u + kWinOffset[d]));

  for (int d = 0; d < NWIN; ++d) lv->ssd[(size_t)k * NWIN + d] = patch_ssd(L, R, w, ox, oy, P, u + kWinOffset[d]);

  int inb = 0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) {
      double xr = (double)(ox + c) + u;
      if (xr >= 0.0 && xr <= (double)(w - 1)) ++inb;
    }
  lv->rho[k] = (double)inb / (double)n;

  const double* s = lv->ssd + (size_t)k * NWIN;
  int centre_min = 1;
  for (int d = 0; d < NWIN; ++d)
    if (d != 2 && s[2] > s[d]) centre_min = 0;
  lv->acc[k] = (centre_min && lv->rho[k] >= p->valid_ratio) ? 1.0 : 0.0;
  mix(&lv->dhash, inb);
  mix(&lv->dhash, (long long)lv->acc[k]);
}

/* ------------------------------------------------------------------------- */
/* O11: spatial mixture mask (Eq. 9, all mixture weights 1, Sec. III-C).      */
/* M(a, b) = sum over patch pixels (c, d) of exp(-((a-c)^2+(b-d)^2)/(2 s^2)); */
/* the 1/(sigma sqrt(2 pi)) factor cancels in the normalised fusion.          */
/* ------------------------------------------------------------------------- */
int bdis_ref_mask(int P, double sigma_s, double* M) {
  if (P < 1 || !(sigma_s > 0.0) || !M) return BDIS_REF_E_ARG;
  for (int b = 0; b < P; ++b)
    for (int a = 0; a < P; ++a) {
      double acc = 0.0;
      for (int d = 0; d < P; ++d)
        for (int c = 0; c < P; ++c) {
          double dx = (double)(a - c), dy = (double)(b - d);
          acc += exp(-(dx * dx + dy * dy) / (2.0 * sigma_s * sigma_s));
        }
      M[b * P + a] = acc;
    }
  return BDIS_REF_OK;
}

/* ------------------------------------------------------------------------- */
/* O13: per-patch variance (Eq. 15-17).  The log objective of Eq. 17, read as */
/* least squares over the window, is linear in (ln c - ln(sqrt(2 pi) sigma),  */
/* -1/(2 sigma^2)), so its Gauss-Newton fixed point is the ordinary least-    */
/* squares line of ln p_delta = -SSD_delta / tau on delta^2:                  */
/* sigma^2 = tau / (2 kappa), kappa the OLS slope of SSD on delta^2.  A fit   */
/* fails (Sec. III-E) when kappa <= 0 or the mean squared residual in ln-p    */
/* units exceeds the threshold; failures and large values get sigma_fail^2.  */
/* ------------------------------------------------------------------------- */
static double patch_variance(const double* s, double tau, double thresh, double sfail2) {
  double x[NWIN], xm = 0.0, ym = 0.0;
  for (int d = 0; d < NWIN; ++d) {
    x[d] = kWinOffset[d] * kWinOffset[d];
    xm += x[d];
    ym += s[d];
  }
  xm /= NWIN;
  ym /= NWIN;
  double sxy = 0.0, sxx = 0.0;
  for (int d = 0; d < NWIN; ++d) {
    sxy += (x[d] - xm) * (s[d] - ym);
    sxx += (x[d] - xm) * (x[d] - xm);
  }
  double kappa = sxy / sxx;
  if (!(kappa > 0.0)) return sfail2;
  double mse = 0.0;
  for (int d = 0; d < NWIN; ++d) {
    double res = (s[d] - (ym + kappa * (x[d] - xm))) / tau;
    mse += res * res;
  }
  mse /= NWIN;
  if (mse > thresh) return sfail2;
  double v = tau / (2.0 * kappa);
  return v < sfail2 ? v : sfail2;
}

/* ------------------------------------------------------------------------- */
/* O4: start of every patch of a level below the coarsest.  Each patch starts  */
/* from the parent level's fused map at its centre (Fig. 1: initialised with  */
/* the prediction of the last level), scaled by 2 because a parent pixel      */
/* spans two pixels of this level (Sec. III-B); the probability propagated to */
/* the patch is the parent confidence at the same point.  Centre             */
/* c = origin + (P - 1) / 2 in this level's pixels, (c_x / 2, c_y / 2) in the  */
/* parent's, bilinear with indices clamped to the parent map.                 */
/* ------------------------------------------------------------------------- */
int bdis_ref_parent_init(const double* ubar, const double* qmap, int pw, int ph, int w, int h, int P, int S,
                         double* uinit, double* pipar) {
  if (!ubar || !qmap || !uinit || !pipar || pw < 1 || ph < 1 || P < 1 || S < 1 || w < P || h < P)
    return BDIS_REF_E_ARG;
  const int nx = grid_count(w, P, S), ny = grid_count(h, P, S);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int k = j * nx + i;
      const double cx = grid_origin(i, w, P, S) + 0.5 * (P - 1);
      const double cy = grid_origin(j, h, P, S) + 0.5 * (P - 1);
      uinit[k] = 2.0 * bilinear(ubar, pw, ph, 0.5 * cx, 0.5 * cy);
      pipar[k] = bilinear(qmap, pw, ph, 0.5 * cx, 0.5 * cy);
    }
  return BDIS_REF_OK;
}

/* ------------------------------------------------------------------------- */
/* driver                                                                    */
/* ------------------------------------------------------------------------- */

static void free_level(ref_level* lv) {
  double** ptrs[] = {&lv->left, &lv->right, &lv->grad, &lv->uinit, &lv->pipar, &lv->u,
                     &lv->ssd,  &lv->rho,   &lv->acc,  &lv->post,  &lv->pi,    &lv->sigk2,
                     &lv->hess, &lv->ubar,  &lv->qmap, &lv->valid, &lv->odisp, &lv->ovar,
                     &lv->oconf, &lv->fv,   &lv->vbar, &lv->gy};
  for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) {
    free(*ptrs[i]);
    *ptrs[i] = NULL;
  }
}

void bdis_ref_trace_free(bdis_ref_trace* t) {
  if (!t) return;
  for (int n = 0; n < MAX_LEVELS; ++n) free_level(&t->lv[n]);
  free(t);
}

static int alloc_level(ref_level* lv, int w, int h, int P, int S) {
  size_t npx = (size_t)w * h;
  lv->w = w;
  lv->h = h;
  lv->dhash = 1469598103934665603ULL;
  lv->nx = grid_count(w, P, S);
  lv->ny = grid_count(h, P, S);
  size_t np = (size_t)lv->nx * lv->ny;
  lv->left = calloc(npx, sizeof(double));
  lv->right = calloc(npx, sizeof(double));
  lv->grad = calloc(npx, sizeof(double));
  lv->ubar = calloc(npx, sizeof(double));
  lv->qmap = calloc(npx, sizeof(double));
  lv->valid = calloc(npx, sizeof(double));
  lv->uinit = calloc(np, sizeof(double));
  lv->pipar = calloc(np, sizeof(double));
  lv->u = calloc(np, sizeof(double));
  lv->ssd = calloc(np * NWIN, sizeof(double));
  lv->rho = calloc(np, sizeof(double));
  lv->acc = calloc(np, sizeof(double));
  lv->post = calloc(np, sizeof(double));
  lv->pi = calloc(np, sizeof(double));
  lv->sigk2 = calloc(np, sizeof(double));
  lv->hess = calloc(np, sizeof(double));
  return (lv->left && lv->right && lv->grad && lv->ubar && lv->qmap && lv->valid && lv->uinit &&
          lv->pipar && lv->u && lv->ssd && lv->rho && lv->acc && lv->post && lv->pi &&
          lv->sigk2 && lv->hess)
             ? 0
             : -1;
}

static int check_params(const bdis_ref_params* p, int w, int h, int pitch) {
  if (!p) return BDIS_REF_E_ARG;
  if (p->levels < 1 || p->levels > MAX_LEVELS) return BDIS_REF_E_ARG;
  if (p->finest_level < 0 || p->finest_level >= p->levels) return BDIS_REF_E_ARG;
  if (p->patch < 3 || p->stride < 1 || p->stride > p->patch || p->iters < 1) return BDIS_REF_E_ARG;
  if (p->fusion < 0 || p->fusion > 2 || (p->propagate != 0 && p->propagate != 1)) return BDIS_REF_E_ARG;
  if (!(p->sigma_s > 0.0) || !(p->sigma_r > 0.0)) return BDIS_REF_E_ARG;
  if (!(p->valid_ratio > 0.0) || p->valid_ratio > 1.0) return BDIS_REF_E_ARG; /* gamma is a fraction of the patch */
  if (w < 1 || h < 1 || pitch < w) return BDIS_REF_E_ARG;
  double wsum = 0.0;
  for (int n = p->finest_level; n < p->levels; ++n) {
    if (!(p->level_weight[n] >= 0.0)) return BDIS_REF_E_ARG;
    wsum += p->level_weight[n];
  }
  if (!(wsum > 0.0)) return BDIS_REF_E_ARG;
  int lw = w, lh = h;
  for (int n = 0; n < p->levels; ++n) {
    if (n >= p->finest_level && (lw < p->patch || lh < p->patch)) return BDIS_REF_E_SIZE;
    lw = (lw + 1) >> 1;
    lh = (lh + 1) >> 1;
  }
  return BDIS_REF_OK;
}

/* Weight of patch k at pixel (x, y) in the fusion.  Eq. 13: mask x patch
 * probability (fusion 0; fusion 2 passes a uniform mask).  Eq. 2 (DIS, fusion
 * 1): the inverse squared photometric residual of the pixel under the patch's
 * displacement, r = I_r(x + u) - I_l(x), floored at 1 as in DIS so that an
 * exact match does not divide by zero (reading). */
static double fusion_weight(int fusion, double m, double pi, const ref_level* lv, int x, int y,
                            double u) {
  if (fusion != 1) return m * pi;
  double r = warp_sample(lv->right + (size_t)y * lv->w, lv->w, x, u) - lv->left[(size_t)y * lv->w + x];
  double r2 = r * r;
  return 1.0 / (r2 > 1.0 ? r2 : 1.0);
}

/* Finest level f > 0 (Sec. IV-A runs levels 5..1): the full-resolution
 * outputs sample the level-f maps bilinearly at (x / 2^f, y / 2^f) -- the
 * pyramid keeps the even pixels, so level-0 pixel 2^f k lies on level-f pixel
 * k -- clamped at the last row and column; disparity is scaled by 2^f (level-f
 * pixels to full-resolution pixels) and variance by 4^f.  A pixel is invalid
 * (NaN, NaN, confidence 0) when any sample it gives a nonzero weight is. */
static void upsample(const ref_level* lf, int f, int w, int h, int variance, double* disp,
                     double* var, double* conf) {
  const double sc = (double)(1 << f);
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      double sx = x / sc, sy = y / sc;
      int x0 = (int)floor(sx), y0 = (int)floor(sy);
      double ax = sx - x0, ay = sy - y0;
      int xs[2] = {x0, x0 + 1 < lf->w ? x0 + 1 : lf->w - 1};
      int ys[2] = {y0, y0 + 1 < lf->h ? y0 + 1 : lf->h - 1};
      double wx[2] = {1.0 - ax, ax}, wy[2] = {1.0 - ay, ay};
      double d = 0.0, v = 0.0, c = 0.0;
      int ok = 1;
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          double wt = wx[a] * wy[b];
          if (wt == 0.0) continue;
          size_t k = (size_t)ys[b] * lf->w + xs[a];
          if (isnan(lf->odisp[k])) ok = 0;
          d += wt * lf->odisp[k];
          v += wt * lf->ovar[k];
          c += wt * lf->oconf[k];
        }
      size_t o = (size_t)y * w + x;
      disp[o] = ok ? sc * d : NAN;
      if (var) var[o] = (ok && variance) ? sc * sc * v : NAN;
      if (conf) conf[o] = ok ? c : 0.0;
    }
}

int bdis_ref_coverage(const double* disp, const double* var, const double* ref, const uint8_t* valid,
                      long n, double k, long* covered, long* total) {
  if (!disp || !var || !ref || !covered || !total || n < 0 || !(k >= 0.0)) return BDIS_REF_E_ARG;
  long c = 0, t = 0;
  for (long i = 0; i < n; ++i) {
    if (valid && !valid[i]) continue;
    if (!isfinite(disp[i]) || !isfinite(var[i]) || !isfinite(ref[i]) || var[i] < 0.0) continue;
    ++t;
    if (fabs(disp[i] - ref[i]) <= k * sqrt(var[i])) ++c;
  }
  *covered = c;
  *total = t;
  return BDIS_REF_OK;
}

int bdis_ref_depth(const double* disp, const double* var, long n, double fb, double* depth,
                   double* depth_var) {
  if (!disp || !depth || n < 0 || !(fb > 0.0)) return BDIS_REF_E_ARG;
  for (long i = 0; i < n; ++i) {
    double d = disp[i];
    int ok = d > 0.0; /* NaN compares false */
    depth[i] = ok ? fb / d : NAN;
    if (depth_var) depth_var[i] = (ok && var) ? fb * fb / (d * d * d * d) * var[i] : NAN;
  }
  return BDIS_REF_OK;
}

static int run(const bdis_ref_params* p, const double* left0, const double* right0, int w, int h,
               int integer, double* disp, double* var, double* conf, bdis_ref_trace** trace_out) {
  const int L = p->levels, f = p->finest_level, P = p->patch, S = p->stride;
  bdis_ref_trace* t = calloc(1, sizeof(*t));
  if (!t) return BDIS_REF_E_NOMEM;
  t->levels = L;

  /* Pyramid (O1) and template gradients (O2). */
  int lw = w, lh = h;
  for (int n = 0; n < L; ++n) {
    if (alloc_level(&t->lv[n], lw, lh, P, S)) {
      bdis_ref_trace_free(t);
      return BDIS_REF_E_NOMEM;
    }
    lw = (lw + 1) >> 1;
    lh = (lh + 1) >> 1;
  }
  memcpy(t->lv[0].left, left0, sizeof(double) * (size_t)w * h);
  memcpy(t->lv[0].right, right0, sizeof(double) * (size_t)w * h);
  for (int n = 1; n < L; ++n) {
    ref_level* a = &t->lv[n - 1];
    ref_level* b = &t->lv[n];
    pyramid_down(a->left, a->w, a->h, b->left, b->w, b->h, integer);
    pyramid_down(a->right, a->w, a->h, b->right, b->w, b->h, integer);
  }
  for (int n = 0; n < L; ++n) sobel_x(t->lv[n].left, t->lv[n].w, t->lv[n].h, t->lv[n].grad);

  /* Level weights Gamma_n = omega_n / sum omega (Eq. 12). */
  double wsum = 0.0;
  for (int n = f; n < L; ++n) wsum += p->level_weight[n];

  double* M = malloc(sizeof(double) * (size_t)P * P);
  if (!M) {
    bdis_ref_trace_free(t);
    return BDIS_REF_E_NOMEM;
  }
  bdis_ref_mask(P, p->sigma_s, M);
  /* Outputs of the finest level: the caller's arrays when f = 0, else level-f
   * maps that are upsampled at the end. */
  double *odisp = disp, *ovar = var, *oconf = conf;
  if (f > 0) {
    ref_level* lf = &t->lv[f];
    size_t nf = (size_t)lf->w * lf->h;
    lf->odisp = calloc(nf, sizeof(double));
    lf->ovar = calloc(nf, sizeof(double));
    lf->oconf = calloc(nf, sizeof(double));
    if (!lf->odisp || !lf->ovar || !lf->oconf) {
      free(M);
      bdis_ref_trace_free(t);
      return BDIS_REF_E_NOMEM;
    }
    odisp = lf->odisp;
    ovar = lf->ovar;
    oconf = lf->oconf;
  }
  const double sfail = p->var_fail_sigma > 0.0 ? p->var_fail_sigma : (double)P;
  const double sfail2 = sfail * sfail;

  for (int n = L - 1; n >= f; --n) {
    ref_level* lv = &t->lv[n];
    const ref_level* par = (n + 1 < L) ? &t->lv[n + 1] : NULL;
    const int np = lv->nx * lv->ny;

    /* O4 */
    if (par)
      bdis_ref_parent_init(par->ubar, par->qmap, par->w, par->h, lv->w, lv->h, P, S, lv->uinit, lv->pipar);
    else
      for (int k = 0; k < np; ++k) lv->uinit[k] = lv->pipar[k] = 0.0;

    /* O5-O8 */
    for (int j = 0; j < lv->ny; ++j)
      for (int i = 0; i < lv->nx; ++i)
        search_patch(lv, p, j * lv->nx + i, grid_origin(i, lv->w, P, S), grid_origin(j, lv->h, P, S));

    /* O9: sigma_r^(n), the spread of the converged residuals of the level
     * (Sec. III-B).  Reading: pooled per-pixel variance of the mean-normalised
     * residual over accepted patches, scaled by alpha_r^2 and floored. */
    double ssum = 0.0;
    long nacc = 0;
    for (int k = 0; k < np; ++k)
      if (lv->acc[k] != 0.0) {
        ssum += lv->ssd[(size_t)k * NWIN + 2];
        ++nacc;
      }
    double sr2;
    if (p->sigma_r_dynamic) {
      double pooled = nacc > 0 ? ssum / ((double)nacc * P * P) : 0.0;
      sr2 = p->sigma_r * p->sigma_r * (pooled > EPS_SIGMA ? pooled : EPS_SIGMA);
    } else {
      sr2 = p->sigma_r * p->sigma_r;
    }
    const double tau = 2.0 * sr2 * (double)(NWIN * NWIN); /* Eq. 6: 2 sigma_r^2 s^2 */
    const double gamma = p->level_weight[n] / wsum;
    lv->sigma_r2 = sr2;
    lv->tau = tau;
    lv->nacc = (double)nacc;
    lv->gamma = gamma;

    /* O10: window posterior p0 / sum_delta p_delta (Eq. 5-6, ratio r taken as
     * 1), and the level contribution plus the propagated parent probability
     * (Eq. 11-12). */
    for (int k = 0; k < np; ++k) {
      if (lv->acc[k] == 0.0) {
        lv->post[k] = 0.0;
        lv->pi[k] = 0.0;
        lv->sigk2[k] = NAN;
        continue;
      }
      const double* s = lv->ssd + (size_t)k * NWIN;
      double den = 0.0;
      for (int d = 0; d < NWIN; ++d) den += exp(-(s[d] - s[2]) / tau);
      lv->post[k] = 1.0 / den;
      /* Eq. 11; with propagation off (ablation) only the level term remains */
      lv->pi[k] = gamma * lv->post[k] + (p->propagate ? lv->pipar[k] : 0.0);
      lv->sigk2[k] = (n == f && p->variance) ? patch_variance(s, tau, p->var_fit_thresh, sfail2) : NAN;
      mix(&lv->dhash, lv->sigk2[k] == sfail2);
    }

    /* O12 / O14: fusion of the covering patches (Eq. 9, 10, 13, 18). */
    for (int y = 0; y < lv->h; ++y)
      for (int x = 0; x < lv->w; ++x) {
        double z = 0.0, zu = 0.0, zm = 0.0, zq = 0.0, zv = 0.0;
        for (int j = 0; j < lv->ny; ++j) {
          int oy = grid_origin(j, lv->h, P, S);
          if (oy > y) break;
          if (oy + P <= y) continue;
          for (int i = 0; i < lv->nx; ++i) {
            int ox = grid_origin(i, lv->w, P, S);
            if (ox > x) break;
            if (ox + P <= x) continue;
            int k = j * lv->nx + i;
            if (lv->acc[k] == 0.0) continue;
            double m = p->fusion == 2 ? 1.0 : M[(y - oy) * P + (x - ox)];
            double wk = fusion_weight(p->fusion, m, lv->pi[k], lv, x, y, lv->u[k]);
            z += wk;
            zu += wk * lv->u[k];
            zm += m;
            zq += m * lv->pi[k];
          }
        }
        size_t idx = (size_t)y * lv->w + x;
        mix(&lv->dhash, z > 0.0);
        if (z > 0.0) {
          lv->ubar[idx] = zu / z;
          lv->qmap[idx] = zq / zm;
          lv->valid[idx] = 1.0;
          if (n == f && p->variance) {
            /* second pass for the normalised weights of Eq. 18 */
            for (int j = 0; j < lv->ny; ++j) {
              int oy = grid_origin(j, lv->h, P, S);
              if (oy > y) break;
              if (oy + P <= y) continue;
              for (int i = 0; i < lv->nx; ++i) {
                int ox = grid_origin(i, lv->w, P, S);
                if (ox > x) break;
                if (ox + P <= x) continue;
                int k = j * lv->nx + i;
                if (lv->acc[k] == 0.0) continue;
                double m = p->fusion == 2 ? 1.0 : M[(y - oy) * P + (x - ox)];
                double wn = fusion_weight(p->fusion, m, lv->pi[k], lv, x, y, lv->u[k]) / z;
                zv += wn * wn * lv->sigk2[k];
              }
            }
          }
        } else if (n == f) {
          lv->ubar[idx] = NAN;
          lv->qmap[idx] = 0.0;
          lv->valid[idx] = 0.0;
        } else if (par) {
          /* hole: take the parent estimate (reading; the paper is silent) */
          lv->ubar[idx] = 2.0 * bilinear(par->ubar, par->w, par->h, 0.5 * x, 0.5 * y);
          lv->qmap[idx] = bilinear(par->qmap, par->w, par->h, 0.5 * x, 0.5 * y);
          lv->valid[idx] = 0.0;
        } else {
          lv->ubar[idx] = 0.0;
          lv->qmap[idx] = 0.0;
          lv->valid[idx] = 0.0;
        }
        if (n == f) {
          int ok = lv->valid[idx] != 0.0 &&
                   !(p->prob_thresh > 0.0 && lv->qmap[idx] < p->prob_thresh);
          /* Eq. 13 gives u on the right image; disparity d = x_l - x_r = -u */
          odisp[idx] = ok ? -lv->ubar[idx] : NAN;
          if (oconf) oconf[idx] = ok ? lv->qmap[idx] : 0.0;
          if (ovar) ovar[idx] = (ok && p->variance) ? zv : NAN;
        }
      }
  }
  free(M);
  if (f > 0) upsample(&t->lv[f], f, w, h, p->variance, disp, var, conf);
  if (trace_out)
    *trace_out = t;
  else
    bdis_ref_trace_free(t);
  return BDIS_REF_OK;
}

int bdis_ref_compute_u8(const bdis_ref_params* p, const uint8_t* left, const uint8_t* right, int w,
                        int h, int pitch, double* disp, double* var, double* conf,
                        bdis_ref_trace** trace) {
  if (trace) *trace = NULL;
  if (!left || !right || !disp) return BDIS_REF_E_ARG;
  int st = check_params(p, w, h, pitch);
  if (st) return st;
  double* l = malloc(sizeof(double) * (size_t)w * h);
  double* r = malloc(sizeof(double) * (size_t)w * h);
  if (!l || !r) {
    free(l);
    free(r);
    return BDIS_REF_E_NOMEM;
  }
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      l[(size_t)y * w + x] = (double)left[(size_t)y * pitch + x];
      r[(size_t)y * w + x] = (double)right[(size_t)y * pitch + x];
    }
  st = run(p, l, r, w, h, 1, disp, var, conf, trace);
  free(l);
  free(r);
  return st;
}

int bdis_ref_compute_f64(const bdis_ref_params* p, const double* left, const double* right, int w,
                         int h, int pitch, double* disp, double* var, double* conf,
                         bdis_ref_trace** trace) {
  if (trace) *trace = NULL;
  if (!left || !right || !disp) return BDIS_REF_E_ARG;
  int st = check_params(p, w, h, pitch);
  if (st) return st;
  double* l = malloc(sizeof(double) * (size_t)w * h);
  double* r = malloc(sizeof(double) * (size_t)w * h);
  if (!l || !r) {
    free(l);
    free(r);
    return BDIS_REF_E_NOMEM;
  }
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      double a = left[(size_t)y * pitch + x], b = right[(size_t)y * pitch + x];
      if (!isfinite(a) || !isfinite(b)) {
        free(l);
        free(r);
        return BDIS_REF_E_ARG;
      }
      l[(size_t)y * w + x] = a;
      r[(size_t)y * w + x] = b;
    }
  st = run(p, l, r, w, h, 0, disp, var, conf, trace);
  free(l);
  free(r);
  return st;
}

/* ------------------------------------------------------------------------- */
/* Optical flow (2-D dense inverse search).  Eq. 1 with u a 2-vector: the     */
/* inverse-compositional update of DIS on a 2 x 2 Hessian, the template       */
/* gradients Sobel-x / 8 and Sobel-y / 8 (reflect-101), the warp bilinear in  */
/* both axes with indices clamped to the image, and the fusion of Eq. 2.      */
/* ------------------------------------------------------------------------- */
static void sobel_y(const double* img, int w, int h, double* g) {
  for (int y = 0; y < h; ++y) {
    int ym = reflect101(y - 1, h), yp = reflect101(y + 1, h);
    for (int x = 0; x < w; ++x) {
      int xm = reflect101(x - 1, w), xp = reflect101(x + 1, w);
      double gs = (img[(size_t)yp * w + xm] - img[(size_t)ym * w + xm]) +
                  2.0 * (img[(size_t)yp * w + x] - img[(size_t)ym * w + x]) +
                  (img[(size_t)yp * w + xp] - img[(size_t)ym * w + xp]);
      g[(size_t)y * w + x] = gs / 8.0;
    }
  }
}

/* One patch: J = (gx - mean gx, gy - mean gy) over the patch, H = sum J J^T;
 * K iterations of (u, v) <- (u, v) - H^-1 sum J (I1(x + u, y + v) - T); no update
 * when det H < EPS_H (reading: the 1-D floor applied to the determinant);
 * reset to the start when the step from it exceeds P in Euclidean length. */
static void flow_patch(ref_level* lv, const bdis_ref_params* p, int k, int ox, int oy, double u0, double v0) {
  const int P = p->patch, w = lv->w, h = lv->h, n = P * P;
  const double *I0 = lv->left, *I1 = lv->right, *GX = lv->grad, *GY = lv->gy;
  double mx = 0.0, my = 0.0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) {
      mx += GX[(size_t)(oy + r) * w + ox + c];
      my += GY[(size_t)(oy + r) * w + ox + c];
    }
  mx /= n;
  my /= n;
  double hxx = 0.0, hxy = 0.0, hyy = 0.0;
  for (int r = 0; r < P; ++r)
    for (int c = 0; c < P; ++c) {
      double jx = GX[(size_t)(oy + r) * w + ox + c] - mx, jy = GY[(size_t)(oy + r) * w + ox + c] - my;
      hxx += jx * jx;
      hxy += jx * jy;
      hyy += jy * jy;
    }
  const double det = hxx * hyy - hxy * hxy;
  lv->hess[k] = det;
  double u = u0, v = v0;
  if (det >= EPS_H) {
    for (int t = 0; t < p->iters; ++t) {
      double bx = 0.0, by = 0.0;
      for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) {
          size_t idx = (size_t)(oy + r) * w + ox + c;
          double e = bilinear(I1, w, h, ox + c + u, oy + r + v) - I0[idx];
          bx += (GX[idx] - mx) * e;
          by += (GY[idx] - my) * e;
        }
      mix(&lv->dhash, (long long)floor(u));
      mix(&lv->dhash, (long long)floor(v));
      /* H^-1 b by the 2 x 2 adjugate */
      u -= (hyy * bx - hxy * by) / det;
      v -= (hxx * by - hxy * bx) / det;
    }
  }
  const int reset = (u - u0) * (u - u0) + (v - v0) * (v - v0) > (double)P * (double)P;
  mix(&lv->dhash, reset);
  if (reset) {
    u = u0;
    v = v0;
  }
  lv->uinit[k] = u0;
  lv->u[k] = u;
  lv->fv[k] = v;
  lv->acc[k] = 1.0;
}

int bdis_ref_flow(const bdis_ref_params* p, const uint8_t* i0, const uint8_t* i1, int w, int h, int pitch,
                  double* flow_u, double* flow_v, bdis_ref_trace** trace_out) {
  if (trace_out) *trace_out = NULL;
  if (!i0 || !i1 || !flow_u || !flow_v) return BDIS_REF_E_ARG;
  int st = check_params(p, w, h, pitch);
  if (st) return st;
  if (p->finest_level != 0) return BDIS_REF_E_ARG;
  const int L = p->levels, P = p->patch, S = p->stride;
  bdis_ref_trace* t = calloc(1, sizeof(*t));
  if (!t) return BDIS_REF_E_NOMEM;
  t->levels = L;
  int lw = w, lh = h;
  for (int n = 0; n < L; ++n) {
    ref_level* lv = &t->lv[n];
    int bad = alloc_level(lv, lw, lh, P, S);
    size_t np = (size_t)lv->nx * lv->ny, npx = (size_t)lw * lh;
    lv->fv = calloc(np, sizeof(double));
    lv->vbar = calloc(npx, sizeof(double));
    lv->gy = calloc(npx, sizeof(double));
    if (bad || !lv->fv || !lv->vbar || !lv->gy) {
      bdis_ref_trace_free(t);
      return BDIS_REF_E_NOMEM;
    }
    lw = (lw + 1) >> 1;
    lh = (lh + 1) >> 1;
  }
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < w; ++x) {
      t->lv[0].left[(size_t)y * w + x] = (double)i0[(size_t)y * pitch + x];
      t->lv[0].right[(size_t)y * w + x] = (double)i1[(size_t)y * pitch + x];
    }
  for (int n = 1; n < L; ++n) {
    ref_level *a = &t->lv[n - 1], *b = &t->lv[n];
    pyramid_down(a->left, a->w, a->h, b->left, b->w, b->h, 1);
    pyramid_down(a->right, a->w, a->h, b->right, b->w, b->h, 1);
  }
  for (int n = L - 1; n >= 0; --n) {
    ref_level* lv = &t->lv[n];
    const ref_level* par = n + 1 < L ? &t->lv[n + 1] : NULL;
    sobel_x(lv->left, lv->w, lv->h, lv->grad);
    sobel_y(lv->left, lv->w, lv->h, lv->gy);
    for (int j = 0; j < lv->ny; ++j)
      for (int i = 0; i < lv->nx; ++i) {
        const int ox = grid_origin(i, lv->w, P, S), oy = grid_origin(j, lv->h, P, S);
        double u0 = 0.0, v0 = 0.0;
        if (par) { /* the parent's fused flow at the patch centre, in this level's pixels */
          const double cx = ox + 0.5 * (P - 1), cy = oy + 0.5 * (P - 1);
          u0 = 2.0 * bilinear(par->ubar, par->w, par->h, 0.5 * cx, 0.5 * cy);
          v0 = 2.0 * bilinear(par->vbar, par->w, par->h, 0.5 * cx, 0.5 * cy);
        }
        flow_patch(lv, p, j * lv->nx + i, ox, oy, u0, v0);
      }
    /* Eq. 2 fusion: weight 1 / max(1, r^2), r = I1(x + u_k) - I0(x) */
    for (int y = 0; y < lv->h; ++y)
      for (int x = 0; x < lv->w; ++x) {
        double z = 0.0, zu = 0.0, zv = 0.0;
        for (int j = 0; j < lv->ny; ++j) {
          int oy = grid_origin(j, lv->h, P, S);
          if (oy > y) break;
          if (oy + P <= y) continue;
          for (int i = 0; i < lv->nx; ++i) {
            int ox = grid_origin(i, lv->w, P, S);
            if (ox > x) break;
            if (ox + P <= x) continue;
            int k = j * lv->nx + i;
            double r = bilinear(lv->right, lv->w, lv->h, x + lv->u[k], y + lv->fv[k]) -
                       lv->left[(size_t)y * lv->w + x];
            double wk = 1.0 / (r * r > 1.0 ? r * r : 1.0);
            z += wk;
            zu += wk * lv->u[k];
            zv += wk * lv->fv[k];
          }
        }
        size_t idx = (size_t)y * lv->w + x;
        lv->ubar[idx] = zu / z; /* every pixel is covered: z > 0 */
        lv->vbar[idx] = zv / z;
        if (n == 0) {
          flow_u[idx] = lv->ubar[idx];
          flow_v[idx] = lv->vbar[idx];
        }
      }
  }
  if (trace_out)
    *trace_out = t;
  else
    bdis_ref_trace_free(t);
  return BDIS_REF_OK;
}

/* Patch-grid origins along an axis of length n; returns the count (or < 0). */
int bdis_ref_grid(int n, int P, int S, int* origins, int cap) {
  if (P < 1 || S < 1 || n < P) return BDIS_REF_E_ARG;
  int cnt = grid_count(n, P, S);
  if (origins) {
    if (cap < cnt) return BDIS_REF_E_ARG;
    for (int i = 0; i < cnt; ++i) origins[i] = grid_origin(i, n, P, S);
  }
  return cnt;
}

/* ------------------------------------------------------------------------- */
/* trace access                                                              */
/* ------------------------------------------------------------------------- */

int bdis_ref_trace_dims(const bdis_ref_trace* t, int level, int* w, int* h, int* nx, int* ny) {
  if (!t || level < 0 || level >= t->levels) return BDIS_REF_E_ARG;
  const ref_level* lv = &t->lv[level];
  if (w) *w = lv->w;
  if (h) *h = lv->h;
  if (nx) *nx = lv->nx;
  if (ny) *ny = lv->ny;
  return BDIS_REF_OK;
}

long bdis_ref_trace_get(const bdis_ref_trace* t, int level, int what, double* dst, long n) {
  if (!t || level < 0 || level >= t->levels || !dst) return BDIS_REF_E_ARG;
  const ref_level* lv = &t->lv[level];
  long npx = (long)lv->w * lv->h, np = (long)lv->nx * lv->ny;
  const double* src = NULL;
  long cnt = 0;
  switch (what) {
    case BDIS_REF_LEFT: src = lv->left; cnt = npx; break;
    case BDIS_REF_RIGHT: src = lv->right; cnt = npx; break;
    case BDIS_REF_GRAD: src = lv->grad; cnt = npx; break;
    case BDIS_REF_UINIT: src = lv->uinit; cnt = np; break;
    case BDIS_REF_PIPAR: src = lv->pipar; cnt = np; break;
    case BDIS_REF_U: src = lv->u; cnt = np; break;
    case BDIS_REF_SSD: src = lv->ssd; cnt = np * NWIN; break;
    case BDIS_REF_RHO: src = lv->rho; cnt = np; break;
    case BDIS_REF_ACC: src = lv->acc; cnt = np; break;
    case BDIS_REF_POST: src = lv->post; cnt = np; break;
    case BDIS_REF_PI: src = lv->pi; cnt = np; break;
    case BDIS_REF_SIGK2: src = lv->sigk2; cnt = np; break;
    case BDIS_REF_HESS: src = lv->hess; cnt = np; break;
    case BDIS_REF_UBAR: src = lv->ubar; cnt = npx; break;
    case BDIS_REF_QMAP: src = lv->qmap; cnt = npx; break;
    case BDIS_REF_VALID: src = lv->valid; cnt = npx; break;
    case BDIS_REF_ODISP: src = lv->odisp; cnt = npx; break;
    case BDIS_REF_OVAR: src = lv->ovar; cnt = npx; break;
    case BDIS_REF_OCONF: src = lv->oconf; cnt = npx; break;
    case BDIS_REF_FV: src = lv->fv; cnt = np; break;
    case BDIS_REF_VBAR: src = lv->vbar; cnt = npx; break;
    case BDIS_REF_GY: src = lv->gy; cnt = npx; break;
    default: return BDIS_REF_E_ARG;
  }
  if (!src || n < cnt) return BDIS_REF_E_ARG;
  memcpy(dst, src, sizeof(double) * (size_t)cnt);
  return cnt;
}

uint64_t bdis_ref_trace_hash(const bdis_ref_trace* t, int level) {
  if (!t || level < 0 || level >= t->levels) return 0;
  return t->lv[level].dhash;
}

double bdis_ref_trace_scalar(const bdis_ref_trace* t, int level, int what) {
  if (!t || level < 0 || level >= t->levels) return NAN;
  const ref_level* lv = &t->lv[level];
  switch (what) {
    case BDIS_REF_SIGMA_R2: return lv->sigma_r2;
    case BDIS_REF_TAU: return lv->tau;
    case BDIS_REF_NACC: return lv->nacc;
    case BDIS_REF_GAMMA: return lv->gamma;
    default: return NAN;
  }
}
