// Device helpers of the fusion: the patch record of Eq. 5-6, 11-12 and 15-17,
// and the mask-weighted sums of Eq. 9-13 that every tile shape of the fusion
// goes through, so a fused value is the same bits whatever the tile.
#pragma once

#include "bdis_internal.h"

namespace bdis {

// The search results of patch k that its fusion record needs.
struct PatchRaw {
  double u, pipar;
  D4 d;  // window SSD differences
  int acc;
};
BDIS_DEV PatchRaw patch_raw(const PairLevel& a, const LevelParams& lp, size_t k) {
  PatchRaw p;
  p.u = gbl(a.pa.u)[k];
  p.acc = gbl(a.pa.acc)[k];
  p.d = ld4(a.pa.dssd + k);
  p.pipar = lp.propagate ? gbl(a.pa.pipar)[k] : 0.0;
  return p;
}

// 1 / x to within about one unit in the last place: the hardware estimate
// refined by two Newton steps, e <- 1 - x r, r <- r + r e (each step squares
// the relative error), for x in [2^-1000, 2^1000]; the correctly rounded
// division elsewhere (zero, huge, subnormal, NaN).  About half the FP64
// instructions of the division; used wherever a result is normalised, by
// every kernel that computes that result, so the kernels agree bit for bit.
BDIS_DEV double recip(double x) {
  if (__builtin_expect(!(fabs(x) >= 0x1p-1000 && fabs(x) <= 0x1p1000), 0)) return 1.0 / x;
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// The variance fit of a patch record (Eq. 15-17): kappa, the least-squares
// slope of SSD_d - SSD_0 on x_d = d^2 (x = 1, 1/4, 0, 1/4, 1; mean x = 1/2,
// sum (x - mean x)^2 = 7/8), and whether it passes: kappa > 0 and the mean
// squared residual of the line, in units of tau (rt = 1 / tau), within the
// threshold.  No contraction; the record and its adjoint both decide here, so
// they take the same decision.
struct VarFit {
  double kappa;
  bool pass;
};
BDIS_DEV VarFit var_fit(const D4& d, double rt, float thresh) {
#pragma clang fp contract(off)
  const double y[5] = {d.x, d.y, 0.0, d.z, d.w};
  const double x[5] = {1.0, 0.25, 0.0, 0.25, 1.0};
  const double ym = (y[0] + y[1] + y[2] + y[3] + y[4]) * 0.2;
  double sxy = 0.0;
  for (int t = 0; t < 5; ++t) sxy += (x[t] - 0.5) * y[t];
  const double kappa = sxy * (8.0 / 7.0);
  bool pass = false;
  if (kappa > 0.0) {
    double mse = 0.0;
    for (int t = 0; t < 5; ++t) {
      const double res = (y[t] - (ym + kappa * (x[t] - 0.5))) * rt;
      mse += res * res;
    }
    mse *= 0.2;
    pass = mse <= (double)thresh;
  }
  return VarFit{kappa, pass};
}

// The fusion record of patch p of pyramid level `level`: (u, pi or -1 when
// rejected, sigma_k^2 at the finest level with variance on, else NaN, post).
// No floating-point contraction, so every kernel that inlines it gets the
// same bits.  Divisions by tau and by the constants of the fit are taken as
// products with their reciprocals.
BDIS_DEV D4 patch_record(const PairLevel& a, const LevelParams& lp, int level, const PatchRaw& p, double tau) {
#pragma clang fp contract(off)
  const double u = p.u;
  const double nan = __builtin_nan("");
  if (!p.acc) return D4{u, -1.0, nan, 0.0};
  const D4 d = p.d;
  const double rt = 1.0 / tau;
  const double den = 1.0 + exp(-d.x * rt) + exp(-d.y * rt) + exp(-d.z * rt) + exp(-d.w * rt);
  const double post = recip(den);
  double wsum = 0.0;
  for (int n = lp.finest; n < a.levels; ++n) wsum += (double)lp.omega[n];
  const double gamma = (double)lp.omega[level] / wsum;
  const double pi = gamma * post + p.pipar;
  double sig = nan;
  if (lp.variance && level == lp.finest) {
    const double sfail = lp.var_fail_sigma > 0.0f ? (double)lp.var_fail_sigma : (double)lp.P;
    double v = sfail * sfail;
    const VarFit vf = var_fit(d, rt, lp.var_fit_thresh);
    if (vf.pass) {
      const double s2 = tau / (2.0 * vf.kappa);
      v = s2 < v ? s2 : v;
    }
    sig = v;
  }
  return D4{u, pi, sig, post};
}

// Mask-weighted sums of one covering patch row at one pixel column, and their
// combination over the patch rows (the mask factors into m(x - o_x) m(y - o_y)):
//   A0 = sum_i m_x pi, A1 = sum_i m_x pi u, A2 = sum_i m_x, A3 = sum_i (m_x pi)^2 sigma^2,
//   z = sum_j m_y A0, zu = sum_j m_y A1, zm = sum_j m_y A2, zv = sum_j m_y^2 A3.
// The staged separable form and the direct per-pixel form both go through
// these two helpers (explicit FMAs, no other contraction, patches in ascending
// index), so the fused maps are the same bits whatever the tile shape and
// whichever kernel inlines them.
struct ColSums {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
};
BDIS_DEV void col_add(ColSums& c, double mx, double pi, double u, double sig) {
#pragma clang fp contract(off)
  const double wx = mx * pi;
  c.a0 += wx;
  c.a1 = fma(wx, u, c.a1);
  c.a2 += mx;
  c.a3 = fma(wx * wx, sig, c.a3);
}
struct PixSums {
  double z = 0.0, zu = 0.0, zm = 0.0, zv = 0.0;
};
BDIS_DEV void row_add(PixSums& p, double my, double a0, double a1, double a2, double a3) {
#pragma clang fp contract(off)
  p.z = fma(my, a0, p.z);
  p.zu = fma(my, a1, p.zu);
  p.zm = fma(my, a2, p.zm);
  p.zv = fma(my * my, a3, p.zv);
}


}  // namespace bdis
