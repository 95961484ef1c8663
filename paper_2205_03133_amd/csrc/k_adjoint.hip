// Adjoint (reverse-mode) kernels of the float path: the backward pass of the
// fixed-K unrolled inverse-compositional search and of the Bayesian fusion,
// level by level from the finest to the coarsest, then the transposed
// pyramid.  Discrete decisions (unit cells, the search-threshold reset,
// acceptance, holes, variance-fit outcomes) are piecewise constant and carry
// no gradient.  All sums are FP64; scatters into images and parent maps use
// hardware FP64 atomics, so gradients are reproducible to rounding only.
//
// Forward relations reversed here (per level n, patch k, pixel x):
//   fusion   W_k = M(x - o_k) pi_k, Z = sum W, SM = sum M,
//            Ubar = sum W u / Z, Q = Z / SM, V = sum W^2 sigma_k^2 / Z^2   (Eq. 9-13, 18)
//   holes    Ubar = 2 B(Ubar^(n+1))(x/2), Q = B(Q^(n+1))(x/2)
//   patch    pi = Gamma_n post + B(Q^(n+1))(c/2), post = 1 / sum_d exp(-(SSD_d - SSD_0) / tau)
//            (Eq. 5-6, 11-12); sigma_k^2 = tau / (2 kappa) (Eq. 15-17)
//   level    tau = 2 sigma_r^2 s^2, sigma_r^2 = alpha^2 pooled SSD_0 / (N_acc P^2)
//   search   u_0 = 2 B(Ubar^(n+1))(c/2), u_{t+1} = u_t - sum J (I_w(u_t) - T) / H,
//            J = g - mean g, H = sum J^2, g = Sobel_x(L) / 8, T = L on the patch
//   window   SSD_d = sum (e - mean e)^2, e = I_w(u + d) - T
//   pyramid  L_n = B5 * L_{n-1} (even samples, reflect-101)
#include "bdis_internal.h"
#include "fuse_common.h"

namespace bdis {

namespace {

constexpr double kXd[4] = {1.0, 0.25, 0.25, 1.0};  // d^2 of the offsets -1, -1/2, +1/2, +1

// Scatter v * bilinear weights of (x, y) onto a w x h map (indices clamped).
BDIS_DEV void bilinear_adj(double* m, int w, int h, double x, double y, double v) {
  const double fx0 = floor(x), fy0 = floor(y);
  const double ax = x - fx0, ay = y - fy0;
  const int ix = (int)fx0, iy = (int)fy0;
  const int x0 = clampi(ix, 0, w - 1), x1 = clampi(ix + 1, 0, w - 1);
  const int y0 = clampi(iy, 0, h - 1), y1 = clampi(iy + 1, 0, h - 1);
  atomic_add_d(m + (size_t)y0 * w + x0, v * (1.0 - ax) * (1.0 - ay));
  atomic_add_d(m + (size_t)y0 * w + x1, v * ax * (1.0 - ay));
  atomic_add_d(m + (size_t)y1 * w + x0, v * (1.0 - ax) * ay);
  atomic_add_d(m + (size_t)y1 * w + x1, v * ax * ay);
}

// Block-wide sum of a double (256 threads) into *dst with one atomic.
BDIS_DEV void block_atomic_sum(double v, double* dst, double* s_buf) {
  const int tid = threadIdx.x;
  s_buf[tid] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) s_buf[tid] += s_buf[tid + off];
    __syncthreads();
  }
  if (tid == 0 && s_buf[0] != 0.0) atomic_add_d(dst, s_buf[0]);
  __syncthreads();
}

// Per patch: gather the fusion adjoint over the patch's pixels.  A workgroup
// holds NPB consecutive patches of one patch row (laid out like the search);
// each patch has a group of lanes, one per patch column.  The P image rows are
// streamed through LDS: per row, one lane per pixel reads the fused maps and
// their adjoints (coalesced, once per workgroup) and forms the per-pixel terms
//   A1 = gU/Z, A2 = gU U/Z, B1 = gQ/SM, B2 = gQ Q/SM, C1 = gV/Z^2, C2 = gV V/Z
// (zero on holes); each patch lane then adds its column's mask-weighted terms.
// With m the mask weight and d m its sigma_s derivative, per patch:
//   du = pi sum m A1,   dpi = sum m (u A1 - A2 + B1) + sum (2 pi s2 m^2 C1 - 2 m C2),
//   dsig2 = pi^2 sum m^2 C1,
//   dsigma_s += sum dm (pi u A1 - pi A2 + pi B1 - B2 + 2 pi^2 s2 m C1 - 2 pi C2).
template <int P>
__global__ __launch_bounds__(kSearchF64Threads) void k_fuse_adj(const PairLevel* tab, int npairs, LevelParams lp) {
  constexpr int G = group_lanes(P);
  constexpr int NPB = kSearchF64Threads / G;
  constexpr int NT = 6;  // per-pixel terms
  __shared__ double s_m1[P], s_dm1[P];
  __shared__ double s_buf[kSearchF64Threads];
  __shared__ double s_t[NT][kSearchF64Threads];
  const int lb = xcd_block();
  const PairLevel& a = tab[find_pair<1>(tab, npairs, lb)];
  const int blk = lb - a.search0;
  const int tid = threadIdx.x;
  const int q = tid / G, c = tid % G;
  const int S = lp.S, W = a.g.w;
  if (tid == 0)  // m1(t) = sum_c exp(-(t - c)^2 / (2 s^2)) and its derivative in s
#pragma unroll
    for (int t = 0; t < P; ++t) {
      s_m1[t] = lp.mask[t];
      s_dm1[t] = lp.dmask[t];
    }
  const int j = blk / a.search_nbx;
  const int i0 = (blk % a.search_nbx) * NPB;
  const int i = i0 + q;
  const int oy = grid_origin(j, a.g.h, P, S);
  const int oxa = grid_origin(i0, W, P, S);
  const int tw = min((NPB - 1) * S + P, W - oxa);  // tile columns (<= 256)
  const bool finest = lp.level == lp.finest;
  const bool vt = finest && lp.variance && a.vmap != nullptr;
  const auto ub = gbl(finest ? a.ubar_keep : a.ubar);
  const auto qm = gbl(finest ? a.qmap_keep : a.qmap);

  bool active = false;
  int k = 0, col = 0;
  D4 d{};
  if (i < a.g.nx) {
    k = j * a.g.nx + i;
    d = ld4(a.pa.dens + k);
    active = d.y >= 0.0 && c < P;  // accepted patch, live column
    col = grid_origin(i, W, P, S) - oxa + c;
  }
  const double u = d.x, pi = d.y, s2 = vt ? d.z : 0.0;
  double su = 0.0, spi = 0.0, ssg = 0.0, sss = 0.0;
  // the fused maps and their adjoints of row b (one lane per tile column), all
  // issued at once and one row ahead of their use
  constexpr int NF = 8;  // Z, gU, gQ, SM, U, Q, gV, V
  // At the finest level the map adjoints come straight from the caller's
  // output gradients: d loss / d Ubar = -d loss / d disparity and d loss / d
  // variance on output pixels (a fused value, and confidence at or above the
  // pixel threshold), 0 elsewhere; the confidence adjoint is 0.
  const float pthr = lp.prob_thresh;
  auto load_row = [&](int b, double (&v)[NF]) {
    if (tid < tw) {
      const size_t idx = (size_t)(oy + b) * W + oxa + tid;
      v[0] = gbl(a.zmap)[idx];
      v[3] = gbl(a.smmap)[idx];
      v[4] = ub[idx];
      v[5] = qm[idx];
      v[7] = vt ? gbl(a.vmap)[idx] : 0.0;
      if (finest) {
        const double gd = a.grad_disp ? (double)gbl(a.grad_disp)[idx] : 0.0;
        const double gv = (vt && a.grad_var) ? (double)gbl(a.grad_var)[idx] : 0.0;
        const bool ok = v[0] > 0.0 && !(pthr > 0.0f && v[5] < (double)pthr);
        v[1] = ok ? -gd : 0.0;
        v[2] = 0.0;
        v[6] = ok ? gv : 0.0;
      } else {
        v[1] = gbl(a.ubar_adj)[idx];
        v[2] = gbl(a.qmap_adj)[idx];
        v[6] = 0.0;
      }
    }
  };
  double cur[NF] = {}, nxt[NF] = {};
  load_row(0, cur);
  for (int b = 0; b < P; ++b) {
    if (b + 1 < P) load_row(b + 1, nxt);
    __syncthreads();  // previous row consumed (and the mask sums written)
    if (tid < tw) {
      const double Z = cur[0];
      double t[NT] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (Z > 0.0) {
        const double gU = cur[1], gQ = cur[2];
        const double SM = cur[3];
        t[0] = gU / Z;
        t[1] = t[0] * cur[4];
        t[2] = gQ / SM;
        t[3] = t[2] * cur[5];
        if (vt) {
          const double gV = cur[6];
          t[4] = gV / (Z * Z);
          t[5] = gV * cur[7] / Z;
        }
      }
#pragma unroll
      for (int e = 0; e < NT; ++e) s_t[e][tid] = t[e];
    }
    __syncthreads();
    if (active) {
      const double mb = s_m1[b], dmb = s_dm1[b];
      const double m = mb * s_m1[c], dm = dmb * s_m1[c] + mb * s_dm1[c];
      const double A1 = s_t[0][col], A2 = s_t[1][col], B1 = s_t[2][col], B2 = s_t[3][col];
      const double C1 = s_t[4][col], C2 = s_t[5][col];
      su += m * A1;
      spi += m * (u * A1 - A2 + B1) + 2.0 * pi * s2 * m * m * C1 - 2.0 * m * C2;
      ssg += m * m * C1;
      sss += dm * (pi * u * A1 - pi * A2 + pi * B1 - B2 + 2.0 * pi * pi * s2 * m * C1 - 2.0 * pi * C2);
    }
#pragma unroll
    for (int e = 0; e < NF; ++e) cur[e] = nxt[e];
  }
  if (i < a.g.nx && d.y >= 0.0) {  // uniform over the group
    su = group_sum_d<G>(su);
    spi = group_sum_d<G>(spi);
    ssg = group_sum_d<G>(ssg);
    if (c == 0) {
      gbl(a.pu_adj)[k] = pi * su;
      gbl(a.ppi_adj)[k] = spi;
      gbl(a.psig_adj)[k] = pi * pi * ssg;
    }
  }
  block_atomic_sum(sss, a.hyper_adj + 0, s_buf);
}

// Per patch: posterior, propagation and patch-variance adjoints -> window SSDs,
// tau, level weights and the parent confidence.
__global__ __launch_bounds__(kPixThreads) void k_prob_adj(const PairLevel* tab, int npairs, LevelParams lp) {
  __shared__ double s_buf[kPixThreads];
  const PairLevel& a = tab[find_pair<2>(tab, npairs, (int)blockIdx.x)];
  const int tid = threadIdx.x;
  const int P = lp.P, S = lp.S;
  const int k = ((int)blockIdx.x - a.prob0) * kPixThreads + tid;
  double wsum = 0.0;
  for (int n = lp.finest; n < a.levels; ++n) wsum += (double)lp.omega[n];
  const double gamma = (double)lp.omega[lp.level] / wsum;
  double gam_adj = 0.0, tau_adj = 0.0;
  if (k < a.g.nx * a.g.ny && gbl(a.pa.acc)[k]) {
    const double pi_adj = gbl(a.ppi_adj)[k];
    const bool vt = lp.variance && lp.level == lp.finest;
    const double sig_adj = vt ? gbl(a.psig_adj)[k] : 0.0;
    const D4 dd = ld4(a.pa.dssd + k);
    const double dl[4] = {dd.x, dd.y, dd.z, dd.w};
    const double tau = gbl(a.scal)[1];
    const double rt = 1.0 / tau;  // the record's own form: exponents as products with 1 / tau
    double e[4], se = 1.0;
    for (int t = 0; t < 4; ++t) {
      e[t] = exp(-dl[t] * rt);
      se += e[t];
    }
    const double post = 1.0 / se;
    const double post_adj = gamma * pi_adj;
    gam_adj = pi_adj * post;
    double dl_adj[4];
    double sedl = 0.0;
    for (int t = 0; t < 4; ++t) {
      dl_adj[t] = post_adj * post * post * e[t] * rt;
      sedl += e[t] * dl[t];
    }
    tau_adj = -post_adj * post * post * sedl * (rt * rt);
    if (vt && sig_adj != 0.0) {
      // the fit passed and was not capped iff sigma_k^2 = tau / (2 kappa) < sigma_fail^2,
      // decided by the record's own arithmetic
      const double sfail = lp.var_fail_sigma > 0.0f ? (double)lp.var_fail_sigma : (double)P;
      const VarFit vf = var_fit(dd, rt, lp.var_fit_thresh);
      const double kappa = vf.kappa;
      const bool pass = vf.pass && tau / (2.0 * kappa) < sfail * sfail;
      if (pass) {
        tau_adj += sig_adj / (2.0 * kappa);
        const double kappa_adj = -sig_adj * tau / (2.0 * kappa * kappa);
        for (int t = 0; t < 4; ++t) dl_adj[t] += kappa_adj * (kXd[t] - 0.5) / 0.875;
      }
    }
    auto sa = gbl(a.pssd_adj) + (size_t)k * kWin;
    sa[0] = dl_adj[0];
    sa[1] = dl_adj[1];
    sa[2] = -(dl_adj[0] + dl_adj[1] + dl_adj[2] + dl_adj[3]);
    sa[3] = dl_adj[2];
    sa[4] = dl_adj[3];
    if (a.par_qmap_adj && pi_adj != 0.0) {
      const int i = k % a.g.nx, j = k / a.g.nx;
      const double cx = 0.5 * ((double)grid_origin(i, a.g.w, P, S) + 0.5 * (double)(P - 1));
      const double cy = 0.5 * ((double)grid_origin(j, a.g.h, P, S) + 0.5 * (double)(P - 1));
      bilinear_adj(a.par_qmap_adj, a.pw, a.ph, cx, cy, pi_adj);
    }
  } else if (k < a.g.nx * a.g.ny) {
    auto sa = gbl(a.pssd_adj) + (size_t)k * kWin;
    for (int t = 0; t < kWin; ++t) sa[t] = 0.0;
  }
  block_atomic_sum(tau_adj, a.scal + 4, s_buf);
  // d Gamma_n / d omega_m = (delta_nm - Gamma_n) / sum omega
  block_atomic_sum(gam_adj, a.scal + 6, s_buf);
}

// The level's d loss / d tau (summed by the probability adjoint) through tau =
// 2 sigma_r^2 s^2: returns the share every accepted SSD(0) of the level receives
// in the dynamic mode (0 otherwise); with `commit` (once per pair) adds the
// hyper-gradients of sigma_r (alpha_r) and of the level weights,
// Gamma_n = omega_n / sum omega.
BDIS_DEV double tau_adjoint(const PairLevel& a, const LevelParams& lp, bool commit) {
  const auto sc = gbl(a.scal);
  const double tau_adj = sc[4];
  const double al = (double)lp.sigma_r;
  const double w2 = 2.0 * kWin * kWin;  // tau = w2 * sigma_r^2
  double shr = 0.0, sr_adj;
  if (lp.sigma_r_dynamic) {
    const double pooled = sc[2], nacc = sc[3];
    if (pooled > kEpsSigma) {
      sr_adj = tau_adj * w2 * 2.0 * al * pooled;
      shr = tau_adj * w2 * al * al / (nacc * (double)(lp.P * lp.P));
    } else {
      sr_adj = tau_adj * w2 * 2.0 * al * kEpsSigma;
    }
  } else {
    sr_adj = tau_adj * w2 * 2.0 * al;
  }
  if (commit) {
    atomic_add_d(a.hyper_adj + 1, sr_adj);
    // level weights: Gamma_n = omega_n / sum_{m=f}^{L-1} omega_m
    const double gam_adj = sc[6];
    double wsum = 0.0;
    for (int n = lp.finest; n < a.levels; ++n) wsum += (double)lp.omega[n];
    const double gamma = (double)lp.omega[lp.level] / wsum;
    for (int m = lp.finest; m < a.levels; ++m)
      atomic_add_d(a.hyper_adj + 2 + m, gam_adj * ((m == lp.level ? 1.0 : 0.0) - gamma) / wsum);
  }
  return shr;
}

// What a patch row's adjoint reads before its first scatter: the template row
// and its zero-mean gradient, H, the patch's final displacement and its
// adjoint, the window's right-image samples and the window SSD adjoints.  The
// search adjoint issues these loads before its workgroup prologue, so that
// their round trips overlap the prologue's.
template <int P>
struct AdjStart {
  double T[P], J[P], H;
  double u, ub;
  double Rw[P + 3];  // right samples at columns ox + m0 - 1 .. ox + m0 + P + 1, m0 = floor(u)
  double sbars[kWin];
};

template <int P>
BDIS_DEV void patch_adj_start(const PairLevel& a, int k, int r, int ox, int oy, double shr, AdjStart<P>& st) {
  constexpr int G = group_lanes(P);
  constexpr int N = P * P;
  const int W = a.g.w, Hh = a.g.h;
  const bool row_live = r < P;
  const int rr = row_live ? r : P - 1;
  const auto Lg = gbl(a.Ld);
  const int dp = a.dpitch;
  const int yr = oy + rr;
  const size_t r0 = (size_t)reflect101(yr - 1, Hh) * dp, r1 = (size_t)yr * dp,
               r2 = (size_t)reflect101(yr + 1, Hh) * dp;
  st.u = gbl(a.pa.u)[k];
  st.ub = gbl(a.pu_adj)[k];
  const auto sa = gbl(a.pssd_adj) + (size_t)k * kWin;
#pragma unroll
  for (int t = 0; t < kWin; ++t) st.sbars[t] = sa[t];
  st.sbars[2] += shr;  // share of d loss / d tau through sigma_r
  double sg = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const int x = ox + c, xm = reflect101(x - 1, W), xp = reflect101(x + 1, W);
    st.T[c] = Lg[r1 + x];
    st.J[c] = ((Lg[r0 + xp] - Lg[r0 + xm]) + 2.0 * (Lg[r1 + xp] - Lg[r1 + xm]) + (Lg[r2 + xp] - Lg[r2 + xm])) / 8.0;
    sg += st.J[c];
  }
  const auto Rrow = gbl(a.Rd) + (size_t)(oy + rr) * dp;
  const int m0 = (int)floor(st.u);
#pragma unroll
  for (int c = 0; c < P + 3; ++c) st.Rw[c] = Rrow[clampi(ox + m0 - 1 + c, 0, W - 1)];
  const double gbar = group_sum_d<G>(row_live ? sg : 0.0) / (double)N;
  double hrow = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    st.J[c] -= gbar;
    hrow += st.J[c] * st.J[c];
  }
  st.H = group_sum_d<G>(row_live ? hrow : 0.0);
}

template <int P>
BDIS_DEV void patch_adj(const PairLevel& a, const LevelParams& lp, int k, int r, int ox, int oy, int oxa, int xr0,
                        int twl, int twr, double* sL, double* sG, double* sR, const AdjStart<P>& st) {
  constexpr int G = group_lanes(P);
  constexpr int N = P * P;
  const int W = a.g.w;
  const bool row_live = r < P;
  const int rr = row_live ? r : P - 1;
  const auto Rg = gbl(a.Rd);
  const int dp = a.dpitch;
  const double* const T = st.T;
  const double* const J = st.J;
  const double H = st.H;

  double Tb[P], Jb[P];
#pragma unroll
  for (int c = 0; c < P; ++c) Tb[c] = Jb[c] = 0.0;
  const auto Rrow = Rg + (size_t)(oy + rr) * dp;
  double* Rbar_row = a.Rbar + (size_t)(oy + rr) * dp;

  // Every warp of this patch row reads R at ox + m + c' (c' = 0..P) for its unit
  // cell m.  Scatters into R are summed in registers while m stays the same (the
  // cell is uniform over the patch, so the flush is too) and written with one
  // atomic per touched pixel when it changes.
  double acc[P + 1];
#pragma unroll
  for (int c = 0; c <= P; ++c) acc[c] = 0.0;
  int mcur = 0;
  bool have = false;
  auto flush = [&]() {
    if (have && row_live) {
#pragma unroll
      for (int c = 0; c <= P; ++c) {
        if (acc[c] == 0.0) continue;
        const int x = clampi(ox + mcur + c, 0, W - 1);
        if (x - xr0 >= 0 && x - xr0 < twr)
          unsafeAtomicAdd(sR + rr * twr + (x - xr0), acc[c]);
        else
          atomic_add_d(Rbar_row + x, acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c <= P; ++c) acc[c] = 0.0;
  };
  auto to_cell = [&](int m) {
    if (!have || m != mcur) {
      flush();
      mcur = m;
      have = true;
    }
  };

  // ---- window: SSD_d = sum (e - mean e)^2 at u + d.  The five offsets fall in
  // the cells m0 - 1, m0, m0 + 1 (m0 = floor u), whose samples are read once.
  const double u = st.u;
  double ub = st.ub;
  const int m0 = (int)floor(u);
  const double* const Rw = st.Rw;
  // one window sample at cell m0 - 1 + O, fraction f
  auto window_term = [&](auto oc, double f, double sbar) {
    constexpr int O = decltype(oc)::value;
    double ev[P], se = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      ev[c] = (1.0 - f) * Rw[O + c] + f * Rw[O + c + 1] - T[c];
      se += ev[c];
    }
    const double emean = group_sum_d<G>(row_live ? se : 0.0) / (double)N;
    double urow = 0.0;
    to_cell(m0 - 1 + O);
#pragma unroll
    for (int c = 0; c < P; ++c) {
      const double g2 = 2.0 * (ev[c] - emean) * sbar;
      urow += g2 * (Rw[O + c + 1] - Rw[O + c]);
      Tb[c] -= g2;
      acc[c] += g2 * (1.0 - f);
      acc[c + 1] += g2 * f;
    }
    ub += group_sum_d<G>(row_live ? urow : 0.0);
  };
#pragma unroll
  for (int t = 0; t < kWin; ++t) {
    const double sbar = st.sbars[t];
    if (sbar == 0.0) continue;
    const double v = u + 0.5 * (double)(t - 2);  // offsets -1, -1/2, 0, 1/2, 1
    const double fm = floor(v);
    const int o = (int)fm - (m0 - 1);  // 0, 1 or 2
    const double f = v - fm;
    if (o == 0)
      window_term(std::integral_constant<int, 0>{}, f, sbar);
    else if (o == 1)
      window_term(std::integral_constant<int, 1>{}, f, sbar);
    else
      window_term(std::integral_constant<int, 2>{}, f, sbar);
  }

  // ---- reset, then the K iterations in reverse.  Within one unit cell m the
  // warp is I_w(u) = (1 - f) Ra + f Rb with fixed samples Ra, Rb, so the
  // per-column adjoints of consecutive iterations in that cell only differ by
  // scalar factors: those are summed (al, be, de) and applied once per cell.
  double u0_adj = ub;
  const bool reset = gbl(a.reset)[k] != 0;
  if (!reset && H >= kEpsH) {
    double crow = 0.0;
#pragma unroll
    for (int c = 0; c < P; ++c) crow += J[c] * T[c];
    const double cT = group_sum_d<G>(row_live ? crow : 0.0);
    const auto uh = gbl(a.uhist) + (size_t)k * (lp.K + 1);
    double Rv[P + 1];
    double C0 = 0.0, C1 = 0.0, al = 0.0, be = 0.0, de = 0.0;
    int mc = 0;
    bool cell = false;
    auto apply = [&]() {
      if (!cell) return;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        Jb[c] += -al * Rv[c] - be * Rv[c + 1] + (al + be) * T[c] + de * J[c];
        Tb[c] += (al + be) * J[c];
        acc[c] -= al * J[c];
        acc[c + 1] -= be * J[c];
      }
      al = be = de = 0.0;
    };
    const double rH = 1.0 / H;    // one division for the K reverse steps
    double u_next = uh[lp.K - 1];  // the next iterate is loaded one step ahead
    // the cell's correlations with the gradient, from its samples in Rv
    auto enter_cell = [&](int m) {
      double c0 = 0.0, c1 = 0.0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        c0 += J[c] * Rv[c];
        c1 += J[c] * Rv[c + 1];
      }
      C0 = group_sum_d<G>(row_live ? c0 : 0.0) - cT;
      C1 = group_sum_d<G>(row_live ? c1 : 0.0) - cT;
      mc = m;
      cell = true;
    };
    {
      // The first cell of the reverse pass (that of u_(K-1)) is nearly always
      // one of the window's three cells, whose samples are already held: the
      // same pixels as a reload, without its round trip.
      const int m = (int)floor(u_next);
      const int o = m - (m0 - 1);
      to_cell(m);
      // (constant indices in each branch keep Rw and Rv in registers)
      if (o == 0) {
#pragma unroll
        for (int c = 0; c <= P; ++c) Rv[c] = Rw[c];
      } else if (o == 1) {
#pragma unroll
        for (int c = 0; c <= P; ++c) Rv[c] = Rw[c + 1];
      } else if (o == 2) {
#pragma unroll
        for (int c = 0; c <= P; ++c) Rv[c] = Rw[c + 2];
      } else {
#pragma unroll
        for (int c = 0; c <= P; ++c) Rv[c] = Rrow[clampi(ox + c + m, 0, W - 1)];
      }
      enter_cell(m);
    }
    for (int t = lp.K - 1; t >= 0; --t) {
      const double ut = u_next;
      if (t > 0) u_next = uh[t - 1];
      const double fm = floor(ut);
      const int m = (int)fm;
      const double f = ut - fm;
      if (m != mc) {
        apply();
        to_cell(m);
#pragma unroll
        for (int c = 0; c <= P; ++c) Rv[c] = Rrow[clampi(ox + c + m, 0, W - 1)];
        enter_cell(m);
      }
      const double b = (1.0 - f) * C0 + f * C1;  // sum J (I_w - T)
      const double s1 = ub * rH;
      al += s1 * (1.0 - f);
      be += s1 * f;
      de += 2.0 * s1 * b * rH;
      ub = ub * (1.0 - (C1 - C0) * rH);
    }
    apply();
    u0_adj = ub;
  }
  flush();

  // ---- J = g - mean g, T and g live on the left level image
  double jb = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) jb += Jb[c];
  const double jmean = group_sum_d<G>(row_live ? jb : 0.0) / (double)N;
  if (row_live && twl > 0) {
    double* Lrow = sL + rr * twl + (ox - oxa);
    double* Grow = sG + rr * twl + (ox - oxa);
#pragma unroll
    for (int c = 0; c < P; ++c) {
      if (Tb[c] != 0.0) unsafeAtomicAdd(Lrow + c, Tb[c]);
      const double gb = Jb[c] - jmean;
      if (gb != 0.0) unsafeAtomicAdd(Grow + c, gb);
    }
  } else if (row_live) {
    double* Lrow = a.Lbar + (size_t)(oy + rr) * dp + ox;
    double* Grow = a.Gbar + (size_t)(oy + rr) * dp + ox;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      if (Tb[c] != 0.0) atomic_add_d(Lrow + c, Tb[c]);
      const double gb = Jb[c] - jmean;
      if (gb != 0.0) atomic_add_d(Grow + c, gb);
    }
  }
  // ---- u_0 = 2 B(Ubar^(n+1))(c/2)
  if (r == 0 && a.par_ubar_adj && u0_adj != 0.0) {
    const double cx = 0.5 * ((double)ox + 0.5 * (double)(P - 1));
    const double cy = 0.5 * ((double)oy + 0.5 * (double)(P - 1));
    bilinear_adj(a.par_ubar_adj, a.pw, a.ph, cx, cy, 2.0 * u0_adj);
  }
}

// Per patch (lane per patch row): window and search adjoints, recomputing the
// warps from the saved iterates; scatters into the level images, the template
// gradient image and the parent displacement map.
//
// The patches of one workgroup are consecutive in one patch row, so they share
// their P image rows: their scatters into the left image, the gradient image
// and the right image are summed in LDS tiles (rows oy .. oy+P-1; the left
// tiles start at the first patch's origin, the right tile at the lowest warp
// cell any patch of the workgroup visits) and written to HBM once per tile
// element.  Right-image samples beyond the tile go straight to HBM.  twl = 0
// (tiles too large for LDS) sends everything straight to HBM.
template <int P>
__global__ __launch_bounds__(kSearchF64Threads) void k_search_adj(const PairLevel* tab, int npairs, LevelParams lp,
                                                                  int twl, int twr) {
  constexpr int G = group_lanes(P);
  constexpr int NPB = kSearchF64Threads / G;
  extern __shared__ double s_tile[];  // [P][twl] left, [P][twl] gradient, [P][twr] right
  __shared__ int s_lo;
  const int lb = xcd_block();
  const PairLevel& a = tab[find_pair<1>(tab, npairs, lb)];
  const int blk = lb - a.search0;
  const int tid = threadIdx.x;
  const int q = tid / G, r = tid % G;
  const int W = a.g.w, Hh = a.g.h, S = lp.S;
  const int j = blk / a.search_nbx;
  const int i0 = (blk % a.search_nbx) * NPB;
  const bool live = (i0 + q) < a.g.nx;
  const int i = live ? i0 + q : a.g.nx - 1;
  const int k = j * a.g.nx + i;
  // whole groups skip rejected or idle patches (uniform within the group)
  const bool active = live && gbl(a.pa.acc)[k] != 0;
  const int ox = grid_origin(i, W, P, S), oy = grid_origin(j, Hh, P, S);
  const int oxa = grid_origin(i0, W, P, S);
  double* sL = s_tile;
  double* sG = s_tile + P * twl;
  double* sR = s_tile + 2 * P * twl;
  // the level's tau adjoint (summed by the probability adjoint): its share per
  // accepted SSD(0), and, once per pair (thread 0 of the pair's first
  // workgroup), the hyper-gradients of sigma_r and of the level weights
  const double shr = tau_adjoint(a, lp, blk == 0 && tid == 0);
  AdjStart<P> st;
  if (active) patch_adj_start<P>(a, k, r, ox, oy, shr, st);
  if (twl > 0) {
    for (int e = tid; e < P * (2 * twl + twr); e += kSearchF64Threads) s_tile[e] = 0.0;
    if (tid == 0) s_lo = INT_MAX;
    __syncthreads();
    if (active && r == 0) {  // lowest warp cell of this patch: window and iterations
      int mlo = (int)floor(gbl(a.pa.u)[k] - 1.0);
      const auto uh = gbl(a.uhist) + (size_t)k * (lp.K + 1);
#pragma unroll 8
      for (int t = 0; t < lp.K; ++t) mlo = min(mlo, (int)floor(uh[t]));  // loads issued eight at a time
      atomicMin(&s_lo, ox + mlo);
    }
    __syncthreads();
    if (s_lo == INT_MAX) return;  // no accepted patch here (uniform)
  }
  // the right tile starts at the lowest cell, but never past the last column:
  // scatters are clamped to the row, so every one of them lands at or after it
  const int xr0 = twl > 0 ? min(s_lo, W - 1) : 0;
  if (active) patch_adj<P>(a, lp, k, r, ox, oy, oxa, xr0, twl, twr, sL, sG, sR, st);
  if (twl == 0) return;
  __syncthreads();
  const int dp = a.dpitch;
  for (int e = tid; e < P * twl; e += kSearchF64Threads) {
    const int rr = e / twl, x = oxa + e % twl;
    const size_t o = (size_t)(oy + rr) * dp + x;
    if (sL[e] != 0.0) atomic_add_d(a.Lbar + o, sL[e]);
    if (sG[e] != 0.0) atomic_add_d(a.Gbar + o, sG[e]);
  }
  for (int e = tid; e < P * twr; e += kSearchF64Threads) {
    const int rr = e / twr, x = xr0 + e % twr;
    if (sR[e] != 0.0) atomic_add_d(a.Rbar + (size_t)(oy + rr) * dp + x, sR[e]);
  }
}

// The transposed template gradient g = Sobel_x(L) / 8 (reflect-101) at pixel
// (x, y), gathered: the sum of the gradient adjoints of the neighbours whose
// stencil (after reflection) reads the pixel, with their stencil weights (the
// caller divides by 8).
BDIS_DEV double sobel_gather(const PairLevel& a, int x, int y) {
  const int w = a.g.w, h = a.g.h;
  const auto Gb = gbl(a.Gbar);
  double acc = 0.0;
  if (x >= 2 && x <= w - 3 && y >= 2 && y <= h - 3) {
    // interior: no reflection reaches the pixel; rows y-1, y, y+1 weigh 1, 2, 1,
    // columns x-1 and x+1 weigh +1 and -1: the nonzero terms of the general
    // form below, in its order, so the same bits
    const double wys[3] = {1.0, 2.0, 1.0};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const size_t row = (size_t)(y - 1 + j) * a.dpitch;
      acc += wys[j] * 1.0 * Gb[row + x - 1];
      acc += wys[j] * -1.0 * Gb[row + x + 1];
    }
    return acc;
  }
  for (int yy = max(y - 1, 0); yy <= min(y + 1, h - 1); ++yy) {
    // rows yy-1, yy, yy+1 of the stencil weigh 1, 2, 1
    const double wy = (reflect101(yy - 1, h) == y ? 1.0 : 0.0) + (yy == y ? 2.0 : 0.0) +
                      (reflect101(yy + 1, h) == y ? 1.0 : 0.0);
    if (wy == 0.0) continue;
    for (int xx = max(x - 1, 0); xx <= min(x + 1, w - 1); ++xx) {
      const double wx = (reflect101(xx + 1, w) == x ? 1.0 : 0.0) - (reflect101(xx - 1, w) == x ? 1.0 : 0.0);
      if (wx != 0.0) acc += wy * wx * Gb[(size_t)yy * a.dpitch + xx];
    }
  }
  return acc;
}

// Per pixel: the transposed template gradient, added to the level image's
// adjoint.  One owner per pixel, no atomics.
__global__ __launch_bounds__(kPixThreads) void k_sobel_adj(const PairLevel* tab, int npairs, int holes) {
  const PairLevel& a = tab[find_pair<0>(tab, npairs, (int)blockIdx.x)];
  const int idx = ((int)blockIdx.x - a.pyr0) * kPixThreads + (int)threadIdx.x;
  const int w = a.g.w, h = a.g.h;
  if (idx >= w * h) return;
  const int y = idx / w, x = idx - y * w;
  // above the finest level, holes (no accepted covering patch) took the parent
  // estimate: their adjoints go to the parent maps (read by the parent level's
  // pass, which runs after this one)
  if (holes && a.par_ubar_adj && !(gbl(a.zmap)[idx] > 0.0)) {
    const double gU = gbl(a.ubar_adj)[idx], gQ = gbl(a.qmap_adj)[idx];
    if (gU != 0.0) bilinear_adj(a.par_ubar_adj, a.pw, a.ph, 0.5 * x, 0.5 * y, 2.0 * gU);
    if (gQ != 0.0) bilinear_adj(a.par_qmap_adj, a.pw, a.ph, 0.5 * x, 0.5 * y, gQ);
  }
  const double acc = sobel_gather(a, x, y);
  if (acc != 0.0) gbl(a.Lbar)[(size_t)y * a.dpitch + x] += acc / 8.0;
}

// Binomial tap weight with which level-(n+1) sample k (at 2k + t - 2, t = 0..4,
// reflect-101 in a source of length n) reads source index i.
BDIS_DEV double pyr_tap_weight(int k, int i, int n) {
  const double kb[5] = {1.0, 4.0, 6.0, 4.0, 1.0};
  double wgt = 0.0;
#pragma unroll
  for (int t = 0; t < 5; ++t)
    if (reflect101(2 * k + t - 2, n) == i) wgt += kb[t];
  return wgt;
}

// Per pixel of level n (n < coarsest): the transposed binomial pyramid step
// from level n+1, gathered.  Parent samples k read source rows 2k-2 .. 2k+2
// (reflected at most once), so only k in [i/2 - 2, i/2 + 2] can reach i.
// sobel: the level's transposed template gradient is added here first (in
// place of a k_sobel_adj launch at this level; the same terms in the same order).
__global__ __launch_bounds__(kPixThreads) void k_pyr_adj(const PairLevel* tab, int npairs, int sobel) {
  const PairLevel& a = tab[find_pair<0>(tab, npairs, (int)blockIdx.x)];
  const int idx = ((int)blockIdx.x - a.pyr0) * kPixThreads + (int)threadIdx.x;
  const int w = a.g.w, h = a.g.h;
  if (idx >= w * h) return;
  const int y = idx / w, x = idx - y * w;
  const size_t o = (size_t)y * a.dpitch + x;
  // adds the parent's share to this pixel's image adjoints; at level 0 (the
  // entries that carry the caller's gradient outputs) writes those instead:
  // nothing reads a level-0 adjoint after this pass
  auto finish = [&](double sl, double sr) {
    const double sg = sobel ? sobel_gather(a, x, y) : 0.0;
    double vl = 0.0, vr = 0.0;
    if (sl != 0.0 || sg != 0.0 || a.grad_left) vl = gbl(a.Lbar)[o];
    if (sr != 0.0 || a.grad_right) vr = gbl(a.Rbar)[o];
    if (sg != 0.0) vl += sg / 8.0;
    if (sl != 0.0) vl += sl / 256.0;
    if (sr != 0.0) vr += sr / 256.0;
    if (a.grad_left)
      gbl(a.grad_left)[idx] = (float)vl;
    else if (sl != 0.0 || sg != 0.0)
      gbl(a.Lbar)[o] = vl;
    if (a.grad_right)
      gbl(a.grad_right)[idx] = (float)vr;
    else if (sr != 0.0)
      gbl(a.Rbar)[o] = vr;
  };
  if (a.upLbar == nullptr) {  // a pair's coarsest level: no parent share
    finish(0.0, 0.0);
    return;
  }
  const auto uL = gbl(a.upLbar), uR = gbl(a.upRbar);
  if (x >= 3 && x <= w - 4 && y >= 3 && y <= h - 4) {
    // interior: no reflected index reaches the pixel, so its parent taps are
    // those with 2k + t - 2 = i: k = i/2 - 1, i/2, i/2 + 1 with weights 1, 6, 1
    // (i even) or k = (i-1)/2, (i+1)/2 with weights 4, 4 (i odd).  The same
    // nonzero terms in the same order as the general form below, so the same
    // bits.
    const int nx = (x & 1) ? 2 : 3, ny = (y & 1) ? 2 : 3;
    const int kx0 = (x & 1) ? x / 2 : x / 2 - 1, ky0 = (y & 1) ? y / 2 : y / 2 - 1;
    const double w3[3] = {1.0, 6.0, 1.0}, w2[2] = {4.0, 4.0};
    double sl = 0.0, sr = 0.0;
    for (int jy = 0; jy < ny; ++jy) {
      const double wy = (y & 1) ? w2[jy] : w3[jy];
      const size_t row = (size_t)(ky0 + jy) * a.updpitch + kx0;
      for (int jx = 0; jx < nx; ++jx) {
        const double wgt = wy * ((x & 1) ? w2[jx] : w3[jx]);
        sl += wgt * uL[row + jx];
        sr += wgt * uR[row + jx];
      }
    }
    finish(sl, sr);
    return;
  }
  const int ky0 = max(y / 2 - 2, 0), ky1 = min(y / 2 + 2, a.uph - 1);
  const int kx0 = max(x / 2 - 2, 0), kx1 = min(x / 2 + 2, a.upw - 1);
  double wxs[5];
  for (int kx = kx0; kx <= kx1; ++kx) wxs[kx - kx0] = pyr_tap_weight(kx, x, w);
  double sl = 0.0, sr = 0.0;
  for (int ky = ky0; ky <= ky1; ++ky) {
    const double wy = pyr_tap_weight(ky, y, h);
    if (wy == 0.0) continue;
    const size_t row = (size_t)ky * a.updpitch;
    for (int kx = kx0; kx <= kx1; ++kx) {
      const double wgt = wy * wxs[kx - kx0];
      if (wgt == 0.0) continue;
      sl += wgt * uL[row + kx];
      sr += wgt * uR[row + kx];
    }
  }
  finish(sl, sr);
}

// Level 0, per pixel: image gradients out (float32, dense W x H).
__global__ __launch_bounds__(kPixThreads) void k_grad_out(const PairLevel* tab, int npairs) {
  const PairLevel& a = tab[find_pair<0>(tab, npairs, (int)blockIdx.x)];
  const int idx = ((int)blockIdx.x - a.pyr0) * kPixThreads + (int)threadIdx.x;
  const int w = a.g.w, h = a.g.h;
  if (idx >= w * h) return;
  const int y = idx / w, x = idx - y * w;
  if (a.grad_left) gbl(a.grad_left)[idx] = (float)gbl(a.Lbar)[(size_t)y * a.dpitch + x];
  if (a.grad_right) gbl(a.grad_right)[idx] = (float)gbl(a.Rbar)[(size_t)y * a.dpitch + x];
}

hipError_t launch_search_adj(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  return by_patch(lp.P, [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    constexpr int NPB = kSearchF64Threads / group_lanes(P);
    int twl = (NPB - 1) * lp.S + P, twr = twl + 64;
    size_t bytes = sizeof(double) * (size_t)P * (2 * twl + twr);
    if (bytes > kAdjTileBytes) {
      twl = twr = 0;
      bytes = 0;
    }
    bdis_launch(k_search_adj<P>, dim3(nblocks), dim3(kSearchF64Threads), bytes, s, tab, npairs, lp, twl, twr);
    return hipGetLastError();
  });
}

hipError_t launch_fuse_adj(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  return by_patch(lp.P, [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    bdis_launch(k_fuse_adj<P>, dim3(nblocks), dim3(kSearchF64Threads), 0, s, tab, npairs, lp);
    return hipGetLastError();
  });
}

}  // namespace

// blocks: [per-pixel workgroups, search workgroups, per-patch workgroups]
hipError_t launch_backward_level(const PairLevel* tab, int npairs, const int* blocks, const LevelParams& lp,
                                 bool sobel_in_pyramid, hipStream_t s) {
  const dim3 pix(kPixThreads);
  hipError_t e = launch_fuse_adj(tab, npairs, blocks[1], lp, s);
  if (e != hipSuccess) return e;
  bdis_launch(k_prob_adj, dim3(blocks[2]), pix, 0, s, tab, npairs, lp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_search_adj(tab, npairs, blocks[1], lp, s)) != hipSuccess) return e;
  if (sobel_in_pyramid) return hipSuccess;
  bdis_launch(k_sobel_adj, dim3(blocks[0]), pix, 0, s, tab, npairs, lp.level > lp.finest ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pyramid_adj(const PairLevel* tab, int npairs, int nblocks, bool sobel, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  bdis_launch(k_pyr_adj, dim3(nblocks), dim3(kPixThreads), 0, s, tab, npairs, sobel ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_grad_out(const PairLevel* tab, int npairs, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  bdis_launch(k_grad_out, dim3(nblocks), dim3(kPixThreads), 0, s, tab, npairs);
  return hipGetLastError();
}

}  // namespace bdis
