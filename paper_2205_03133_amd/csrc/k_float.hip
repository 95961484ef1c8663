// Float (differentiable) path of the pyramid and the patch search, in FP64.
//
// The caller's float images become FP64 level 0; levels 1..L-1 are the same
// binomial pyramid as the integer path without rounding (Sec. III-B).  The
// search follows Eq. 1 (inverse compositional, mean-normalised residual) and
// the 5-sample window of Eq. 5-6 with the same lane-per-patch-row mapping as
// the integer kernel, but with FP64 sums: the image values are arbitrary
// reals, so the exact integer form does not apply.  Training contexts keep
// the iterates u_0 .. u_K and the reset flag of every patch; the backward
// pass recomputes the warps from them.
#include "bdis_internal.h"

#include <climits>

namespace bdis {

namespace {

// Level 0: float -> double copy.  Levels n >= 1: 5x5 binomial / 256, reflect-101,
// even samples.  One lane per output pixel of both views.
__global__ __launch_bounds__(kPixThreads) void k_pyr_f64(const PairLevel* tab, int npairs, int level) {
  const PairLevel& a = tab[find_pair<0>(tab, npairs, (int)blockIdx.x)];
  const int idx = ((int)blockIdx.x - a.pyr0) * kPixThreads + (int)threadIdx.x;
  const int w = a.g.w, h = a.g.h;
  if (idx >= w * h) return;
  const int y = idx / w, x = idx - y * w;
  if (level == 0) {
    gbl(a.Ld)[(size_t)y * a.dpitch + x] = (double)gbl(a.src32L)[(size_t)y * a.src32pitch + x];
    gbl(a.Rd)[(size_t)y * a.dpitch + x] = (double)gbl(a.src32R)[(size_t)y * a.src32pitch + x];
    return;
  }
  const int kb[5] = {1, 4, 6, 4, 1};
  const auto sl = gbl(a.srcdL);
  const auto sr = gbl(a.srcdR);
  double accl = 0.0, accr = 0.0;
  for (int b = 0; b < 5; ++b) {
    const size_t row = (size_t)reflect101(2 * y + b - 2, a.sh) * a.srcdpitch;
    for (int c = 0; c < 5; ++c) {
      const int xx = reflect101(2 * x + c - 2, a.sw);
      const double wgt = (double)(kb[c] * kb[b]);
      accl += wgt * sl[row + xx];
      accr += wgt * sr[row + xx];
    }
  }
  gbl(a.Ld)[(size_t)y * a.dpitch + x] = accl / 256.0;
  gbl(a.Rd)[(size_t)y * a.dpitch + x] = accr / 256.0;
}

// N consecutive samples of a right-image row from column x: from the staged
// LDS window (columns xs .. xs+rw-1) when it holds them all, else from global
// memory with the columns clamped to the row.
template <int N>
BDIS_DEV void fetch_f64(double (&v)[N], const double* win, int xs, int rw,
                        const __attribute__((address_space(1))) double* grow, int x, int W) {
  const int off = x - xs;
  if (off >= 0 && off + N <= rw) {
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = win[off + n];
  } else {
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = grow[clampi(x + n, 0, W - 1)];
  }
}

template <int P>
__global__ __launch_bounds__(kSearchF64Threads) void k_search_f64(const PairLevel* tab, int npairs, LevelParams lp) {
  constexpr int G = group_lanes(P);
  constexpr int NPB = kSearchF64Threads / G;
  constexpr int N = P * P;
  __shared__ double s_psum[NPB];
  __shared__ int s_pcnt[NPB];

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
  const int ox = grid_origin(i, W, P, S);
  const int oy = grid_origin(j, Hh, P, S);
  const int k = j * a.g.nx + i;

  double uinit = 0.0, pipar = 0.0;
  if (a.par_ubar) {
    const double cx = 0.5 * ((double)ox + 0.5 * (double)(P - 1));
    const double cy = 0.5 * ((double)oy + 0.5 * (double)(P - 1));
    uinit = 2.0 * bilinear(a.par_ubar, a.pw, a.ph, cx, cy);
    pipar = bilinear(a.par_q, a.pw, a.ph, cx, cy);
  }

  // ---- template row and its gradient (loaded before the staging barriers so
  // that their loads overlap the window's)
  const bool row_live = r < P;
  const int rr = row_live ? r : P - 1;
  const auto Lg = gbl(a.Ld);
  const auto Rg = gbl(a.Rd);
  const int dp = a.dpitch;
  const int yr = oy + rr;
  const size_t r0 = (size_t)reflect101(yr - 1, Hh) * dp, r1 = (size_t)yr * dp,
               r2 = (size_t)reflect101(yr + 1, Hh) * dp;
  double T[P], J[P];
  double sg = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const int x = ox + c, xm = reflect101(x - 1, W), xp = reflect101(x + 1, W);
    T[c] = Lg[r1 + x];
    const double gs = (Lg[r0 + xp] - Lg[r0 + xm]) + 2.0 * (Lg[r1 + xp] - Lg[r1 + xm]) + (Lg[r2 + xp] - Lg[r2 + xm]);
    J[c] = gs / 8.0;
    sg += J[c];
  }
  const double gbar = group_sum_d<G>(row_live ? sg : 0.0) / (double)N;
  double hrow = 0.0, crow = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    J[c] -= gbar;
    hrow += J[c] * J[c];
    crow += J[c] * T[c];
  }
  const double H = group_sum_d<G>(row_live ? hrow : 0.0);
  const double cT = group_sum_d<G>(row_live ? crow : 0.0);
  const bool invert = H >= kEpsH;

  // ---- right rows oy .. oy+P-1 around the patches' starting displacements,
  // staged in LDS (columns xs .. xs+rw-1, clamped to the image); samples
  // outside come from global memory (identical values)
  extern __shared__ double s_rwin[];  // [P][rwd]
  __shared__ int s_umin, s_umax;
  constexpr int MARG = P + 4;
  const int rwd = f64_window_cols(P, S);
  if (tid == 0) {
    s_umin = INT_MAX;
    s_umax = INT_MIN;
  }
  __syncthreads();
  if (r == 0 && live) {
    const int mu = (int)floor(uinit);
    atomicMin(&s_umin, mu);
    atomicMax(&s_umax, mu);
  }
  __syncthreads();
  const int ox0 = grid_origin(i0, W, P, S);
  const int oxl = grid_origin(min(i0 + NPB - 1, a.g.nx - 1), W, P, S);
  const int xs = ox0 + s_umin - MARG;
  const int rw = min(oxl + P + s_umax + MARG + 2 - xs, rwd);
  for (int e = tid; e < P * rw; e += kSearchF64Threads) {
    const int ty = e / rw, cx = e - ty * rw;
    s_rwin[ty * rwd + cx] = gbl(a.Rd)[(size_t)(oy + ty) * a.dpitch + clampi(xs + cx, 0, W - 1)];
  }
  __syncthreads();

  const auto Rrow = Rg + (size_t)(oy + rr) * dp;
  double u = uinit;
  const bool keep = a.uhist != nullptr && r == 0 && live;
  {
    int mc = INT_MIN;
    double C0 = 0.0, C1 = 0.0;
    // one division by the Hessian per patch, off the iterations' dependent
    // chain; the adjoint's reverse steps use the same reciprocal
    const double rH = invert ? 1.0 / H : 0.0;
    for (int t = 0; t < lp.K; ++t) {
      if (keep) gbl(a.uhist)[(size_t)k * (lp.K + 1) + t] = u;
      if (!invert) continue;
      const double fm = floor(u);
      const int m = (int)fm;
      const double f = u - fm;
      if (m != mc) {
        double c0 = 0.0, c1 = 0.0;
        double Rv[P + 1];
        fetch_f64<P + 1>(Rv, s_rwin + rr * rwd, xs, rw, Rrow, ox + m, W);
#pragma unroll
        for (int c = 0; c < P; ++c) {
          c0 += J[c] * Rv[c];
          c1 += J[c] * Rv[c + 1];
        }
        C0 = group_sum_d<G>(row_live ? c0 : 0.0) - cT;
        C1 = group_sum_d<G>(row_live ? c1 : 0.0) - cT;
        mc = m;
      }
      u -= ((1.0 - f) * C0 + f * C1) * rH;
    }
  }
  if (keep) gbl(a.uhist)[(size_t)k * (lp.K + 1) + lp.K] = u;
  const bool reset = fabs(u - uinit) > (double)P;
  if (reset) u = uinit;
  if (a.reset != nullptr && r == 0 && live) gbl(a.reset)[k] = reset ? 1 : 0;

  // window: cells q = 0, 1, 2 are [m-1+q, m+q]; per cell, with a_i the left-end
  // sample minus T_i and d_i the step to the right end, SSD(f) = X0 + 2 f X1 + f^2 X2
  const double fm = floor(u);
  const int m = (int)fm;
  const double f = u - fm;
  double X0[3], X1[3], X2[3];
  {
    double Rv[P + 3];
    fetch_f64<P + 3>(Rv, s_rwin + rr * rwd, xs, rw, Rrow, ox + m - 1, W);
#pragma unroll
    for (int cq = 0; cq < 3; ++cq) {
      double sa = 0.0, saa = 0.0, sd = 0.0, sdd = 0.0, sad = 0.0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const double av = Rv[c + cq] - T[c];
        const double dv = Rv[c + cq + 1] - Rv[c + cq];
        sa += av;
        saa += av * av;
        sd += dv;
        sdd += dv * dv;
        sad += av * dv;
      }
      sa = group_sum_d<G>(row_live ? sa : 0.0);
      saa = group_sum_d<G>(row_live ? saa : 0.0);
      sd = group_sum_d<G>(row_live ? sd : 0.0);
      sdd = group_sum_d<G>(row_live ? sdd : 0.0);
      sad = group_sum_d<G>(row_live ? sad : 0.0);
      X0[cq] = saa - sa * sa / (double)N;
      X1[cq] = sad - sa * sd / (double)N;
      X2[cq] = sdd - sd * sd / (double)N;
    }
  }
  auto ssd = [&](int cq, double fr) { return X0[cq] + fr * (2.0 * X1[cq] + fr * X2[cq]); };
  const double s0 = ssd(1, f), sm1 = ssd(0, f), sp1 = ssd(2, f);
  double smh, sph;
  if (f >= 0.5) {
    smh = ssd(1, f - 0.5);
    sph = ssd(2, f - 0.5);
  } else {
    smh = ssd(0, f + 0.5);
    sph = ssd(1, f + 0.5);
  }
  int inb = 0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const double xr = (double)(ox + c) + u;
    inb += (xr >= 0.0 && xr <= (double)(W - 1)) ? 1 : 0;
  }
  const double rho = (double)(inb * P) / (double)N;
  const bool acc = s0 <= sm1 && s0 <= smh && s0 <= sph && s0 <= sp1 && rho >= (double)lp.valid_ratio;
  if (r == 0 && live) {
    gbl(a.pa.uinit)[k] = uinit;
    gbl(a.pa.pipar)[k] = pipar;
    gbl(a.pa.u)[k] = u;
    gbl(a.pa.ssd0)[k] = s0;
    st4(a.pa.dssd + k, D4{sm1 - s0, smh - s0, sph - s0, sp1 - s0});
    gbl(a.pa.rho)[k] = (float)rho;
    gbl(a.pa.acc)[k] = acc ? 1 : 0;
    gbl(a.pa.hess)[k] = (float)H;
  }
  if (r == 0) {
    s_psum[q] = (live && acc) ? s0 : 0.0;
    s_pcnt[q] = (live && acc) ? 1 : 0;
  }
  __syncthreads();
  if (tid == 0) {
    double ps = 0.0;
    int pc = 0;
    for (int t = 0; t < NPB; ++t) {
      ps += s_psum[t];
      pc += s_pcnt[t];
    }
    gbl(a.part_sum)[blk] = ps;
    gbl(a.part_cnt)[blk] = pc;
  }
}

template <int P>
hipError_t launch_f64(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)P * f64_window_cols(P, lp.S);
  bdis_launch(k_search_f64<P>, dim3(nblocks), dim3(kSearchF64Threads), lds, s, tab, npairs, lp);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pyramid_f64(const PairLevel* tab, int npairs, int nblocks, int level, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  bdis_launch(k_pyr_f64, dim3(nblocks), dim3(kPixThreads), 0, s, tab, npairs, level);
  return hipGetLastError();
}

hipError_t launch_search_f64(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  switch (lp.P) {
    case 3: return launch_f64<3>(tab, npairs, nblocks, lp, s);
    case 4: return launch_f64<4>(tab, npairs, nblocks, lp, s);
    case 5: return launch_f64<5>(tab, npairs, nblocks, lp, s);
    case 6: return launch_f64<6>(tab, npairs, nblocks, lp, s);
    case 7: return launch_f64<7>(tab, npairs, nblocks, lp, s);
    case 8: return launch_f64<8>(tab, npairs, nblocks, lp, s);
    case 9: return launch_f64<9>(tab, npairs, nblocks, lp, s);
    case 10: return launch_f64<10>(tab, npairs, nblocks, lp, s);
    case 11: return launch_f64<11>(tab, npairs, nblocks, lp, s);
    case 12: return launch_f64<12>(tab, npairs, nblocks, lp, s);
    case 13: return launch_f64<13>(tab, npairs, nblocks, lp, s);
    case 14: return launch_f64<14>(tab, npairs, nblocks, lp, s);
    case 15: return launch_f64<15>(tab, npairs, nblocks, lp, s);
    case 16: return launch_f64<16>(tab, npairs, nblocks, lp, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdis
