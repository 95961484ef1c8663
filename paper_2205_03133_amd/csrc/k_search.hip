// Per-patch inverse-compositional 1-D search, Bayesian window and acceptance
// (Eq. 1 with the inverse roles of Sec. III-A; window of Eq. 5-6 with offsets
// -1, -1/2, 0, +1/2, +1 of Sec. IV-A; saddle / in-bounds rejection of
// Sec. III-B and III-F), plus the per-pair reduction that sets sigma_r^(n)
// (Sec. III-B): workgroups write partial sums, which k_reduce (large levels)
// or every fusion workgroup of the level (small levels) adds in a fixed order.
//
// Mapping: one lane per patch row, an aligned group of G = 8 or 16 lanes per
// patch (a DPP quad/half-row/row, so group reductions are 3-4 DPP adds),
// THREADS/G patches of one patch row of one pair per workgroup (THREADS is
// picked per level by the tuner).  The left rows around those
// patches (for the template and its Sobel gradient) and a window of the right
// rows around the patches' starting displacements are staged in LDS once;
// right-image samples outside the window fall back to (clamped) global loads.
//
// Arithmetic.  The uint8 path keeps every image sum exact in int32:
//   with e_i(u) = I_w,i(u) - T_i and J_i = (G_i - sum G / N) / 8 (N = P^2),
//   sum J_i e_i = [(1-f) E(m) + f E(m+1)] / (8 N),  u = m + f, m = floor(u),
//   E(m) = N (sum G R(m) - sum G T) - sum G (sum R(m) - sum T),
//   H = sum J^2 = (N sum G^2 - (sum G)^2) / (64 N),
// so the update u <- u - sum J e / H (Eq. 1, inverse compositional) needs the
// integer correlations of two cells; they are cached per cell, so iterations
// that stay in the same unit cell cost a few scalar flops.  The window SSD of a
// unit cell is an exact quadratic in the fraction f:
//   SSD = [X0 + 2 f X1 + f^2 X2] / N with integer X0, X1, X2 (see below).
// Only the final combinations are rounded (in double).  Every product of two
// image-derived integers has factors within 24 bits (samples 0..255, Sobel sums
// within +-1020), so they use the full-rate 24-bit multiply.
#include "bdis_internal.h"

#include <climits>

namespace bdis {

namespace {

// Exact product of two integers known to lie within +-2^23.
BDIS_DEV int mul24(int a, int b) { return __mul24(a, b); }

// a*b - c*d of int32 values whose products and difference stay below 2^53 in
// magnitude (true for every combination below: at most about 2^36), so the
// double result is exact; full-rate FP64 instead of quarter-rate 64-bit mads.
BDIS_DEV double exact_ab_cd(int a, int b, int c, int d) {
  return fma((double)a, (double)b, -((double)c * (double)d));
}

// Reads N consecutive right-image samples of one row starting at column x:
// from the LDS window when it covers them, else from global memory with the
// column clamped to the image (identical values either way).
template <int N>
BDIS_DEV void fetch_row(int (&v)[N], const uint8_t* win, int xs, int rw, const uint8_t* grow,
                        int x, int W) {
  const int off = x - xs;
  if (off >= 0 && off + N <= rw) {
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = win[off + n];
  } else {
    const auto g = gbl(grow);
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = g[clampi(x + n, 0, W - 1)];
  }
}

// Copies columns [x0, x0 + 4 nd) of image row `rp` (width W) into LDS as nd
// dwords; x0 is a multiple of 4.  Columns outside the row are mapped by
// reflect-101 (REFLECT) or clamping, and then clamped, so every access stays
// in the row.  Interior dwords of a 4-aligned row are single global loads.
template <bool REFLECT>
BDIS_DEV void stage_row(uint32_t* dst, const uint8_t* rp, int W, int x0, int nd, int lane, bool aligned) {
  const auto g = gbl(rp);
  for (int k = lane; k < nd; k += 64) {
    const int c = x0 + 4 * k;
    uint32_t v;
    if (aligned && c >= 0 && c + 3 < W) {
      v = *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(g + c);
    } else {
      v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        int x = c + b;
        x = REFLECT ? reflect101(x, W) : x;
        x = clampi(x, 0, W - 1);
        v |= (uint32_t)g[x] << (8 * b);
      }
    }
    dst[k] = v;
  }
}

template <int P, int THREADS>
__global__ __launch_bounds__(THREADS) void k_search_u8(const PairLevel* tab, int npairs, LevelParams lp) {
  constexpr int G = group_lanes(P);
  constexpr int NPB = THREADS / G;               // patches per workgroup
  constexpr int LTW = ((NPB - 1) * P + P + 2 + 3 + 3) / 4 * 4;  // left tile row bytes (S <= P, 4-aligned start)
  constexpr int RWB = kWinRow;                   // right window row bytes
  constexpr int MARG = P + 4;                    // window margin around the start range
  constexpr int N = P * P;
  constexpr int NWAVES = THREADS / 64;

  __shared__ uint32_t s_left32[(P + 2) * LTW / 4];
  __shared__ uint32_t s_right32[P * RWB / 4];
  __shared__ int s_umin, s_umax;
  __shared__ double s_psum[NPB];
  __shared__ int s_pcnt[NPB];
  const uint8_t* s_left = reinterpret_cast<const uint8_t*>(s_left32);
  const uint8_t* s_right = reinterpret_cast<const uint8_t*>(s_right32);

  const int lb = xcd_block();
  const PairLevel& a = tab[find_pair<1>(tab, npairs, lb)];
  const int blk = lb - a.search0;   // workgroup within the pair
  const int tid = threadIdx.x;
  const int q = tid / G;  // patch slot in the workgroup
  const int r = tid % G;  // patch row of this lane
  const int W = a.g.w, Hh = a.g.h, S = lp.S;
  const int j = blk / a.search_nbx;
  const int i0 = (blk % a.search_nbx) * NPB;
  const bool live = (i0 + q) < a.g.nx;
  const int i = live ? i0 + q : a.g.nx - 1;
  const int ilast = min(i0 + NPB - 1, a.g.nx - 1);
  const int ox = grid_origin(i, W, P, S);
  const int oy = grid_origin(j, Hh, P, S);
  const int ox0 = grid_origin(i0, W, P, S);
  const int oxl = grid_origin(ilast, W, P, S);

  // ---- start from the parent level (Fig. 1): 2 * fused map at the centre
  double uinit = 0.0, pipar = 0.0;
  if (a.par_ubar) {
    const double cx = 0.5 * ((double)ox + 0.5 * (double)(P - 1));
    const double cy = 0.5 * ((double)oy + 0.5 * (double)(P - 1));
    uinit = 2.0 * bilinear(a.par_ubar, a.pw, a.ph, cx, cy);
    pipar = bilinear(a.par_q, a.pw, a.ph, cx, cy);
  }

  if (tid == 0) {
    s_umin = INT_MAX;
    s_umax = INT_MIN;
  }
  const int wave = tid / 64, lane = tid % 64;
  // ---- left tile: image rows oy-1 .. oy+P, columns xa .. oxl+P (reflect-101),
  // xa = (ox0 - 1) rounded down to a multiple of 4
  const int xa = (ox0 - 1) & ~3;
  const int ndl = (oxl + P + 1 - xa + 3) / 4;
  for (int ty = wave; ty < P + 2; ty += NWAVES) {
    const uint8_t* rp = a.L + (size_t)reflect101(oy - 1 + ty, Hh) * a.pitch;
    stage_row<true>(s_left32 + ty * (LTW / 4), rp, W, xa, ndl, lane, ((uintptr_t)rp & 3) == 0);
  }
  __syncthreads();
  if (r == 0 && live) {
    const int mu = (int)floor(uinit);
    atomicMin(&s_umin, mu);
    atomicMax(&s_umax, mu);
  }
  __syncthreads();
  // ---- right window: rows oy .. oy+P-1, columns xs .. xs+rw-1 (clamped to the
  // image), xs a multiple of 4
  const int xs = (ox0 + s_umin - MARG) & ~3;
  const int ndr = min((oxl + P + s_umax + MARG + 2 - xs + 3) / 4, RWB / 4);
  const int rw = 4 * ndr;
  for (int ty = wave; ty < P; ty += NWAVES) {
    const uint8_t* rp = a.R + (size_t)(oy + ty) * a.pitch;
    stage_row<false>(s_right32 + ty * (RWB / 4), rp, W, xs, ndr, lane, ((uintptr_t)rp & 3) == 0);
  }
  __syncthreads();

  // ---- template row: T and Sobel-x G (integer), rows r >= P are idle lanes
  const bool row_live = r < P;
  const int rr = row_live ? r : P - 1;
  int T[P], Gx[P];
  {
    const uint8_t* l0 = s_left + rr * LTW + (ox - 1 - xa);
    const uint8_t* l1 = l0 + LTW;
    const uint8_t* l2 = l1 + LTW;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T[c] = l1[c + 1];
      Gx[c] = (l0[c + 2] - l0[c]) + 2 * (l1[c + 2] - l1[c]) + (l2[c + 2] - l2[c]);
    }
  }
  int sG = 0, sT = 0, sGG = 0, sGT = 0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    sG += Gx[c];
    sT += T[c];
    sGG += mul24(Gx[c], Gx[c]);
    sGT += mul24(Gx[c], T[c]);
  }
  if (!row_live) sG = sT = sGG = sGT = 0;
  sG = group_sum<G>(sG);
  sT = group_sum<G>(sT);
  sGG = group_sum<G>(sGG);
  sGT = group_sum<G>(sGT);
  const double Hs = exact_ab_cd(N, sGG, sG, sG);  // = 64 N H, exact
  const double H = Hs / (64.0 * N);
  const bool invert = H >= kEpsH;
  const double step = invert ? 8.0 / Hs : 0.0;

  const uint8_t* win = s_right + rr * RWB;
  const uint8_t* grow = a.R + (size_t)(oy + rr) * a.pitch;

  // ---- K inverse-compositional iterations (Eq. 1), cached cell correlations
  double u = uinit;
  if (invert) {
    int mc = INT_MIN;
    double E0 = 0.0, E1 = 0.0;
    for (int t = 0; t < lp.K; ++t) {
      const double fm = floor(u);
      const int m = (int)fm;
      const double f = u - fm;
      if (m != mc) {
        int Rv[P + 1];
        fetch_row<P + 1>(Rv, win, xs, rw, grow, ox + m, W);
        int cg0 = 0, cs0 = 0, cg1 = 0;
#pragma unroll
        for (int c = 0; c < P; ++c) {
          cg0 += mul24(Gx[c], Rv[c]);
          cs0 += Rv[c];
          cg1 += mul24(Gx[c], Rv[c + 1]);
        }
        int cs1 = cs0 + Rv[P] - Rv[0];
        if (!row_live) cg0 = cs0 = cg1 = cs1 = 0;
        cg0 = group_sum<G>(cg0);
        cs0 = group_sum<G>(cs0);
        cg1 = group_sum<G>(cg1);
        cs1 = group_sum<G>(cs1);
        E0 = exact_ab_cd(N, cg0 - sGT, sG, cs0 - sT);
        E1 = exact_ab_cd(N, cg1 - sGT, sG, cs1 - sT);
        mc = m;
      }
      u -= ((1.0 - f) * E0 + f * E1) * step;
    }
  }
  // patch searching threshold: a run-away patch falls back to its start
  if (fabs(u - uinit) > (double)P) u = uinit;

  // ---- window SSDs.  Cell q in {0,1,2} is [m-1+q, m+q]; with a_i the sample
  // at the cell's left end minus T_i and d_i the step to its right end,
  // e_i(f) = a_i + f d_i and SSD(f) = sum (e - mean e)^2 = [X0 + 2fX1 + f^2X2]/N,
  // X0 = N sum a^2 - (sum a)^2, X1 = N sum ad - sum a sum d, X2 = N sum d^2 - (sum d)^2.
  const double fm = floor(u);
  const int m = (int)fm;
  const double f = u - fm;
  double X0[3], X1[3], X2[3];
  {
    int Rv[P + 3], D[P + 2];
    fetch_row<P + 3>(Rv, win, xs, rw, grow, ox + m - 1, W);
#pragma unroll
    for (int c = 0; c < P + 2; ++c) D[c] = Rv[c + 1] - Rv[c];
    int sa = 0;
#pragma unroll
    for (int c = 0; c < P; ++c) sa += Rv[c] - T[c];
#pragma unroll
    for (int cq = 0; cq < 3; ++cq) {
      // sum of d telescopes; sum of a slides by one sample per cell
      if (cq > 0) sa += Rv[cq + P - 1] - Rv[cq - 1];
      int sd = Rv[cq + P] - Rv[cq];
      int saa = 0, sdd = 0, sad = 0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const int av = Rv[c + cq] - T[c];
        saa += mul24(av, av);
        sdd += mul24(D[c + cq], D[c + cq]);
        sad += mul24(av, D[c + cq]);
      }
      const int ga = group_sum<G>(row_live ? sa : 0);
      saa = group_sum<G>(row_live ? saa : 0);
      sd = group_sum<G>(row_live ? sd : 0);
      sdd = group_sum<G>(row_live ? sdd : 0);
      sad = group_sum<G>(row_live ? sad : 0);
      X0[cq] = exact_ab_cd(N, saa, ga, ga);
      X1[cq] = exact_ab_cd(N, sad, ga, sd);
      X2[cq] = exact_ab_cd(N, sdd, sd, sd);
    }
  }
  constexpr double kInvN = 1.0 / (double)N;  // SSD = [X0 + 2 f X1 + f^2 X2] / N, by the rounded 1/N
  auto ssd = [&](int cq, double fr) { return (X0[cq] + fr * (2.0 * X1[cq] + fr * X2[cq])) * kInvN; };
  const double s0 = ssd(1, f);
  const double sm1 = ssd(0, f);
  const double sp1 = ssd(2, f);
  double smh, sph;
  if (f >= 0.5) {
    smh = ssd(1, f - 0.5);
    sph = ssd(2, f - 0.5);
  } else {
    smh = ssd(0, f + 0.5);
    sph = ssd(1, f + 0.5);
  }
  // in-bounds count of the columns c = 0..P-1 with (ox + c) + u in [0, W-1]:
  // the rounded sample position is monotone in c, so the count is the length
  // of an interval whose ends are found by testing the same rounded predicate
  // around the real-valued boundaries.
  auto inside_lo = [&](int c) { return (double)(ox + c) + u >= 0.0; };
  auto inside_hi = [&](int c) { return (double)(ox + c) + u <= (double)(W - 1); };
  int clo = (int)fmin(fmax(ceil(-(double)ox - u), 0.0), (double)P);
  while (clo > 0 && inside_lo(clo - 1)) --clo;
  while (clo < P && !inside_lo(clo)) ++clo;
  int chi = (int)fmin(fmax(floor((double)(W - 1 - ox) - u), -1.0), (double)(P - 1));
  while (chi < P - 1 && inside_hi(chi + 1)) ++chi;
  while (chi >= 0 && !inside_hi(chi)) --chi;
  const int inb = chi >= clo ? chi - clo + 1 : 0;
  const double rho = (double)(inb * P) / (double)N;
  const bool acc = s0 <= sm1 && s0 <= smh && s0 <= sph && s0 <= sp1 && rho >= (double)lp.valid_ratio;

  const int k = j * a.g.nx + i;
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

  // ---- per-workgroup partial of the level reduction: sum of SSD(0) and count
  // over accepted patches (summed per pair, in workgroup order, by k_reduce)
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

// One workgroup per pair: the level scalars (sigma_r^2, tau, pooled residual,
// accepted count) from the search partials.
__global__ __launch_bounds__(256) void k_reduce(const PairLevel* tab, LevelParams lp) {
  __shared__ double s_red[256];
  __shared__ long long s_redc[256];
  const PairLevel& a = tab[blockIdx.x];
  double sc[4];
  pair_scalars(a, lp, s_red, s_redc, sc);
  if (threadIdx.x == 0)
    for (int t = 0; t < 4; ++t) gbl(a.scal)[t] = sc[t];
}

template <int P>
hipError_t launch_p(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, int threads,
                    hipStream_t s) {
  switch (threads) {
    case 64: hipLaunchKernelGGL((k_search_u8<P, 64>), dim3(nblocks), dim3(64), 0, s, tab, npairs, lp); break;
    case 128: hipLaunchKernelGGL((k_search_u8<P, 128>), dim3(nblocks), dim3(128), 0, s, tab, npairs, lp); break;
    case 256: hipLaunchKernelGGL((k_search_u8<P, 256>), dim3(nblocks), dim3(256), 0, s, tab, npairs, lp); break;
    case 512: hipLaunchKernelGGL((k_search_u8<P, 512>), dim3(nblocks), dim3(512), 0, s, tab, npairs, lp); break;
    case 1024: hipLaunchKernelGGL((k_search_u8<P, 1024>), dim3(nblocks), dim3(1024), 0, s, tab, npairs, lp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reduce(const PairLevel* tab, int npairs, const LevelParams& lp, hipStream_t s) {
  if (npairs <= 0 || lp.inline_prob) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(npairs), dim3(256), 0, s, tab, lp);
  return hipGetLastError();
}

hipError_t launch_search(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, int threads,
                         hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  switch (lp.P) {
    case 3: return launch_p<3>(tab, npairs, nblocks, lp, threads, s);
    case 4: return launch_p<4>(tab, npairs, nblocks, lp, threads, s);
    case 5: return launch_p<5>(tab, npairs, nblocks, lp, threads, s);
    case 6: return launch_p<6>(tab, npairs, nblocks, lp, threads, s);
    case 7: return launch_p<7>(tab, npairs, nblocks, lp, threads, s);
    case 8: return launch_p<8>(tab, npairs, nblocks, lp, threads, s);
    case 9: return launch_p<9>(tab, npairs, nblocks, lp, threads, s);
    case 10: return launch_p<10>(tab, npairs, nblocks, lp, threads, s);
    case 11: return launch_p<11>(tab, npairs, nblocks, lp, threads, s);
    case 12: return launch_p<12>(tab, npairs, nblocks, lp, threads, s);
    case 13: return launch_p<13>(tab, npairs, nblocks, lp, threads, s);
    case 14: return launch_p<14>(tab, npairs, nblocks, lp, threads, s);
    case 15: return launch_p<15>(tab, npairs, nblocks, lp, threads, s);
    case 16: return launch_p<16>(tab, npairs, nblocks, lp, threads, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdis
