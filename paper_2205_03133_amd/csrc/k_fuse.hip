// Patch probability and fusion of the overlapping patches into the level maps.
//
// Patch record (computed by the fusion workgroups for the patches covering
// their tile; the tile holding a patch's origin stores it): window posterior
// post = p0 / sum_d p_d with
//   p_d = exp(-SSD_d / tau), tau = 2 sigma_r^2 s^2 (Eq. 5-6), in the stable
//   form 1 / sum_d exp(-(SSD_d - SSD_0) / tau); the level's contribution
//   Gamma_n * post plus the probability propagated from the parent level
//   (Eq. 11-12); at the finest level the patch variance of Eq. 15-17, whose
//   Gauss-Newton fixed point is the least-squares line of ln p on d^2:
//   sigma_k^2 = tau / (2 kappa), kappa the slope of SSD_d on d^2.
//
// k_fuse (gather over 64 x 4, 64 x 16 or 64 x 32 pixel tiles): over the accepted patches
//   covering the pixel, in ascending patch index, weights W_k = M(x - o_k) pi_k
//   with the spatial mixture mask M(a, b) = m(a) m(b),
//   m(a) = sum_c exp(-(a - c)^2 / (2 sigma_s^2)) (Eq. 9-10, unit mixture
//   weights); fused displacement sum W u / sum W (Eq. 13, normalised),
//   confidence sum M pi / sum M, variance sum (W / sum W)^2 sigma_k^2 (Eq. 18,
//   disparity form).  A gather has no atomics, so results are deterministic.
//   With the mask weights (fusion 0, 2) the sums are evaluated separably: the
//   mask factors into m(a) m(b), so the column sums over the covering patch
//   columns are formed once per staged patch row and tile column in LDS and
//   the pixel rows of the tile combine them.
#include "bdis_internal.h"
#include "fuse_common.h"

namespace bdis {

namespace {

// One lane per patch: the patch records of a level (used when the level is
// large enough that computing them once beats recomputing them per tile).
__global__ __launch_bounds__(kProbThreads) void k_prob(const PairLevel* tab, int npairs, LevelParams lp) {
  const PairLevel& a = tab[find_pair<2>(tab, npairs, xcd_block())];
  const int k = (xcd_block() - a.prob0) * kProbThreads + (int)threadIdx.x;
  if (k >= a.g.nx * a.g.ny) return;
  st4(a.pa.dens + k, patch_record(a, lp, lp.level, patch_raw(a, lp, (size_t)k), gbl(a.scal)[1]));
}

// Records staged per workgroup: the patches covering a tile (about 25 x 5
// for 64 x 4, 25 x 9 for 64 x 16 and 25 x 15 for 64 x 32 at patch 8, stride 3;
// tiles that cover more than the level's lp.fuse_rec use direct loads).  The
// record arrays and the separable column sums live in dynamic LDS sized per
// level (fuse_lds_bytes), so small strides do not cost every level occupancy.
constexpr int kMaxRec = kFuseMaxRec;

// INLINE: the patch records are computed here (small levels) instead of read
// from a preceding k_prob launch.
template <bool INLINE, int TY>
__global__ __launch_bounds__(fuse_threads(TY)) void k_fuse(const PairLevel* __restrict__ tab, int npairs, LevelParams lp) {
  constexpr int kThreads = fuse_threads(TY);
  constexpr int kRowsPerLane = TY / (kThreads / kFuseTx);
  __shared__ double s_m[kMaxPatch];
  extern __shared__ double s_fdyn[];
  const int rec_cap = lp.fuse_rec;
  double* const s_u = s_fdyn;
  double* const s_w = s_u + rec_cap;
  double* const s_v = s_w + rec_cap;
  double* const s_A = s_v + rec_cap;  // [lp.fuse_sep][4][kFuseTx]
  const int lb = xcd_block();
  const PairLevel& a = tab[find_pair<3>(tab, npairs, lb)];
  const int tid = threadIdx.x;
  const int P = lp.P, S = lp.S;
  if (tid == 0)
#pragma unroll
    for (int c = 0; c < kMaxPatch; ++c) s_m[c] = lp.mask[c];
  const int tiles_x = (a.g.w + kFuseTx - 1) / kFuseTx;
  const int t = lb - a.fuse0;
  const int x0 = (t % tiles_x) * kFuseTx, y0 = (t / tiles_x) * TY;
  const int x1 = min(x0 + kFuseTx, a.g.w) - 1, y1 = min(y0 + TY, a.g.h) - 1;
  // patch index ranges covering the tile: [lo, hi] plus the border patch `ex`
  int ilo, ihi, iex, jlo, jhi, jex, dummy0, dummy1, dummy2;
  cover_range(x0, a.g.w, P, S, a.g.nx, ilo, dummy0, dummy1);
  cover_range(x1, a.g.w, P, S, a.g.nx, dummy2, ihi, iex);
  cover_range(y0, a.g.h, P, S, a.g.ny, jlo, dummy0, dummy1);
  cover_range(y1, a.g.h, P, S, a.g.ny, dummy2, jhi, jex);
  const int ni = ihi - ilo + 1 + (iex >= 0 ? 1 : 0);
  const int nj = jhi - jlo + 1 + (jex >= 0 ? 1 : 0);
  const bool staged = ni * nj <= rec_cap;
  // staged records: slot s of this lane is record tid + s * kThreads
  constexpr int kSlots = (kMaxRec + kThreads - 1) / kThreads;
  auto rec_index = [&](int r, int& i, int& j) {
    const int rj = div_small(r, ni), ri = r - rj * ni;
    i = ilo + ri <= ihi ? ilo + ri : iex;
    j = jlo + rj <= jhi ? jlo + rj : jex;
  };
  double tau = 0.0;
  if (INLINE) {
    // the search results of the staged patches are loaded before the level
    // reduction, so both global round trips overlap
    PatchRaw raw[kSlots];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const int r = tid + sl * kThreads;
      if (staged && r < ni * nj) {
        int i, j;
        rec_index(r, i, j);
        raw[sl] = patch_raw(a, lp, (size_t)j * a.g.nx + i);
      }
    }
    __shared__ double s_red[256];
    __shared__ long long s_redc[256];
    double sc[4];
    pair_scalars(a, lp, s_red, s_redc, sc);
    tau = sc[1];
    if (t == 0 && tid < 4) gbl(a.scal)[tid] = sc[tid];  // kept for the backward pass and debug
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
      const int r = tid + sl * kThreads;
      if (staged && r < ni * nj) {
        int i, j;
        rec_index(r, i, j);
        const D4 d = patch_record(a, lp, lp.level, raw[sl], tau);
        // the tile holding the patch origin keeps its record (backward pass, debug dumps)
        const int ox = grid_origin(i, a.g.w, P, S), oy = grid_origin(j, a.g.h, P, S);
        if (lp.keep && ox >= x0 && ox <= x1 && oy >= y0 && oy <= y1) st4(a.pa.dens + (size_t)j * a.g.nx + i, d);
        s_u[r] = d.x;
        s_w[r] = d.y;
        s_v[r] = d.z;
      }
    }
  } else if (staged) {
    for (int r = tid; r < ni * nj; r += kThreads) {
      int i, j;
      rec_index(r, i, j);
      const D4 d = ld4(a.pa.dens + (size_t)j * a.g.nx + i);
      s_u[r] = d.x;
      s_w[r] = d.y;
      s_v[r] = d.z;
    }
  }
  __syncthreads();
  // Separable form (mask weights, fusion 0 and 2): the mask is m(x - o_x) m(y - o_y),
  // so per staged patch row j and tile column the sums over the covering patch
  // columns i are formed once and shared by the tile's pixel rows:
  //   A0 = sum_i m_x pi, A1 = sum_i m_x pi u, A2 = sum_i m_x, A3 = sum_i (m_x pi)^2 sigma^2,
  // then z = sum_j m_y A0, ..., zv = sum_j m_y^2 A3 per pixel.
  const bool separable = staged && lp.fusion != 1 && nj <= lp.fuse_sep;
  if (separable) {
    for (int e = tid; e < nj * kFuseTx; e += kThreads) {
      const int rj = e / kFuseTx, xl = e - rj * kFuseTx;
      const int xc = x0 + xl;
      ColSums cs;
      if (xc < a.g.w) {
        int clo, chi, cex;
        cover_range(xc, a.g.w, P, S, a.g.nx, clo, chi, cex);
        const int cend = cex >= 0 ? chi + 1 : chi;
        for (int ii = clo; ii <= cend; ++ii) {
          const int i = ii <= chi ? ii : cex;
          const int r = rj * ni + (i <= ihi ? i - ilo : ni - 1);
          const double dw = s_w[r];
          if (dw < 0.0) continue;  // rejected patch
          col_add(cs, lp.fusion == 2 ? 1.0 : s_m[xc - grid_origin(i, a.g.w, P, S)], dw, s_u[r], s_v[r]);
        }
      }
      double* const A = s_A + rj * (4 * kFuseTx) + xl;
      A[0] = cs.a0;
      A[kFuseTx] = cs.a1;
      A[2 * kFuseTx] = cs.a2;
      A[3 * kFuseTx] = cs.a3;
    }
    __syncthreads();
  }
  // every lane fuses kRowsPerLane pixels of its tile column
  const int xl = tid % kFuseTx;
  const int x = x0 + xl;
  const bool finest = lp.level == lp.finest;
  // the table fields the pixel loop uses, read once: a scalar load of each
  // would otherwise sit inside the loop, after the stores of every pixel
  double* const o_ubar = a.ubar;
  double* const o_qmap = a.qmap;
  float* const o_disp = a.disparity;
  float* const o_conf = a.confidence;
  float* const o_var = a.variance;
  double* const o_zmap = a.zmap;
  auto fuse_pixel = [&](int y) {
    int pilo = 0, pihi = -1, piex = -1, pjlo = 0, pjhi = -1, pjex = -1;
    cover_range(y, a.g.h, P, S, a.g.ny, pjlo, pjhi, pjex);
    PixSums ps;
    double zq = 0.0;  // Eq. 2 weights only: sum M pi (with mask weights it equals sum W)
    const int jend = pjex >= 0 ? pjhi + 1 : pjhi;
    if (separable) {
      for (int jj = pjlo; jj <= jend; ++jj) {
        const int j = jj <= pjhi ? jj : pjex;
        const int rj = j <= jhi ? j - jlo : nj - 1;
        const double my = lp.fusion == 2 ? 1.0 : s_m[y - grid_origin(j, a.g.h, P, S)];
        const double* const A = s_A + rj * (4 * kFuseTx) + xl;
        row_add(ps, my, A[0], A[kFuseTx], A[2 * kFuseTx], A[3 * kFuseTx]);
      }
    }
    if (!separable) cover_range(x, a.g.w, P, S, a.g.nx, pilo, pihi, piex);
    // Eq. 2 (DIS weights): this pixel's left value and its right-image row
    double lx = 0.0;
    if (lp.fusion == 1) lx = a.Ld ? gbl(a.Ld)[(size_t)y * a.dpitch + x] : (double)gbl(a.L)[(size_t)y * a.pitch + x];
    const int iend = piex >= 0 ? pihi + 1 : pihi;
    for (int jj = pjlo; !separable && jj <= jend; ++jj) {
      const int j = jj <= pjhi ? jj : pjex;
      const double mb = lp.fusion == 2 ? 1.0 : s_m[y - grid_origin(j, a.g.h, P, S)];
      const int rj = j <= jhi ? j - jlo : nj - 1;  // row of j in the staged block
      ColSums cs;  // mask weights: this patch row's sums, as the separable form forms them
      for (int ii = pilo; ii <= iend; ++ii) {
        const int i = ii <= pihi ? ii : piex;
        double du, dw, dv;
        if (staged) {
          const int r = rj * ni + (i <= ihi ? i - ilo : ni - 1);
          du = s_u[r];
          dw = s_w[r];
          dv = s_v[r];
        } else {
          const size_t k = (size_t)j * a.g.nx + i;
          D4 d;
          if (INLINE) {
            d = patch_record(a, lp, lp.level, patch_raw(a, lp, k), tau);
            if (lp.keep && x == grid_origin(i, a.g.w, P, S) && y == grid_origin(j, a.g.h, P, S)) st4(a.pa.dens + k, d);
          } else {
            d = ld4(a.pa.dens + k);
          }
          du = d.x;
          dw = d.y;
          dv = d.z;
        }
        if (dw < 0.0) continue;  // rejected patch
        if (lp.fusion != 1) {
          col_add(cs, lp.fusion == 2 ? 1.0 : s_m[x - grid_origin(i, a.g.w, P, S)], dw, du, dv);
          continue;
        }
        {
          // 1 / max(1, r^2), r = I_r(x + u) - I_l(x): linear warp, indices clamped to the row
          const double fm = floor(du);
          const int mm = (int)fm;
          const double fr = du - fm;
          const int xa = clampi(x + mm, 0, a.g.w - 1), xb = clampi(x + mm + 1, 0, a.g.w - 1);
          double ra, rb;
          if (a.Rd) {
            ra = gbl(a.Rd)[(size_t)y * a.dpitch + xa];
            rb = gbl(a.Rd)[(size_t)y * a.dpitch + xb];
          } else {
            ra = (double)gbl(a.R)[(size_t)y * a.pitch + xa];
            rb = (double)gbl(a.R)[(size_t)y * a.pitch + xb];
          }
          const double r = (1.0 - fr) * ra + fr * rb - lx;
          const double wk = 1.0 / fmax(1.0, r * r);
          const double m = s_m[x - grid_origin(i, a.g.w, P, S)] * mb;
          ps.z += wk;
          ps.zu += wk * du;
          ps.zm += m;
          zq += m * dw;
          ps.zv += wk * wk * dv;
        }
      }
      if (lp.fusion != 1) row_add(ps, mb, cs.a0, cs.a1, cs.a2, cs.a3);
    }
    if (lp.fusion != 1) zq = ps.z;
    const double z = ps.z, zu = ps.zu, zm = ps.zm, zv = ps.zv;
    const size_t idx = (size_t)y * a.g.w + x;
    double ub, qv;
    bool valid = z > 0.0;
    // the normalisations by sum W (displacement and variance) and by sum M
    // (confidence) through refined reciprocals
    const double rz = valid ? recip(z) : 0.0;
    if (valid) {
      ub = zu * rz;
      qv = zq * recip(zm);
    } else if (finest) {
      ub = __builtin_nan("");
      qv = 0.0;
    } else if (a.par_ubar) {
      // hole above the finest level: the parent estimate
      ub = 2.0 * bilinear(a.par_ubar, a.pw, a.ph, 0.5 * x, 0.5 * y);
      qv = bilinear(a.par_q, a.pw, a.ph, 0.5 * x, 0.5 * y);
    } else {
      ub = 0.0;
      qv = 0.0;
    }
    if (o_zmap) {  // training contexts keep the fusion sums for the backward pass
      gbl(o_zmap)[idx] = valid ? z : 0.0;
      gbl(a.smmap)[idx] = zm;
      if (finest) {
        gbl(a.ubar_keep)[idx] = ub;
        gbl(a.qmap_keep)[idx] = qv;
        if (a.vmap) gbl(a.vmap)[idx] = (valid && lp.variance) ? zv * (rz * rz) : 0.0;
      }
    }
    if (!finest) {
      gbl(o_ubar)[idx] = ub;
      gbl(o_qmap)[idx] = qv;
      return;
    }
    if (lp.prob_thresh > 0.0f && qv < (double)lp.prob_thresh) valid = false;
    const float nan = __builtin_nanf("");
    gbl(o_disp)[idx] = valid ? (float)(-ub) : nan;
    if (o_conf) gbl(o_conf)[idx] = valid ? (float)qv : 0.0f;
    if (o_var) gbl(o_var)[idx] = (valid && lp.variance) ? (float)(zv * (rz * rz)) : nan;
  };
  // A wavefront holds one pixel row of the tile, so y and everything derived
  // from it (covering patch rows, vertical mask weights) are wave-uniform.
  static_assert(kFuseTx == 64, "one tile row per wavefront");
  if (x < a.g.w)
    for (int rr = 0; rr < kRowsPerLane; ++rr) {
      const int y = __builtin_amdgcn_readfirstlane(y0 + tid / kFuseTx + rr * (kThreads / kFuseTx));
      if (y < a.g.h) fuse_pixel(y);
    }
}

// Finest level f > 0, per output pixel: bilinear sample of the level-f maps at
// (x / 2^f, y / 2^f) (the pyramid keeps even pixels, so level-0 pixel 2^f k
// lies on level-f pixel k), clamped at the last row and column; disparity
// scaled by 2^f, variance by 4^f.  Invalid when a sample with nonzero weight is.
__global__ __launch_bounds__(kPixThreads) void k_upsample(const PairLevel* tab, int npairs) {
  const PairLevel& a = tab[find_pair<4>(tab, npairs, (int)blockIdx.x)];
  const int idx = ((int)blockIdx.x - a.up0) * kPixThreads + (int)threadIdx.x;
  const int w = a.g.w, h = a.g.h;
  if (idx >= w * h) return;
  const int y = idx / w, x = idx - y * w;
  const double sc = (double)(1 << a.fshift);
  const double sx = x / sc, sy = y / sc;
  const int x0 = (int)floor(sx), y0 = (int)floor(sy);
  const double ax = sx - x0, ay = sy - y0;
  const int xs[2] = {x0, min(x0 + 1, a.fw - 1)};
  const int ys[2] = {y0, min(y0 + 1, a.fh - 1)};
  const double wx[2] = {1.0 - ax, ax}, wy[2] = {1.0 - ay, ay};
  const auto fd = gbl(a.fdisp), fv = gbl(a.fvar), fc = gbl(a.fconf);
  double d = 0.0, v = 0.0, c = 0.0;
  bool ok = true;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const double wt = wx[e] * wy[b];
      if (wt == 0.0) continue;
      const size_t k = (size_t)ys[b] * a.fw + xs[e];
      const float dk = fd[k];
      if (dk != dk) ok = false;
      d += wt * (double)dk;
      v += wt * (double)fv[k];
      c += wt * (double)fc[k];
    }
  const float nan = __builtin_nanf("");
  gbl(a.disparity)[idx] = ok ? (float)(sc * d) : nan;
  if (a.variance) gbl(a.variance)[idx] = ok ? (float)(sc * sc * v) : nan;
  if (a.confidence) gbl(a.confidence)[idx] = ok ? (float)c : 0.0f;
}

// Per pixel: depth fb / d and its variance (fb)^2 / d^4 var (Eq. 14, 18).
__global__ __launch_bounds__(kPixThreads) void k_depth(const float* disp, const float* var, int w, int h,
                                                       int pitch, float fb, float* depth, float* dvar) {
  const int idx = (int)blockIdx.x * kPixThreads + (int)threadIdx.x;
  if (idx >= w * h) return;
  const int y = idx / w, x = idx - y * w;
  const double d = (double)gbl(disp)[(size_t)y * pitch + x];
  const bool ok = d > 0.0;
  const double z = (double)fb / d;
  gbl(depth)[idx] = ok ? (float)z : __builtin_nanf("");
  if (dvar) {
    const double v = (double)gbl(var)[(size_t)y * pitch + x];
    gbl(dvar)[idx] = ok ? (float)(z * z / (d * d) * v) : __builtin_nanf("");
  }
}

// Per pixel: does the reference disparity lie within k standard deviations?
// Block sums in LDS, one integer atomic per block (order-independent).
__global__ __launch_bounds__(kPixThreads) void k_coverage(const float* disp, const float* var, const float* ref,
                                                          const uint8_t* valid, int w, int h, int pitch, double k,
                                                          unsigned long long* counts) {
  __shared__ unsigned s_c[kPixThreads], s_t[kPixThreads];
  const int tid = threadIdx.x;
  const int idx = (int)blockIdx.x * kPixThreads + tid;
  unsigned c = 0, t = 0;
  if (idx < w * h) {
    const int y = idx / w, x = idx - y * w;
    const size_t o = (size_t)y * pitch + x;
    const double d = (double)gbl(disp)[o], v = (double)gbl(var)[o], r = (double)gbl(ref)[o];
    const bool use = (!valid || gbl(valid)[o] != 0) && isfinite(d) && isfinite(v) && isfinite(r) && v >= 0.0;
    if (use) {
      t = 1;
      c = fabs(d - r) <= k * sqrt(v) ? 1 : 0;
    }
  }
  s_c[tid] = c;
  s_t[tid] = t;
  __syncthreads();
  for (int off = kPixThreads / 2; off > 0; off >>= 1) {
    if (tid < off) {
      s_c[tid] += s_c[tid + off];
      s_t[tid] += s_t[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0 && s_t[0] > 0) {
    atomicAdd(counts, (unsigned long long)s_c[0]);
    atomicAdd(counts + 1, (unsigned long long)s_t[0]);
  }
}

// Zeroes the two counters (a kernel, so that the call stays capturable).
__global__ void k_zero2(unsigned long long* counts) {
  if (threadIdx.x < 2) counts[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_prob(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  if (nblocks <= 0 || lp.inline_prob) return hipSuccess;
  bdis_launch(k_prob, dim3(nblocks), dim3(kProbThreads), 0, s, tab, npairs, lp);
  return hipGetLastError();
}

hipError_t launch_fuse(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (!fuse_ty_ok(lp.fuse_ty) || lp.fuse_rec < 0 || lp.fuse_rec > kFuseMaxRec || lp.fuse_sep < 0 ||
      lp.fuse_sep > fuse_sep_rows(lp.fuse_ty))
    return hipErrorInvalidValue;
  const dim3 threads(fuse_threads(lp.fuse_ty));
  const size_t lds = fuse_lds_bytes(lp.fuse_rec, lp.fuse_sep);
  const bool inl = lp.inline_prob != 0;
  switch (lp.fuse_ty) {
    case kFuseTyHuge:
      if (inl) bdis_launch((k_fuse<true, kFuseTyHuge>), dim3(nblocks), threads, lds, s, tab, npairs, lp);
      else bdis_launch((k_fuse<false, kFuseTyHuge>), dim3(nblocks), threads, lds, s, tab, npairs, lp);
      break;
    case kFuseTyTall:
      if (inl) bdis_launch((k_fuse<true, kFuseTyTall>), dim3(nblocks), threads, lds, s, tab, npairs, lp);
      else bdis_launch((k_fuse<false, kFuseTyTall>), dim3(nblocks), threads, lds, s, tab, npairs, lp);
      break;
    default:
      if (inl) bdis_launch((k_fuse<true, kFuseTyShort>), dim3(nblocks), threads, lds, s, tab, npairs, lp);
      else bdis_launch((k_fuse<false, kFuseTyShort>), dim3(nblocks), threads, lds, s, tab, npairs, lp);
  }
  return hipGetLastError();
}

hipError_t launch_upsample(const PairLevel* tab, int npairs, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  bdis_launch(k_upsample, dim3(nblocks), dim3(kPixThreads), 0, s, tab, npairs);
  return hipGetLastError();
}

hipError_t launch_depth(const float* disp, const float* var, int w, int h, int pitch, float fb, float* depth,
                        float* dvar, hipStream_t s) {
  const long n = (long)w * h;
  bdis_launch(k_depth, dim3((unsigned)((n + kPixThreads - 1) / kPixThreads)), dim3(kPixThreads), 0, s, disp,
                     var, w, h, pitch, fb, depth, dvar);
  return hipGetLastError();
}

hipError_t launch_coverage(const float* disp, const float* var, const float* ref, const uint8_t* valid, int w,
                           int h, int pitch, double k, unsigned long long* counts, hipStream_t s) {
  bdis_launch(k_zero2, dim3(1), dim3(64), 0, s, counts);
  const long n = (long)w * h;
  bdis_launch(k_coverage, dim3((unsigned)((n + kPixThreads - 1) / kPixThreads)), dim3(kPixThreads), 0, s,
                     disp, var, ref, valid, w, h, pitch, k, counts);
  return hipGetLastError();
}

}  // namespace bdis
