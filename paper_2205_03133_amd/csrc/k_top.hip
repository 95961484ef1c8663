// The coarsest level of each pair in one workgroup: the level's pyramid step
// (binomial 5 x 5, reflect-101, rounded), the patch search (Eq. 1, window of
// Eq. 5-6, acceptance of Sec. III-B / III-F), the level sum behind sigma_r
// (Sec. III-B), the patch records (Eq. 5-6, 11-12) and the fusion into the
// level maps (Eq. 9-13).  This is the work of that level's pyramid, search and
// fusion launches without the launch boundaries between them: the level is
// small (at most a few thousand pixels), so one workgroup holds both level
// images, every patch of the level (one aligned lane group each) and the
// records in LDS, and its barriers replace the kernel boundaries.
//
// Every step goes through the same arithmetic as the per-phase kernels (the
// shared per-patch search, the exact fixed-point level sum, patch_record and
// the fusion sums in patch order), so the outputs are the same bits.
#include "fuse_common.h"
#include "search_common.h"

namespace bdis {

namespace {

constexpr int kTopThreads = 1024;
constexpr int kTopWaves = kTopThreads / 64;
constexpr int kTopSrcWordsPerThread = 8;  // staged words of the level below per thread (at most 32 KB)

template <int P, int G>
__global__ __launch_bounds__(kTopThreads) void k_top(const PairLevel* tab, LevelParams lp, TopShape ts) {
  constexpr int MARG = P + 4;  // right-window margin beyond the image (as the search launch's full rows)
  extern __shared__ __align__(16) unsigned char s_top[];
  __shared__ double s_m[kMaxPatch];
  __shared__ unsigned long long s_wlo[kTopWaves], s_whi[kTopWaves];
  __shared__ int s_wcnt[kTopWaves];

  const PairLevel& a = tab[blockIdx.x];
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int W = a.g.w, Hh = a.g.h, S = lp.S, nx = a.g.nx, ny = a.g.ny, np = nx * ny;
  const int sw = a.sw, sh = a.sh;
  uint8_t* const s_srcL = s_top;
  uint8_t* const s_srcR = s_top + sh * ts.sw4;  // this pair's rows of the left view, then of the right
  uint8_t* const s_imgL = s_top + ts.off_img;
  uint8_t* const s_imgR = s_imgL + ts.img_px;
  uint8_t* const s_left = s_top + ts.off_left;
  uint8_t* const s_right = s_top + ts.off_right;
  double* const s_pu = reinterpret_cast<double*>(s_top + ts.off_pat);
  D4* const s_pd = reinterpret_cast<D4*>(s_pu + ts.np_max);
  double* const s_u = reinterpret_cast<double*>(s_pd + ts.np_max);
  double* const s_w = s_u + ts.np_max;
  double* const s_v = s_w + ts.np_max;
  unsigned long long* const s_psum = reinterpret_cast<unsigned long long*>(s_v + ts.np_max);
  int* const s_pacc = reinterpret_cast<int*>(s_psum + ts.np_max);
  if (tid < kMaxPatch) s_m[tid] = lp.mask[tid];

  // ---- 1. the level below, both views, into LDS (columns past its width
  // clamped): every thread issues all its loads before it stores any, so the
  // whole level is one global round trip
  {
    const int swd = ts.sw4 / 4, words = 2 * sh * swd;
    uint32_t v[kTopSrcWordsPerThread];
#pragma unroll
    for (int t = 0; t < kTopSrcWordsPerThread; ++t) {
      const int idx = tid + t * kTopThreads;
      v[t] = 0;
      if (idx < words) {
        const int row = idx / swd, c = 4 * (idx - row * swd);
        const bool right = row >= sh;
        const uint8_t* rp = (right ? a.srcR : a.srcL) + (size_t)(right ? row - sh : row) * a.spitch;
        const auto gp = gbl(rp);
        if (((uintptr_t)rp & 3) == 0 && c + 3 < sw) {
          v[t] = *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(gp + c);
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b) v[t] |= (uint32_t)gp[min(c + b, sw - 1)] << (8 * b);
        }
      }
    }
    uint32_t* const s_src32 = reinterpret_cast<uint32_t*>(s_srcL);  // views back to back: row r of both
#pragma unroll
    for (int t = 0; t < kTopSrcWordsPerThread; ++t) {
      const int idx = tid + t * kTopThreads;
      if (idx < words) s_src32[idx] = v[t];
    }
  }
  __syncthreads();

  // ---- 2. this level: sum over the 5 x 5 binomial taps (reflect-101), (s + 128) >> 8;
  // into LDS and into the level images in global memory
  for (int idx = tid; idx < 2 * W * Hh; idx += kTopThreads) {
    const int v = idx >= W * Hh, p2 = v ? idx - W * Hh : idx;
    const int y = p2 / W, x = p2 - y * W;
    const uint8_t* src = v ? s_srcR : s_srcL;
    int cx[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) cx[k] = reflect101(2 * x - 2 + k, sw);
    int s = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint8_t* row = src + reflect101(2 * y - 2 + k, sh) * ts.sw4;
      const int hsum = row[cx[0]] + 4 * row[cx[1]] + 6 * row[cx[2]] + 4 * row[cx[3]] + row[cx[4]];
      s += (k == 2 ? 6 : (k == 1 || k == 3) ? 4 : 1) * hsum;
    }
    const uint8_t o = (uint8_t)((s + 128) >> 8);
    (v ? s_imgR : s_imgL)[p2] = o;
    gbl(v ? a.dstR : a.dstL)[(size_t)y * a.pitch + x] = o;
  }
  __syncthreads();

  // ---- 3. the search's views of the level: left rows -1 .. Hh (reflect-101
  // rows and columns, byte 0 = column xa), right rows 0 .. Hh-1 (clamped
  // columns, byte 0 = column xs), the layouts the search launch stages per row
  const int xa = -4, xs = (-MARG) & ~3;
  for (int idx = tid; idx < (Hh + 2) * ts.ltw; idx += kTopThreads) {
    const int ty = idx / ts.ltw, b = idx - ty * ts.ltw;
    s_left[idx] = s_imgL[reflect101(ty - 1, Hh) * W + clampi(reflect101(xa + b, W), 0, W - 1)];
  }
  for (int idx = tid; idx < Hh * ts.rwb; idx += kTopThreads) {
    const int y = idx / ts.rwb, b = idx - y * ts.rwb;
    s_right[idx] = s_imgR[y * W + clampi(xs + b, 0, W - 1)];
  }
  __syncthreads();

  // ---- 4. the search: one aligned group of G lanes per patch, no parent (start 0)
  {
    const int q = tid / G, g = tid % G;
    const bool live = q < np;
    const int k = live ? q : np - 1;
    const int j = k / nx, i = k - j * nx;
    const int ox = grid_origin(i, W, P, S), oy = grid_origin(j, Hh, P, S);
    const PatchOut po = search_patch_u8<P, G>(a, lp, g, ox, oy, reinterpret_cast<const uint32_t*>(s_left + oy * ts.ltw),
                                              ts.ltw, xa, s_right + oy * ts.rwb, ts.rwb, xs, ts.rwb, 0.0);
    if (g == 0 && live) {
      const D4 d = po.d;
      gbl(a.pa.pipar)[k] = 0.0;
      gbl(a.pa.u)[k] = po.u;
      st4(a.pa.dssd + k, d);
      gbl(a.pa.acc)[k] = po.acc ? 1 : 0;
      if (lp.keep) {
        gbl(a.pa.uinit)[k] = 0.0;
        gbl(a.pa.ssd0)[k] = po.s0;
        gbl(a.pa.rho)[k] = (float)po.rho;
        gbl(a.pa.hess)[k] = (float)po.H;
      }
      s_pu[k] = po.u;
      s_pd[k] = d;
      s_pacc[k] = po.acc ? 1 : 0;
      s_psum[k] = po.acc ? ssd_fixed(po.s0) : 0ull;
    }
  }
  __syncthreads();

  // ---- 5. the level sum of SSD(0) over the accepted patches (exact integer
  // halves, so the same value as the partials of the search launch) and the
  // level scalars
  {
    unsigned long long lo = 0, hi = 0;
    int c = 0;
    for (int k = tid; k < np; k += kTopThreads) {
      lo += s_psum[k] & 0xffffffffull;
      hi += s_psum[k] >> 32;
      c += s_pacc[k];
    }
    lo = wave_sum_u64(lo);
    hi = wave_sum_u64(hi);
    c = wave_sum_i32(c);
    if (lane == 0) {
      s_wlo[wave] = lo;
      s_whi[wave] = hi;
      s_wcnt[wave] = c;
    }
  }
  __syncthreads();
  double tau;
  {
    unsigned long long tlo = 0, thi = 0;
    long long cnt = 0;
    for (int w = 0; w < kTopWaves; ++w) {
      tlo += s_wlo[w];
      thi += s_whi[w];
      cnt += s_wcnt[w];
    }
    double sc[4];
    level_scalars(lp, fixed_sum_value(thi, tlo), cnt, sc);
    if (tid < 4) gbl(a.scal)[tid] = sc[tid];
    tau = sc[1];
  }

  // ---- 6. the patch records
  for (int k = tid; k < np; k += kTopThreads) {
    PatchRaw raw;
    raw.u = s_pu[k];
    raw.pipar = 0.0;
    raw.d = s_pd[k];
    raw.acc = s_pacc[k];
    const D4 d = patch_record(a, lp, lp.level, raw, tau);
    if (lp.keep) st4(a.pa.dens + k, d);
    s_u[k] = d.x;
    s_w[k] = d.y;
    s_v[k] = d.z;
  }
  __syncthreads();

  // ---- 7. the fusion of every pixel over its covering patches (mask weights),
  // the sums in the order of the fusion launch; holes keep 0 (no parent)
  for (int idx = tid; idx < W * Hh; idx += kTopThreads) {
    const int y = idx / W, x = idx - y * W;
    int pilo, pihi, piex, pjlo, pjhi, pjex;
    cover_range(x, W, P, S, nx, pilo, pihi, piex);
    cover_range(y, Hh, P, S, ny, pjlo, pjhi, pjex);
    const int iend = piex >= 0 ? pihi + 1 : pihi, jend = pjex >= 0 ? pjhi + 1 : pjhi;
    PixSums ps;
    for (int jj = pjlo; jj <= jend; ++jj) {
      const int j = jj <= pjhi ? jj : pjex;
      const double mb = lp.fusion == 2 ? 1.0 : s_m[y - grid_origin(j, Hh, P, S)];
      ColSums cs;
      for (int ii = pilo; ii <= iend; ++ii) {
        const int i = ii <= pihi ? ii : piex;
        const int r = j * nx + i;
        const double dw = s_w[r];
        if (dw < 0.0) continue;  // rejected patch
        col_add(cs, lp.fusion == 2 ? 1.0 : s_m[x - grid_origin(i, W, P, S)], dw, s_u[r], s_v[r]);
      }
      row_add(ps, mb, cs.a0, cs.a1, cs.a2, cs.a3);
    }
    const bool valid = ps.z > 0.0;
    gbl(a.ubar)[idx] = valid ? ps.zu * recip(ps.z) : 0.0;  // as the fusion launch normalises
    gbl(a.qmap)[idx] = valid ? ps.z * recip(ps.zm) : 0.0;
  }
}

template <int P>
hipError_t launch_top_p(const PairLevel* tab, int npairs, const LevelParams& lp, const TopShape& ts, hipStream_t s) {
  constexpr int g0 = search_lanes(P, 0), g1 = search_lanes(P, 1), g2 = search_lanes(P, 2);
  if (ts.g == g0) bdis_launch((k_top<P, g0>), dim3(npairs), dim3(kTopThreads), ts.lds, s, tab, lp, ts);
  else if (ts.g == g1) bdis_launch((k_top<P, g1>), dim3(npairs), dim3(kTopThreads), ts.lds, s, tab, lp, ts);
  else if (ts.g == g2) bdis_launch((k_top<P, g2>), dim3(npairs), dim3(kTopThreads), ts.lds, s, tab, lp, ts);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

TopShape top_shape(int P, int S, int maxw, int maxh, int maxsw, int maxsh, int maxnp) {
  (void)S;
  TopShape ts{};
  if (P < 3 || P > kMaxPatch || maxnp <= 0) return ts;
  // the fewest lanes per patch: the whole level runs on one compute unit, so
  // the instruction count, not the per-lane chain, bounds the search there
  const int g = search_lanes(P, kSearchKinds - 1);
  if ((long)maxnp * g <= kTopThreads) ts.g = g;
  if (ts.g == 0 || 2L * maxsh * ((maxsw + 3) / 4) > (long)kTopSrcWordsPerThread * kTopThreads) {
    ts.g = 0;
    return ts;
  }
  auto up16 = [](long v) { return (v + 15) / 16 * 16; };
  const int marg = P + 4, xs = (-marg) & ~3;
  ts.sw4 = (maxsw + 3) / 4 * 4;
  ts.src_rows = maxsh;
  ts.img_px = maxw * maxh;
  ts.ltw = (int)up16(maxw + 16);            // columns -4 .. w + 11: every word the template reads
  ts.rwb = (int)up16(maxw + marg + 8 - xs);  // columns xs .. w + marg + 7
  ts.np_max = maxnp;
  long off = up16(2L * maxsh * ts.sw4);
  ts.off_img = (int)off;
  off = up16(off + 2L * ts.img_px);
  ts.off_left = (int)off;
  off = up16(off + (long)(maxh + 2) * ts.ltw);
  ts.off_right = (int)off;
  off = up16(off + (long)maxh * ts.rwb);
  ts.off_pat = (int)off;
  off += (long)maxnp * (8 + 32 + 3 * 8 + 8 + 4);
  if (off > kSearchMaxLds) {
    ts.g = 0;
    return ts;
  }
  ts.lds = (int)up16(off);
  return ts;
}

hipError_t launch_top(const PairLevel* tab, int npairs, const LevelParams& lp, const TopShape& ts, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  if (ts.g == 0) return hipErrorInvalidValue;
  return by_patch(lp.P, [&](auto pc) { return launch_top_p<decltype(pc)::value>(tab, npairs, lp, ts, s); });
}

}  // namespace bdis
