// Per-patch inverse-compositional 1-D search, Bayesian window and acceptance
// (Eq. 1 with the inverse roles of Sec. III-A; window of Eq. 5-6 with offsets
// -1, -1/2, 0, +1/2, +1 of Sec. IV-A; saddle / in-bounds rejection of
// Sec. III-B and III-F), plus the per-pair reduction that sets sigma_r^(n)
// (Sec. III-B): workgroups write partial sums, which k_reduce (large levels)
// or every fusion workgroup of the level (small levels) adds in a fixed order.
//
// Mapping: an aligned group of G = 2..16 lanes per patch (a DPP pair, quad,
// half-row or row, so group reductions are 1-4 DPP adds), each lane holding
// R = ceil(P / G) consecutive patch rows; THREADS/G patches of one patch row
// of one pair per workgroup.  The tuner picks G and THREADS per level: one
// row per lane keeps the per-lane chain of the K dependent iterations short
// (small, latency-bound levels), several rows per lane repeat the per-patch
// iteration logic on fewer lanes (large, throughput-bound levels).  The left
// rows around those patches (for the template and its Sobel gradient) and a
// window of the right rows around the patches' starting displacements are
// staged in LDS once; right-image samples outside the window fall back to
// (clamped) global loads.
//
// The packed-byte arithmetic and the per-patch search live in search_common.h.
#include "search_common.h"

namespace bdis {

namespace {

// Waves per SIMD the register allocation must allow: five for the
// several-rows-per-lane mappings (throughput-bound levels).
template <int P, int G>
constexpr int search_min_waves() {
  return (P + G - 1) / G >= 2 ? 5 : 1;
}

// Workgroups of one patch row that each stage the whole right row (beyond
// this, the repeated row loads cost more than the window's placement step).
constexpr int kFullRowWorkgroups = 4;

template <int P, int G, int THREADS>
__global__ __launch_bounds__(THREADS, (search_min_waves<P, G>())) void k_search_u8(const PairLevel* tab, int npairs, LevelParams lp) {
  static_assert(G >= 2 && G <= 16 && THREADS % 64 == 0, "lanes per patch and workgroup size");
  constexpr int NPB = THREADS / G;               // patches per workgroup
  constexpr int MARG = P + 4;                    // window margin around the start range
  constexpr int NWAVES = THREADS / 64;

  extern __shared__ uint32_t s_dyn[];
  __shared__ int s_umin, s_umax;
  __shared__ unsigned long long s_psum[NPB];
  __shared__ int s_pcnt[NPB];

  const int lb = xcd_block();
  const PairLevel& a = tab[find_pair<1>(tab, npairs, lb)];
  const int blk = lb - a.search0;   // workgroup within the pair
  const int tid = threadIdx.x;
  const int q = tid / G;   // patch slot in the workgroup
  const int g = tid % G;   // lane within the patch
  const int W = a.g.w, Hh = a.g.h, S = lp.S;
  int LTW, RWB;
  search_lds_layout(P, NPB, S, LTW, RWB);
  uint32_t* s_left32 = s_dyn;
  uint32_t* s_right32 = s_dyn + (P + 2) * LTW / 4;
  const uint8_t* s_right = reinterpret_cast<const uint8_t*>(s_right32);

  const int j = blk / a.search_nbx;
  const int i0 = (blk % a.search_nbx) * NPB;
  const bool live = (i0 + q) < a.g.nx;
  const int i = live ? i0 + q : a.g.nx - 1;
  const int ilast = min(i0 + NPB - 1, a.g.nx - 1);
  const int ox = grid_origin(i, W, P, S);
  const int oy = grid_origin(j, Hh, P, S);
  const int ox0 = grid_origin(i0, W, P, S);
  const int oxl = grid_origin(ilast, W, P, S);

  if (tid == 0) {
    s_umin = INT_MAX;
    s_umax = INT_MIN;
  }
  const int wave = tid / 64, lane = tid % 64;
  // ---- right window: rows oy .. oy+P-1, columns xs .. xs+rw-1 (clamped to the
  // image), xs a multiple of 4.  When at most four workgroups share the patch
  // row and the image row with a margin of MARG columns on each side fits, that
  // row is staged at once together with the left tile (no barrier and no
  // second round trip for the window's placement); otherwise the columns
  // around the patches' starting displacements, after a workgroup min/max of
  // floor(u0).
  // ---- left tile: image rows oy-1 .. oy+P, columns xa .. oxl+P (reflect-101),
  // xa = (ox0 - 1) rounded down to a multiple of 4.
  // The first word of every row a lane stages (the left tile's, and the full
  // right rows') is loaded before the parent maps are read, so those loads and
  // the parent's are one round trip; the words are stored afterwards.
  const bool full_row = a.search_nbx <= kFullRowWorkgroups && W + 2 * MARG + 8 <= RWB;
  int xs = (-MARG) & ~3;
  int ndr = (W + MARG - xs + 3) / 4;
  const int xa = (ox0 - 1) & ~3;
  const int ndl = (oxl + P + 1 - xa + 3) / 4;
  constexpr int LR = (P + 2 + NWAVES - 1) / NWAVES, RR = (P + NWAVES - 1) / NWAVES;
  uint32_t lw0[LR], rw0[RR];
#pragma unroll
  for (int r = 0; r < LR; ++r) {
    const int ty = wave + r * NWAVES;
    lw0[r] = 0;
    if (ty < P + 2 && lane < ndl) {
      const uint8_t* rp = a.L + (size_t)reflect101(oy - 1 + ty, Hh) * a.pitch;
      lw0[r] = row_word<true>(rp, W, xa + 4 * lane, ((uintptr_t)rp & 3) == 0);
    }
  }
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const int ty = wave + r * NWAVES;
    rw0[r] = 0;
    if (full_row && ty < P && lane < ndr) {
      const uint8_t* rp = a.R + (size_t)(oy + ty) * a.pitch;
      rw0[r] = row_word<false>(rp, W, xs + 4 * lane, ((uintptr_t)rp & 3) == 0);
    }
  }

  // ---- start from the parent level (Fig. 1): 2 * fused map at the centre
  double uinit = 0.0, pipar = 0.0;
  if (a.par_ubar) {
    const double cx = 0.5 * ((double)ox + 0.5 * (double)(P - 1));
    const double cy = 0.5 * ((double)oy + 0.5 * (double)(P - 1));
    uinit = 2.0 * bilinear(a.par_ubar, a.pw, a.ph, cx, cy);
    pipar = bilinear(a.par_q, a.pw, a.ph, cx, cy);
  }

  auto stage_right = [&](int x0r, int nd) {
    for (int ty = wave; ty < P; ty += NWAVES) {
      const uint8_t* rp = a.R + (size_t)(oy + ty) * a.pitch;
      stage_row<false>(s_right32 + ty * (RWB / 4), rp, W, x0r, nd, lane, ((uintptr_t)rp & 3) == 0);
    }
  };
#pragma unroll
  for (int r = 0; r < LR; ++r) {
    const int ty = wave + r * NWAVES;
    if (ty < P + 2) {
      if (lane < ndl) s_left32[ty * (LTW / 4) + lane] = lw0[r];
      const uint8_t* rp = a.L + (size_t)reflect101(oy - 1 + ty, Hh) * a.pitch;
      stage_row<true>(s_left32 + ty * (LTW / 4), rp, W, xa, ndl, lane, ((uintptr_t)rp & 3) == 0, 64);
    }
  }
  if (full_row) {
#pragma unroll
    for (int r = 0; r < RR; ++r) {
      const int ty = wave + r * NWAVES;
      if (ty < P) {
        if (lane < ndr) s_right32[ty * (RWB / 4) + lane] = rw0[r];
        const uint8_t* rp = a.R + (size_t)(oy + ty) * a.pitch;
        stage_row<false>(s_right32 + ty * (RWB / 4), rp, W, xs, ndr, lane, ((uintptr_t)rp & 3) == 0, 64);
      }
    }
  }
  if (!full_row) {
    __syncthreads();
    if (g == 0 && live) {
      const int mu = (int)floor(uinit);
      atomicMin(&s_umin, mu);
      atomicMax(&s_umax, mu);
    }
    __syncthreads();
    // on small launches the window's spare columns widen both margins, so that
    // iterations that wander off still read LDS
    const int need = oxl + P + s_umax + MARG + 2 - (ox0 + s_umin - MARG);
    const int extra = lp.wide_win ? max(0, (RWB - 8 - need) / 2) : 0;
    xs = (ox0 + s_umin - MARG - extra) & ~3;
    ndr = min((oxl + P + s_umax + MARG + 2 + extra - xs + 3) / 4, RWB / 4);
    stage_right(xs, ndr);
  }
  const int rw = 4 * ndr;
  __syncthreads();

  const PatchOut po = search_patch_u8<P, G>(a, lp, g, ox, oy, s_left32, LTW, xa, s_right, RWB, xs, rw, uinit);
  const double u = po.u, s0 = po.s0, rho = po.rho, H = po.H;
  const bool acc = po.acc;


  // the search results the probability and fusion read (52 B per patch), and
  // with lp.keep the rest of the patch state (debug dumps)
  const int k = j * a.g.nx + i;
  if (g == 0 && live) {
    gbl(a.pa.pipar)[k] = pipar;
    gbl(a.pa.u)[k] = u;
    st4(a.pa.dssd + k, po.d);
    gbl(a.pa.acc)[k] = acc ? 1 : 0;
    if (lp.keep) {
      gbl(a.pa.uinit)[k] = uinit;
      gbl(a.pa.ssd0)[k] = s0;
      gbl(a.pa.rho)[k] = (float)rho;
      gbl(a.pa.hess)[k] = (float)H;
    }
  }

  // ---- this workgroup's partial of the level reduction: the exact
  // fixed-point sum of SSD(0) over its accepted patches and their count
  if (g == 0) {
    s_psum[q] = (live && acc) ? ssd_fixed(s0) : 0ull;
    s_pcnt[q] = (live && acc) ? 1 : 0;
  }
  __syncthreads();
  if (wave == 0) {
    unsigned long long lo = 0, hi = 0;
    int pc = 0;
    for (int t = lane; t < NPB; t += 64) {
      lo += s_psum[t] & 0xffffffffull;
      hi += s_psum[t] >> 32;
      pc += s_pcnt[t];
    }
    lo = wave_sum_u64(lo);
    hi = wave_sum_u64(hi);
    pc = wave_sum_i32(pc);
    if (lane == 0) {
      const auto pw = gbl(reinterpret_cast<unsigned long long*>(a.part_sum));
      pw[2 * blk] = lo;
      pw[2 * blk + 1] = hi;
      gbl(a.part_cnt)[blk] = pc;
    }
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

template <int P, int G>
hipError_t launch_pg(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, int threads, int lds,
                     hipStream_t s) {
  switch (threads) {
    case 64: bdis_launch((k_search_u8<P, G, 64>), dim3(nblocks), dim3(64), lds, s, tab, npairs, lp); break;
    case 128: bdis_launch((k_search_u8<P, G, 128>), dim3(nblocks), dim3(128), lds, s, tab, npairs, lp); break;
    case 256: bdis_launch((k_search_u8<P, G, 256>), dim3(nblocks), dim3(256), lds, s, tab, npairs, lp); break;
    case 512: bdis_launch((k_search_u8<P, G, 512>), dim3(nblocks), dim3(512), lds, s, tab, npairs, lp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_p(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, int opt, hipStream_t s) {
  if (opt < 0 || opt >= kNumSearchOptions) return hipErrorInvalidValue;
  const int lds = search_lds_bytes(P, opt, lp.S);
  if (lds > kSearchMaxLds) return hipErrorInvalidValue;
  const int threads = search_option_threads(opt);
  switch (search_option_kind(opt)) {
    case 0: return launch_pg<P, search_lanes(P, 0)>(tab, npairs, nblocks, lp, threads, lds, s);
    case 1: return launch_pg<P, search_lanes(P, 1)>(tab, npairs, nblocks, lp, threads, lds, s);
    case 2: return launch_pg<P, search_lanes(P, 2)>(tab, npairs, nblocks, lp, threads, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_reduce(const PairLevel* tab, int npairs, const LevelParams& lp, hipStream_t s) {
  if (npairs <= 0 || lp.inline_prob) return hipSuccess;
  bdis_launch(k_reduce, dim3(npairs), dim3(256), 0, s, tab, lp);
  return hipGetLastError();
}

hipError_t launch_search(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, int opt,
                         hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  switch (lp.P) {
    case 3: return launch_p<3>(tab, npairs, nblocks, lp, opt, s);
    case 4: return launch_p<4>(tab, npairs, nblocks, lp, opt, s);
    case 5: return launch_p<5>(tab, npairs, nblocks, lp, opt, s);
    case 6: return launch_p<6>(tab, npairs, nblocks, lp, opt, s);
    case 7: return launch_p<7>(tab, npairs, nblocks, lp, opt, s);
    case 8: return launch_p<8>(tab, npairs, nblocks, lp, opt, s);
    case 9: return launch_p<9>(tab, npairs, nblocks, lp, opt, s);
    case 10: return launch_p<10>(tab, npairs, nblocks, lp, opt, s);
    case 11: return launch_p<11>(tab, npairs, nblocks, lp, opt, s);
    case 12: return launch_p<12>(tab, npairs, nblocks, lp, opt, s);
    case 13: return launch_p<13>(tab, npairs, nblocks, lp, opt, s);
    case 14: return launch_p<14>(tab, npairs, nblocks, lp, opt, s);
    case 15: return launch_p<15>(tab, npairs, nblocks, lp, opt, s);
    case 16: return launch_p<16>(tab, npairs, nblocks, lp, opt, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdis
