// Image pyramid of both views (one pixel of level n covers 2^n x 2^n input
// pixels, Sec. III-B).  Separable binomial [1 4 6 4 1]/16 with reflect-101
// borders, sampled at even pixels, integer rounding (sum + 128) >> 8: exact
// uint8 arithmetic, bit-identical to any correct implementation.
//
// Two forms, chosen per level by its pixel count over the batch:
// k_pyr_small (small levels, latency-bound): 64 x 4 output tiles, each lane
//   gathers its five source columns of 11 source rows and filters them
//   horizontally into LDS, then vertically: few dependent steps.
// k_pyr_tall (large levels, bandwidth-bound): 120 x 12 output tiles, in three
//   passes:
//   1. the 2 x 12 + 3 source rows of the tile (62 words of 4 bytes each) are
//      staged in LDS, one 4-byte load per word, all of a lane's loads in
//      flight at once; out-of-image columns of border tiles are then filled
//      from the staged in-image bytes (reflect-101);
//   2. horizontal pass: each lane filters four output columns of a row from
//      four LDS words, a 4-tap v_dot4_u32_u8 (taps 1 4 6 4) plus the fifth tap,
//      and writes the four 16-bit sums as one 8-byte LDS word;
//   3. vertical pass: each lane combines five such rows into four output
//      bytes and writes them as one dword (bytes at a ragged right edge).
//   Every source byte is read from HBM about once (rows shared by
//   neighbouring tiles come from L2), every output byte written once.
#include "bdis_internal.h"

namespace bdis {

namespace {

constexpr int kSmallRows = 2 * kPyrSmallTy + 3;  // source rows touched by kPyrSmallTy output rows

__global__ __launch_bounds__(kPyrSmallTx* kPyrSmallTy) void k_pyr_small(const PairLevel* tab, int npairs) {
  __shared__ int hL[kSmallRows][kPyrSmallTx];
  __shared__ int hR[kSmallRows][kPyrSmallTx];
  const int b = xcd_block();
  const PairLevel& a = tab[find_pair<0>(tab, npairs, b)];
  const int tiles_x = (a.g.w + kPyrSmallTx - 1) / kPyrSmallTx;
  const int t = b - a.pyr0;
  const int tx = threadIdx.x % kPyrSmallTx;
  const int ty = threadIdx.x / kPyrSmallTx;
  const int x = (t % tiles_x) * kPyrSmallTx + tx;  // output column
  const int y0 = (t / tiles_x) * kPyrSmallTy;      // first output row of the tile
  const int dw = a.g.w, dh = a.g.h;
  const int xs = x < dw ? x : dw - 1;  // idle lanes read valid columns
  int cx[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) cx[k] = reflect101(2 * xs - 2 + k, a.sw);
  for (int r = ty; r < kSmallRows; r += kPyrSmallTy) {
    int sy = 2 * y0 - 2 + r;
    // rows beyond sh + 1 feed only idle output rows: keep them in range
    sy = sy > a.sh + 1 ? a.sh - 1 : reflect101(sy, a.sh);
    const auto rl = gbl(a.srcL + (size_t)sy * a.spitch);
    const auto rr = gbl(a.srcR + (size_t)sy * a.spitch);
    hL[r][tx] = rl[cx[0]] + 4 * rl[cx[1]] + 6 * rl[cx[2]] + 4 * rl[cx[3]] + rl[cx[4]];
    hR[r][tx] = rr[cx[0]] + 4 * rr[cx[1]] + 6 * rr[cx[2]] + 4 * rr[cx[3]] + rr[cx[4]];
  }
  __syncthreads();
  const int y = y0 + ty;
  if (x >= dw || y >= dh) return;
  const int q = 2 * ty;  // local row of source row 2y - 2
  const int sl = hL[q][tx] + 4 * hL[q + 1][tx] + 6 * hL[q + 2][tx] + 4 * hL[q + 3][tx] + hL[q + 4][tx];
  const int sr = hR[q][tx] + 4 * hR[q + 1][tx] + 6 * hR[q + 2][tx] + 4 * hR[q + 3][tx] + hR[q + 4][tx];
  gbl(a.dstL)[(size_t)y * a.pitch + x] = (uint8_t)((sl + 128) >> 8);
  gbl(a.dstR)[(size_t)y * a.pitch + x] = (uint8_t)((sr + 128) >> 8);
}

constexpr int kPyrThreads = 256;
constexpr int kSrcRows = 2 * kPyrTallTy + 3;         // source rows 2 y0 - 2 .. 2 y0 + 2 kPyrTallTy
constexpr int kSrcWords = (2 * kPyrTallTx + 8) / 4;  // source columns 2 x0 - 4 .. 2 x0 + 2 kPyrTallTx + 3
static_assert(kSrcWords <= 64, "one staged word per lane");
constexpr int kQuads = kPyrTallTx / 4;               // output column quads per row
static_assert(kPyrTallTx % 4 == 0, "four output columns per lane");

// Five waves per SIMD (at most 96 VGPRs, no spills; 26 KB of LDS allows six
// workgroups per CU).
__global__ __launch_bounds__(kPyrThreads, 5) void k_pyr_tall(const PairLevel* tab, int npairs) {
  __shared__ uint32_t s_src[2][kSrcRows][kSrcWords];
  __shared__ uint2 s_h[2][kSrcRows][kQuads];  // four 16-bit horizontal sums per entry
  const int b = xcd_block();
  const PairLevel& a = tab[find_pair<0>(tab, npairs, b)];
  const int tiles_x = (a.g.w + kPyrTallTx - 1) / kPyrTallTx;
  const int t = b - a.pyr0;
  const int x0 = (t % tiles_x) * kPyrTallTx;  // first output column of the tile
  const int y0 = (t / tiles_x) * kPyrTallTy;  // first output row of the tile
  const int dw = a.g.w, dh = a.g.h, sw = a.sw, sh = a.sh;
  const int cs = 2 * x0 - 4;              // source column of staged byte 0 (a multiple of 4)
  const int tid = threadIdx.x;

  // valid outputs of the tile: columns x0 .. x1, rows y0 .. y1; they read
  // staged words 0 .. kmax and source rows 0 .. rmax
  const int x1 = min(x0 + kPyrTallTx, dw) - 1, y1 = min(y0 + kPyrTallTy, dh) - 1;
  const int nq = (x1 - x0) / 4 + 1;                 // output column quads
  const int kmax = min((2 * x1 + 2 - cs) / 4, kSrcWords - 1);
  const int rmax = 2 * (y1 - y0) + 4;

  // ---- 1. stage the source rows (both views).  Wave w stages rows w, w + 4,
  // ...; lane l the word l of each.  Every lane first issues all its loads
  // (4-byte loads, the column clamped into the row) and then stores them; the
  // bytes of words that reach past an image border are then rewritten from the
  // staged in-image bytes with reflect-101 columns.
  constexpr int kWaves = kPyrThreads / 64;
  constexpr int kRowSlots = (kSrcRows + kWaves - 1) / kWaves;
  const int wave = tid / 64, lane = tid % 64;
  const int kl = min(lane, kSrcWords - 1);
  const int c = cs + 4 * kl;  // first source column of this lane's word
  auto src_row = [&](int v, int r) {
    int sy = 2 * y0 - 2 + r;
    // rows beyond sh + 1 feed only output rows past the level: keep them in range
    sy = sy > sh + 1 ? sh - 1 : reflect101(sy, sh);
    return (v ? a.srcR : a.srcL) + (size_t)sy * a.spitch;
  };
  const bool stage = lane <= kmax;
  if (sw >= 4) {
    // 4-byte loads at any byte address (global memory allows unaligned access)
    const int cc = clampi(c, 0, sw - 4);
    uint32_t wv[2][kRowSlots];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int i = 0; i < kRowSlots; ++i) {
        const int r = min(wave + kWaves * i, kSrcRows - 1);
        __builtin_memcpy(&wv[v][i], src_row(v, r) + cc, 4);
      }
    // a word that starts left of the row or ends past it keeps the loaded bytes
    // of its in-image columns at their place (the rest is rewritten below)
    const int shift = c >= 0 ? 8 * min(c - cc, 3) : 0;
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int i = 0; i < kRowSlots; ++i) {
        const int r = wave + kWaves * i;
        if (r < kSrcRows && r <= rmax && stage) s_src[v][r][lane] = wv[v][i] >> shift;
      }
  } else {
    for (int v = 0; v < 2; ++v)
      for (int r = wave; r < kSrcRows && r <= rmax; r += kWaves)
        if (stage) {
          const auto g = gbl(src_row(v, r));
          uint32_t word = 0;
          for (int bb = 0; bb < 4; ++bb) word |= (uint32_t)g[clampi(c + bb, 0, sw - 1)] << (8 * bb);
          s_src[v][r][lane] = word;
        }
  }
  __syncthreads();
  // out-of-image columns of border tiles: reflect-101 into staged in-image bytes
  // (every needed target column lies in [max(cs, 0), sw - 1]); the few border
  // lanes read all their target bytes first, then rewrite their words
  if (cs < 0 || cs + 4 * (kmax + 1) > sw) {
    if (stage && (c < 0 || c + 3 >= sw)) {
      const uint8_t* sb = reinterpret_cast<const uint8_t*>(&s_src[0][0][0]);
      int tgt[4];
      uint32_t keep = 0;  // byte mask of the in-image columns of the word
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int col = c + bb;
        if (col >= 0 && col < sw) keep |= 0xffu << (8 * bb);
        tgt[bb] = clampi(reflect101(col, sw), max(cs, 0), min(sw - 1, cs + 4 * kSrcWords - 1)) - cs;
      }
      uint32_t fixed[2][kRowSlots];
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int i = 0; i < kRowSlots; ++i) {
          const int r = min(wave + kWaves * i, kSrcRows - 1);
          const uint8_t* row = sb + ((size_t)v * kSrcRows + r) * (kSrcWords * 4);
          uint32_t word = 0;
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) word |= (uint32_t)row[tgt[bb]] << (8 * bb);
          fixed[v][i] = (s_src[v][r][lane] & keep) | (word & ~keep);
        }
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int i = 0; i < kRowSlots; ++i) {
          const int r = wave + kWaves * i;
          if (r < kSrcRows && r <= rmax) s_src[v][r][lane] = fixed[v][i];
        }
    }
    __syncthreads();
  }

  // ---- 2. horizontal pass: output columns 4q .. 4q+3 of the tile need staged
  // bytes 8q + 2 .. 8q + 12 (words 2q .. 2q+3)
  constexpr uint32_t kTaps = 0x04060401u;  // bytes 1, 4, 6, 4
  const int nr = rmax + 1;
  for (int e = tid; e < 2 * nr * nq; e += kPyrThreads) {
    const int vr = div_small(e, nq), q = e - vr * nq;
    const int v = vr >= nr ? 1 : 0, r = vr - v * nr;
    const uint32_t d0 = s_src[v][r][2 * q], d1 = s_src[v][r][2 * q + 1];
    const uint32_t d2 = s_src[v][r][2 * q + 2], d3 = s_src[v][r][2 * q + 3];
    const uint32_t h0 = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(d1, d0, 2u), kTaps, (d1 >> 16) & 255u, false);
    const uint32_t h1 = __builtin_amdgcn_udot4(d1, kTaps, d2 & 255u, false);
    const uint32_t h2 = __builtin_amdgcn_udot4(__builtin_amdgcn_alignbyte(d2, d1, 2u), kTaps, (d2 >> 16) & 255u, false);
    const uint32_t h3 = __builtin_amdgcn_udot4(d2, kTaps, d3 & 255u, false);
    s_h[v][r][q] = make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
  }
  __syncthreads();

  // ---- 3. vertical pass: output row y0 + yl from local rows 2 yl .. 2 yl + 4
  const int ny = y1 - y0 + 1;
  for (int e = tid; e < 2 * ny * nq; e += kPyrThreads) {
    const int vy = div_small(e, nq), q = e - vy * nq;
    const int v = vy >= ny ? 1 : 0, yl = vy - v * ny;
    const int y = y0 + yl, x = x0 + 4 * q;
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    constexpr uint32_t kW[5] = {1u, 4u, 6u, 4u, 1u};
#pragma unroll
    for (int tr = 0; tr < 5; ++tr) {
      const uint2 hv = s_h[v][2 * yl + tr][q];
      acc[0] += kW[tr] * (hv.x & 0xffffu);
      acc[1] += kW[tr] * (hv.x >> 16);
      acc[2] += kW[tr] * (hv.y & 0xffffu);
      acc[3] += kW[tr] * (hv.y >> 16);
    }
    uint32_t out = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) out |= ((acc[kk] + 128u) >> 8) << (8 * kk);
    uint8_t* row = (v ? a.dstR : a.dstL) + (size_t)y * a.pitch;
    if (x + 3 < dw && ((uintptr_t)row & 3) == 0) {
      gbl(reinterpret_cast<uint32_t*>(row + x))[0] = out;
    } else {
      for (int kk = 0; kk < 4 && x + kk < dw; ++kk) gbl(row)[x + kk] = (uint8_t)(out >> (8 * kk));
    }
  }
}

// Several small levels in one launch.  Workgroup b owns a tile x tile block of
// the top level n0 + m of one pair and, scaled by 2^(top - k), the matching
// block of every level k in between; it stages the region of level n0 those
// pixels depend on (the block grown by two source pixels per side per level,
// clipped to the level) with every load in flight at once, then builds each
// level's region in LDS from the one below (a pixel reads its 5 x 5 taps at
// reflect-101 positions, which stay inside the region below) and writes the
// pixels it owns.  Halo pixels are computed by every neighbouring workgroup
// that needs them; there is no communication between workgroups.
constexpr int kChainThreads = 512;
constexpr int kChainWordsPerThread = 16;  // staged source words per thread
constexpr int kChainMaxLevels = 4;        // levels one chain launch builds

__global__ __launch_bounds__(kChainThreads) void k_pyr_chain(const PairLevel* tab, int npairs, PyrChain ca) {
  extern __shared__ __align__(16) uint8_t s_ch[];
  const int b = xcd_block();
  const int top = ca.n0 + ca.m;
  const PairLevel* ttab = tab + ca.first[top];
  const int e = find_pair<0>(ttab, npairs, b);
  const PairLevel& at = ttab[e];
  const int tiles_x = (at.g.w + ca.tile - 1) / ca.tile;
  const int t = b - at.pyr0;
  const int tid = threadIdx.x;
  const int tx = (t % tiles_x) * ca.tile, ty = (t / tiles_x) * ca.tile;
  // level sizes relative to n0 (j = 0 .. m), in registers (the loops below are unrolled)
  int lw[kChainMaxLevels + 1], lh[kChainMaxLevels + 1];
  lw[0] = tab[ca.first[ca.n0 + 1] + e].sw;
  lh[0] = tab[ca.first[ca.n0 + 1] + e].sh;
#pragma unroll
  for (int j = 1; j <= kChainMaxLevels; ++j) {
    const PairLevel& q = tab[ca.first[min(ca.n0 + j, top)] + e];
    lw[j] = q.g.w;
    lh[j] = q.g.h;
  }
  const int wtop = at.g.w, htop = at.g.h;
  const int tx1 = min(tx + ca.tile, wtop), ty1 = min(ty + ca.tile, htop);
  // region of level n0 + j needed by the tile, d = m - j levels below the top:
  // [2^d (tx - 2) + 2, 2^d (tx1 + 1) - 1) (the tile grown by two source pixels
  // per side per level), clipped to the level
  auto region = [&](int j, int& x0, int& x1, int& y0, int& y1) {
    const int d = ca.m - j;
    x0 = max((tx - 2) * (1 << d) + 2, 0);
    x1 = min((tx1 + 1) * (1 << d) - 1, lw[j]);
    y0 = max((ty - 2) * (1 << d) + 2, 0);
    y1 = min((ty1 + 1) * (1 << d) - 1, lh[j]);
  };
  int rx0, rx1, ry0, ry1;
  region(0, rx0, rx1, ry0, ry1);
  // the source region starts at a 4-aligned column (dword loads)
  const int ax0 = rx0 & ~3;
  const int sw_words = (rx1 - ax0 + 3) / 4;
  const int srows = ry1 - ry0;

  // ---- 1. stage the level-n0 region of both views
  {
    const PairLevel& a1 = tab[ca.first[ca.n0 + 1] + e];
    const int words = 2 * srows * sw_words;
    uint32_t v[kChainWordsPerThread];
#pragma unroll
    for (int i = 0; i < kChainWordsPerThread; ++i) {
      const int idx = tid + i * kChainThreads;
      v[i] = 0;
      if (idx < words) {
        const int row = idx / sw_words, c = ax0 + 4 * (idx - row * sw_words);
        const bool right = row >= srows;
        const int y = ry0 + (right ? row - srows : row);
        const uint8_t* rp = (right ? a1.srcR : a1.srcL) + (size_t)y * a1.spitch;
        const auto gp = gbl(rp);
        if (((uintptr_t)rp & 3) == 0 && c + 3 < lw[0]) {
          v[i] = *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(gp + c);
        } else {
#pragma unroll
          for (int bb = 0; bb < 4; ++bb) v[i] |= (uint32_t)gp[min(c + bb, lw[0] - 1)] << (8 * bb);
        }
      }
    }
    uint32_t* const dst = reinterpret_cast<uint32_t*>(s_ch);
#pragma unroll
    for (int i = 0; i < kChainWordsPerThread; ++i) {
      const int idx = tid + i * kChainThreads;
      if (idx < words) dst[idx] = v[i];
    }
  }
  __syncthreads();

  // ---- 2. each level from the one below (the LDS halves alternate)
  const uint8_t* src = s_ch;
  int src_x0 = ax0, src_y0 = ry0, src_stride = 4 * sw_words, src_rows = srows;
  uint8_t* buf = s_ch + ca.lds_half;
#pragma unroll
  for (int j = 1; j <= kChainMaxLevels; ++j) {
    if (j > ca.m) break;
    const int k = ca.n0 + j;
    const PairLevel& q = tab[ca.first[k] + e];
    int x0, x1, y0, y1;
    region(j, x0, x1, y0, y1);
    const int cw = x1 - x0, chh = y1 - y0;
    const int stride = (cw + 3) & ~3;
    // owned block of this level: the top tile scaled by 2^(m - j); the last
    // tile of a row or column reaches the level's edge
    const int d = ca.m - j;
    const int ox0 = tx << d, oy0 = ty << d;
    const int ox1 = tx + ca.tile >= wtop ? lw[j] : min((tx + ca.tile) << d, lw[j]);
    const int oy1 = ty + ca.tile >= htop ? lh[j] : min((ty + ca.tile) << d, lh[j]);
    const int sw = lw[j - 1], shh = lh[j - 1];
    const bool last = j == ca.m;
    for (int idx = tid; idx < 2 * cw * chh; idx += kChainThreads) {
      const int v = idx >= cw * chh, p = v ? idx - cw * chh : idx;
      const int yl = div_small(p, cw), xl = p - yl * cw;
      const int x = x0 + xl, y = y0 + yl;
      const uint8_t* sv = src + v * src_rows * src_stride;
      int cx[5];
#pragma unroll
      for (int kk = 0; kk < 5; ++kk) cx[kk] = reflect101(2 * x - 2 + kk, sw) - src_x0;
      int acc = 0;
#pragma unroll
      for (int kk = 0; kk < 5; ++kk) {
        const uint8_t* row = sv + (reflect101(2 * y - 2 + kk, shh) - src_y0) * src_stride;
        const int hsum = row[cx[0]] + 4 * row[cx[1]] + 6 * row[cx[2]] + 4 * row[cx[3]] + row[cx[4]];
        acc += (kk == 2 ? 6 : (kk == 1 || kk == 3) ? 4 : 1) * hsum;
      }
      const uint8_t o = (uint8_t)((acc + 128) >> 8);
      if (!last) buf[v * chh * stride + yl * stride + xl] = o;
      if (x >= ox0 && x < ox1 && y >= oy0 && y < oy1) gbl(v ? q.dstR : q.dstL)[(size_t)y * q.pitch + x] = o;
    }
    if (last) break;
    __syncthreads();
    uint8_t* const old = const_cast<uint8_t*>(src);
    src = buf;
    buf = old;
    src_x0 = x0;
    src_y0 = y0;
    src_stride = stride;
    src_rows = chh;
  }
}

}  // namespace

PyrChain pyr_chain_shape(int n0, int m, int tile_top) {
  PyrChain ca{};
  ca.n0 = n0;
  ca.m = m;
  ca.tile = tile_top;
  // the largest region of any level of the chain (the source level's), both
  // views, twice (ping-pong between levels)
  int wmax = tile_top;
  for (int k = 0; k < m; ++k) wmax = 2 * wmax + 3;
  const int src_bytes = 2 * wmax * ((wmax + 3 + 3) & ~3);
  ca.lds_half = (src_bytes + 15) & ~15;
  ca.lds = 2 * ca.lds_half;
  if (m > kChainMaxLevels || 2L * wmax * (((wmax + 3 + 3) & ~3) / 4) > (long)kChainWordsPerThread * kChainThreads)
    ca.lds = 0;
  return ca;
}

hipError_t launch_pyr_chain(const PairLevel* tab, int npairs, int nblocks, const PyrChain& ca, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (ca.lds <= 0 || ca.m < 1) return hipErrorInvalidValue;
  bdis_launch(k_pyr_chain, dim3(nblocks), dim3(kChainThreads), ca.lds, s, tab, npairs, ca);
  return hipGetLastError();
}

hipError_t launch_pyramid(const PairLevel* tab, int npairs, int nblocks, bool tall, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (tall)
    bdis_launch(k_pyr_tall, dim3(nblocks), dim3(kPyrThreads), 0, s, tab, npairs);
  else
    bdis_launch(k_pyr_small, dim3(nblocks), dim3(kPyrSmallTx * kPyrSmallTy), 0, s, tab, npairs);
  return hipGetLastError();
}

}  // namespace bdis
