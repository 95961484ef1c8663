// Shared by the per-level search kernel and the single-workgroup top-level
// kernel: the packed-byte helpers and the search of one patch by its group of
// lanes, so both give the same bits.
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
// Only the final combinations are rounded (in double).  Image samples, template
// bytes and the two bytes of Gx + 1024 are packed four per dword, so the sums
// of products are v_dot4_u32_u8 (exact 8-bit products, 32-bit accumulation).
#pragma once

#include "bdis_internal.h"

#include <climits>

namespace bdis {

namespace {

// a*b - c*d of int32 values whose products and difference stay below 2^53 in
// magnitude (true for every combination below: at most about 2^36), so the
// double result is exact; full-rate FP64 instead of quarter-rate 64-bit mads.
BDIS_DEV double exact_ab_cd(int a, int b, int c, int d) {
  return fma((double)a, (double)b, -((double)c * (double)d));
}

// Packed samples: four uint8 samples per dword, little-endian (byte b of word
// w is column 4w + b), so byte-vector sums and dot products are v_dot4_u32_u8
// (four exact 8-bit products per instruction).
BDIS_DEV uint32_t dot4(uint32_t a, uint32_t b, uint32_t acc) { return __builtin_amdgcn_udot4(a, b, acc, false); }

// Two 16-bit lanes in one register (packed integer v_pk_* arithmetic).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
BDIS_DEV u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
BDIS_DEV uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// Word w of a P-sample vector: mask of its valid bytes, and 1 in each valid byte.
__host__ __device__ constexpr uint32_t valid_bytes(int w, int P) {
  return P - 4 * w >= 4 ? 0xffffffffu : ((1u << (8 * (P - 4 * w))) - 1u);
}
__host__ __device__ constexpr uint32_t ones_word(int w, int P) { return valid_bytes(w, P) & 0x01010101u; }

// Right-image samples of one row at columns x .. x + 4 NW + 3 as NW + 1 packed
// words: from the LDS window (aligned dword reads, realigned with
// v_alignbyte) when it holds every word read, else from global memory with each
// column clamped to the image (identical values either way).  `grow` is the
// image row, W its width.
template <int NW>
BDIS_DEV void fetch_words(uint32_t (&B)[NW + 1], const uint8_t* win, int xs, int rw, const uint8_t* grow, int x,
                          int W) {
  const int off = x - xs;
  const int a4 = off & ~3;
  if (off >= 0 && a4 + 4 * (NW + 2) <= rw) {
    const uint32_t* wp = reinterpret_cast<const uint32_t*>(win + a4);
    const uint32_t sh = (uint32_t)(off & 3);
    uint32_t D[NW + 2];
#pragma unroll
    for (int i = 0; i < NW + 2; ++i) D[i] = wp[i];
#pragma unroll
    for (int w = 0; w <= NW; ++w) B[w] = __builtin_amdgcn_alignbyte(D[w + 1], D[w], sh);
  } else {
    // samples outside the staged window (patches whose iterations wander off):
    // aligned dwords of the image row when the row is 4-aligned and the words
    // lie inside it
    const auto g = gbl(grow);
    const int x4 = x & ~3;
    if (x4 >= 0 && x4 + 4 * (NW + 2) <= W && ((uintptr_t)grow & 3) == 0) {
      const auto gw = reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(g + x4);
      const uint32_t sh = (uint32_t)(x & 3);
      uint32_t D[NW + 2];
#pragma unroll
      for (int i = 0; i < NW + 2; ++i) D[i] = gw[i];
#pragma unroll
      for (int w = 0; w <= NW; ++w) B[w] = __builtin_amdgcn_alignbyte(D[w + 1], D[w], sh);
    } else {
      // near the image borders: clamped samples, one word (four loads) per
      // step; the empty asm keeps the address arithmetic inside this branch
      int xx = x;
      asm volatile("" : "+v"(xx));
#pragma unroll 1
      for (int w = 0; w <= NW; ++w) {
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) v |= (uint32_t)g[clampi(xx + 4 * w + b, 0, W - 1)] << (8 * b);
#pragma unroll
        for (int t = 0; t < NW; ++t) B[t] = B[t + 1];
        B[NW] = v;
      }
    }
  }
}

// Words of the P samples starting J columns after the first sample of B.
template <int NW, int J>
BDIS_DEV uint32_t shifted_word(const uint32_t (&B)[NW + 1], int w) {
  if constexpr (J == 0) return B[w];
  else return __builtin_amdgcn_alignbyte(B[w + 1], B[w], (uint32_t)J);
}

// Copies columns [x0, x0 + 4 nd) of image row `rp` (width W) into LDS as nd
// dwords; x0 is a multiple of 4.  Columns outside the row are mapped by
// reflect-101 (REFLECT) or clamping, and then clamped, so every access stays
// in the row.  Interior dwords of a 4-aligned row are single global loads.
// The dword of columns c .. c + 3 of row `rp` as stage_row stores it.
template <bool REFLECT>
BDIS_DEV uint32_t row_word(const uint8_t* rp, int W, int c, bool aligned) {
  const auto g = gbl(rp);
  if (aligned && c >= 0 && c + 3 < W) return *reinterpret_cast<const __attribute__((address_space(1))) uint32_t*>(g + c);
  uint32_t v = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int x = c + b;
    x = REFLECT ? reflect101(x, W) : x;
    x = clampi(x, 0, W - 1);
    v |= (uint32_t)g[x] << (8 * b);
  }
  return v;
}

template <bool REFLECT>
BDIS_DEV void stage_row(uint32_t* dst, const uint8_t* rp, int W, int x0, int nd, int lane, bool aligned, int k0 = 0) {
  for (int k = k0 + lane; k < nd; k += 64) dst[k] = row_word<REFLECT>(rp, W, x0 + 4 * k, aligned);
}


// The result of one patch search; every lane of the patch's group holds it.
struct PatchOut {
  double u;    // final displacement (after the search-threshold reset)
  double s0;   // window SSD at d = 0
  D4 d;        // SSD(d) - SSD(0), d = -1, -1/2, +1/2, +1
  double rho;  // in-bounds ratio
  double H;    // Gauss-Newton Hessian
  bool acc;    // accepted (centre minimum, enough pixels in bounds)
};

// The search of one patch (Eq. 1 iterations, window SSDs, acceptance) by its
// aligned group of G lanes; g is the lane within the group.  The patch origin
// is (ox, oy) on a level of width a.g.w.  Left tile: LDS words of the image rows
// oy - 1 .. oy + P (reflect-101), row stride LTW bytes, byte 0 of a row is
// image column xa (a multiple of 4, at most ox - 1).  Right window: LDS rows
// oy .. oy + P - 1 from s_right with row stride RWB bytes holding columns
// xs .. xs + rw - 1 (clamped to the image); samples outside it come from the
// global rows of a.R.  uinit is the start displacement.
// Floating-point contraction is off here and the fused multiply-adds are
// written out, so every kernel that inlines this gets the same bits.
template <int P, int G>
BDIS_DEV PatchOut search_patch_u8(const PairLevel& a, const LevelParams& lp, int g, int ox, int oy,
                                  const uint32_t* s_left32, int LTW, int xa, const uint8_t* s_right, int RWB,
                                  int xs, int rw, double uinit) {
#pragma clang fp contract(off)
  constexpr int R = (P + G - 1) / G;     // patch rows per lane: rows g*R .. g*R+R-1
  constexpr bool kAllRows = R * G == P;  // no lane holds rows past the patch
  constexpr int N = P * P;
  constexpr int NW = (P + 3) / 4;        // packed words per patch row
  const int r0 = g * R;                  // first patch row of this lane
  const int W = a.g.w;

  // ---- template rows of this lane: T and Sobel-x G (integer); rows past the
  // patch (only when G does not divide P) read valid LDS and are masked out
  bool rlive[R];
  int rrow[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    rlive[k] = kAllRows || r0 + k < P;
    rrow[k] = kAllRows ? r0 + k : min(r0 + k, P - 1);
  }
  // packed rows: T, and Gx + 1024 (4..2044) split into its high (0..7) and low
  // bytes, so sum Gx R = 256 (Gh . R) + (Gl . R) - 1024 sum R; padding bytes 0.
  // Built from realigned LDS words of three tile rows at a time: the vertical
  // [1 2 1] sums S as 16-bit pairs (v_pk_add_u16), Gx + 1024 = S[c + 2] + 1024
  // - S[c] per pixel pair, its bytes gathered with v_perm; the row sums by dot4.
  uint32_t Tw[R][NW], Ghw[R][NW], Glw[R][NW];
  int sG = 0, sT = 0, sGG = 0, sGT = 0, sTT = 0;
  {
    constexpr int NPAIR = 2 * (NW + 1);  // 16-bit pairs of bytes 0 .. 4 NW + 3
    const int o0 = ox - 1 - xa;          // byte of column ox - 1 within a tile row
    auto tile_words = [&](int k, uint32_t (&Bw)[NW + 1], u16x2 (&Pr)[NPAIR]) {
      const int ty = kAllRows ? r0 + k : min(r0 + k, P + 1);  // tile row = image row oy - 1 + ty
      const int o = ty * LTW + o0;
      const uint32_t* wp = s_left32 + (o >> 2);
      const uint32_t sh = (uint32_t)(o & 3);
      uint32_t D[NW + 2];
#pragma unroll
      for (int q2 = 0; q2 < NW + 2; ++q2) D[q2] = wp[q2];
#pragma unroll
      for (int w = 0; w <= NW; ++w) {
        Bw[w] = __builtin_amdgcn_alignbyte(D[w + 1], D[w], sh);
        Pr[2 * w] = as_u16x2(__builtin_amdgcn_perm(0u, Bw[w], 0x0c010c00u));      // bytes 0, 1
        Pr[2 * w + 1] = as_u16x2(__builtin_amdgcn_perm(0u, Bw[w], 0x0c030c02u));  // bytes 2, 3
      }
    };
    uint32_t Bu[NW + 1], Bc[NW + 1], Bd[NW + 1];
    u16x2 Pu[NPAIR], Pc[NPAIR], Pd[NPAIR];
    tile_words(0, Bu, Pu);
    tile_words(1, Bc, Pc);
    const u16x2 k1024 = {1024, 1024};
#pragma unroll
    for (int k = 0; k < R; ++k) {
      tile_words(k + 2, Bd, Pd);
      u16x2 Sv[NPAIR];
#pragma unroll
      for (int p = 0; p < NPAIR; ++p) Sv[p] = Pu[p] + Pd[p] + Pc[p] + Pc[p];
      uint32_t t1 = 0, t4 = 0, gh = 0, gl = 0, hh = 0, hl = 0, ll = 0, ht = 0, lt = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        // T: columns ox + 4w .. ox + 4w + 3 = bytes 4w + 1 .. 4w + 4 of the centre row
        const uint32_t tw = __builtin_amdgcn_alignbyte(Bc[w + 1], Bc[w], 1u) & valid_bytes(w, P);
        const uint32_t ga = as_u32((Sv[2 * w + 1] + k1024) - Sv[2 * w]);      // pixels 4w, 4w + 1
        const uint32_t gb = as_u32((Sv[2 * w + 2] + k1024) - Sv[2 * w + 1]);  // pixels 4w + 2, 4w + 3
        const uint32_t lw = __builtin_amdgcn_perm(gb, ga, 0x06040200u) & valid_bytes(w, P);
        const uint32_t hw = __builtin_amdgcn_perm(gb, ga, 0x07050301u) & valid_bytes(w, P);
        Tw[k][w] = tw;
        Ghw[k][w] = hw;
        Glw[k][w] = lw;
        t1 = dot4(tw, 0x01010101u, t1);
        t4 = dot4(tw, tw, t4);
        gh = dot4(hw, 0x01010101u, gh);
        gl = dot4(lw, 0x01010101u, gl);
        hh = dot4(hw, hw, hh);
        hl = dot4(hw, lw, hl);
        ll = dot4(lw, lw, ll);
        ht = dot4(hw, tw, ht);
        lt = dot4(lw, tw, lt);
      }
      if (rlive[k]) {
        // with g = Gx + 1024 = 256 Gh + Gl: sum Gx = sum g - 1024 P,
        // sum Gx^2 = sum g^2 - 2048 sum g + 1024^2 P, sum Gx T = sum g T - 1024 sum T
        const int sg = 256 * (int)gh + (int)gl;
        const int sgg = 65536 * (int)hh + 512 * (int)hl + (int)ll;
        sG += sg - 1024 * P;
        sT += (int)t1;
        sGG += sgg - 2048 * sg + 1048576 * P;
        sGT += 256 * (int)ht + (int)lt - 1024 * (int)t1;
        sTT += (int)t4;
      }
#pragma unroll
      for (int p = 0; p < NPAIR; ++p) {
        Pu[p] = Pc[p];
        Pc[p] = Pd[p];
      }
#pragma unroll
      for (int w = 0; w <= NW; ++w) Bc[w] = Bd[w];
    }
  }
  const int sT_lane = sT, sTT_lane = sTT;  // this lane's rows (the window sums below are per lane)
  sG = group_sum<G>(sG);
  sT = group_sum<G>(sT);
  sGG = group_sum<G>(sGG);
  sGT = group_sum<G>(sGT);
  const double Hs = exact_ab_cd(N, sGG, sG, sG);  // = 64 N H, exact
  const double H = Hs / (64.0 * N);
  const bool invert = H >= kEpsH;
  const double step = invert ? 8.0 / Hs : 0.0;

  const uint8_t* win = s_right;
  const uint8_t* grow = a.R + (size_t)oy * a.pitch;

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
        // E(m) and E(m + 1).  With several rows per lane (throughput-bound
        // mappings), a step into a neighbouring cell keeps the shared end's
        // value and correlates one position; the whole wavefront skips the
        // second position when none of its patches jumped further.  One row per
        // lane (latency-bound mappings) always correlates both positions, which
        // keeps the two dependent chains interleaved.
        constexpr bool kReuse = R >= 2;
        const bool up = kReuse && m == mc + 1, down = kReuse && mc == m + 1, both = !up && !down;
        const int pos = up ? m + 1 : m;
        int cg0 = 0, cs0 = 0, cg1 = 0, cs1 = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          uint32_t B[NW + 1];
          fetch_words<NW>(B, win + rrow[k] * RWB, xs, rw, grow + (size_t)rrow[k] * a.pitch, ox + pos, W);
          uint32_t h0 = 0, l0 = 0, s0 = 0;
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            h0 = dot4(B[w], Ghw[k][w], h0);
            l0 = dot4(B[w], Glw[k][w], l0);
            s0 = dot4(B[w], ones_word(w, P), s0);
          }
          if (rlive[k]) {
            cg0 += 256 * (int)h0 + (int)l0 - 1024 * (int)s0;
            cs0 += (int)s0;
          }
          if (both) {
            uint32_t h1 = 0, l1 = 0, s1 = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
              const uint32_t a1 = shifted_word<NW, 1>(B, w);
              h1 = dot4(a1, Ghw[k][w], h1);
              l1 = dot4(a1, Glw[k][w], l1);
              s1 = dot4(a1, ones_word(w, P), s1);
            }
            if (rlive[k]) {
              cg1 += 256 * (int)h1 + (int)l1 - 1024 * (int)s1;
              cs1 += (int)s1;
            }
          }
        }
        cg0 = group_sum<G>(cg0);
        cs0 = group_sum<G>(cs0);
        const double En = exact_ab_cd(N, cg0 - sGT, sG, cs0 - sT);
        if (both) {
          cg1 = group_sum<G>(cg1);
          cs1 = group_sum<G>(cs1);
          E0 = En;
          E1 = exact_ab_cd(N, cg1 - sGT, sG, cs1 - sT);
        } else if (up) {
          E0 = E1;
          E1 = En;
        } else {
          E1 = E0;
          E0 = En;
        }
        mc = m;
      }
      u = fma(-fma(f, E1, (1.0 - f) * E0), step, u);
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
    // With A_j the P samples from column m - 1 + j of a row (j = 0..3):
    //   sum a = S_q - sum T,  sum d = S_{q+1} - S_q,
    //   sum a^2 = AA_q - 2 TA_q + TT,  sum d^2 = AA_{q+1} - 2 AB_q + AA_q,
    //   sum a d = AB_q - AA_q - TA_{q+1} + TA_q,
    // S_j = sum A_j, AA_j = A_j . A_j, AB_j = A_j . A_{j+1}, TA_j = T . A_j.
    int gS[4] = {0, 0, 0, 0}, gAA[4] = {0, 0, 0, 0}, gAB[3] = {0, 0, 0}, gTA[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < R; ++k) {
      uint32_t B[NW + 1];
      fetch_words<NW>(B, win + rrow[k] * RWB, xs, rw, grow + (size_t)rrow[k] * a.pitch, ox + m - 1, W);
      uint32_t A[4][NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        A[0][w] = shifted_word<NW, 0>(B, w) & valid_bytes(w, P);
        A[1][w] = shifted_word<NW, 1>(B, w) & valid_bytes(w, P);
        A[2][w] = shifted_word<NW, 2>(B, w) & valid_bytes(w, P);
        A[3][w] = shifted_word<NW, 3>(B, w) & valid_bytes(w, P);
      }
      uint32_t S4[4] = {0, 0, 0, 0}, AA[4] = {0, 0, 0, 0}, AB[3] = {0, 0, 0}, TA[4] = {0, 0, 0, 0};
#pragma unroll
      for (int w = 0; w < NW; ++w) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          S4[jj] = dot4(A[jj][w], ones_word(w, P), S4[jj]);
          AA[jj] = dot4(A[jj][w], A[jj][w], AA[jj]);
          TA[jj] = dot4(A[jj][w], Tw[k][w], TA[jj]);
        }
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) AB[jj] = dot4(A[jj][w], A[jj + 1][w], AB[jj]);
      }
      if (rlive[k]) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          gS[jj] += (int)S4[jj];
          gAA[jj] += (int)AA[jj];
          gTA[jj] += (int)TA[jj];
        }
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) gAB[jj] += (int)AB[jj];
      }
    }
#pragma unroll
    for (int cq = 0; cq < 3; ++cq) {
      const int sa = group_sum<G>(gS[cq] - sT_lane);
      const int sd = group_sum<G>(gS[cq + 1] - gS[cq]);
      const int saa = group_sum<G>(gAA[cq] - 2 * gTA[cq] + sTT_lane);
      const int sdd = group_sum<G>(gAA[cq + 1] - 2 * gAB[cq] + gAA[cq]);
      const int sad = group_sum<G>(gAB[cq] - gAA[cq] - gTA[cq + 1] + gTA[cq]);
      X0[cq] = exact_ab_cd(N, saa, sa, sa);
      X1[cq] = exact_ab_cd(N, sad, sa, sd);
      X2[cq] = exact_ab_cd(N, sdd, sd, sd);
    }
  }
  constexpr double kInvN = 1.0 / (double)N;  // SSD = [X0 + 2 f X1 + f^2 X2] / N, by the rounded 1/N
  auto ssd = [&](int cq, double fr) { return fma(fr, fma(fr, X2[cq], 2.0 * X1[cq]), X0[cq]) * kInvN; };
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
  // The candidates come from one rounded subtraction each, so they are at most
  // one column off the rounded predicate's boundary (each moves only when the
  // boundary lies within an ulp of an integer); two correcting steps each way.
  int clo = (int)fmin(fmax(ceil(-(double)ox - u), 0.0), (double)P);
  int chi = (int)fmin(fmax(floor((double)(W - 1 - ox) - u), -1.0), (double)(P - 1));
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    if (clo > 0 && inside_lo(clo - 1)) --clo;
    else if (clo < P && !inside_lo(clo)) ++clo;
    if (chi < P - 1 && inside_hi(chi + 1)) ++chi;
    else if (chi >= 0 && !inside_hi(chi)) --chi;
  }
  const int inb = chi >= clo ? chi - clo + 1 : 0;
  const double rho = (double)(inb * P) / (double)N;
  const bool acc = s0 <= sm1 && s0 <= smh && s0 <= sph && s0 <= sp1 && rho >= (double)lp.valid_ratio;
  return PatchOut{u, s0, D4{sm1 - s0, smh - s0, sph - s0, sp1 - s0}, rho, H, acc};
}

}  // namespace

}  // namespace bdis
