// Image pyramid of both views (one pixel of level n covers 2^n x 2^n input
// pixels, Sec. III-B).  Separable binomial [1 4 6 4 1]/16 with reflect-101
// borders, sampled at even pixels, integer rounding (sum + 128) >> 8: exact
// uint8 arithmetic, bit-identical to any correct implementation.
//
// One workgroup computes a 64 x 4 tile of level n for both views of one pair:
// the 11 source rows it needs are filtered horizontally into LDS (integer),
// then the vertical pass reads them back.  The kernel moves ~1.33x the
// level-(n-1) bytes: HBM/latency bound and small next to the patch search.
#include "bdis_internal.h"

namespace bdis {

namespace {

constexpr int kSrcRows = 2 * kPyrTy + 3;  // source rows touched by kPyrTy output rows

__global__ __launch_bounds__(kPyrTx* kPyrTy) void k_pyr_u8(const PairLevel* tab, int npairs) {
  __shared__ int hL[kSrcRows][kPyrTx];
  __shared__ int hR[kSrcRows][kPyrTx];
  const int b = xcd_block();
  const PairLevel& a = tab[find_pair<0>(tab, npairs, b)];
  const int tiles_x = (a.g.w + kPyrTx - 1) / kPyrTx;
  const int t = b - a.pyr0;
  const int tx = threadIdx.x % kPyrTx;
  const int ty = threadIdx.x / kPyrTx;
  const int x = (t % tiles_x) * kPyrTx + tx;    // output column
  const int y0 = (t / tiles_x) * kPyrTy;        // first output row of the tile
  const int dw = a.g.w, dh = a.g.h;
  const int xs = x < dw ? x : dw - 1;           // idle lanes read valid columns
  const int cx[5] = {reflect101(2 * xs - 2, a.sw), reflect101(2 * xs - 1, a.sw), reflect101(2 * xs, a.sw),
                     reflect101(2 * xs + 1, a.sw), reflect101(2 * xs + 2, a.sw)};
  for (int r = ty; r < kSrcRows; r += kPyrTy) {
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
  const int q = 2 * ty;  // local row of source row 2*y-2
  const int sl = hL[q][tx] + 4 * hL[q + 1][tx] + 6 * hL[q + 2][tx] + 4 * hL[q + 3][tx] + hL[q + 4][tx];
  const int sr = hR[q][tx] + 4 * hR[q + 1][tx] + 6 * hR[q + 2][tx] + 4 * hR[q + 3][tx] + hR[q + 4][tx];
  gbl(a.dstL)[(size_t)y * a.pitch + x] = (uint8_t)((sl + 128) >> 8);
  gbl(a.dstR)[(size_t)y * a.pitch + x] = (uint8_t)((sr + 128) >> 8);
}

}  // namespace

hipError_t launch_pyramid(const PairLevel* tab, int npairs, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pyr_u8, dim3(nblocks), dim3(kPyrTx * kPyrTy), 0, s, tab, npairs);
  return hipGetLastError();
}

}  // namespace bdis
