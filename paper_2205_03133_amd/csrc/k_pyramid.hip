// Image pyramid of both views (one pixel of level n covers 2^n x 2^n input
// pixels, Sec. III-B).  Separable binomial [1 4 6 4 1]/16 with reflect-101
// borders, sampled at even pixels, integer rounding (sum + 128) >> 8: exact
// uint8 arithmetic, bit-identical to any correct implementation.
//
// Layout: one workgroup computes a 64 x 4 tile of level n for both views.  The
// 5 source rows x (2*64+3) source columns it needs per output row pair are
// read once into LDS as the horizontally filtered rows (integer), then the
// vertical pass reads them back.  The kernel moves ~1.33x the level-(n-1)
// bytes, so it is HBM/latency bound and tiny next to the patch search.
#include "bdis_internal.h"

namespace bdis {

namespace {

constexpr int kTx = 64;   // output columns per tile
constexpr int kTy = 4;    // output rows per tile
constexpr int kSrcRows = 2 * kTy + 3;  // source rows touched by kTy output rows

__global__ __launch_bounds__(kTx * kTy) void k_pyr_u8(PyrArgs a) {
  // horizontally filtered source rows for both views: rows 2*y0-2 .. 2*y0+2*kTy
  __shared__ int hL[kSrcRows][kTx];
  __shared__ int hR[kSrcRows][kTx];
  const int tx = threadIdx.x % kTx;
  const int ty = threadIdx.x / kTx;
  const int x = blockIdx.x * kTx + tx;       // output column
  const int y0 = blockIdx.y * kTy;            // first output row of the tile
  const int xs = x < a.dw ? x : a.dw - 1;     // clamp idle lanes onto valid columns
  const int cx[5] = {reflect101(2 * xs - 2, a.sw), reflect101(2 * xs - 1, a.sw),
                     reflect101(2 * xs, a.sw), reflect101(2 * xs + 1, a.sw),
                     reflect101(2 * xs + 2, a.sw)};
  for (int r = ty; r < kSrcRows; r += kTy) {
    int sy = 2 * y0 - 2 + r;
    // rows beyond sh + 1 feed only idle output rows: keep them in range
    sy = sy > a.sh + 1 ? a.sh - 1 : reflect101(sy, a.sh);
    const uint8_t* rl = a.srcL + (size_t)sy * a.spitch;
    const uint8_t* rr = a.srcR + (size_t)sy * a.spitch;
    hL[r][tx] = rl[cx[0]] + 4 * rl[cx[1]] + 6 * rl[cx[2]] + 4 * rl[cx[3]] + rl[cx[4]];
    hR[r][tx] = rr[cx[0]] + 4 * rr[cx[1]] + 6 * rr[cx[2]] + 4 * rr[cx[3]] + rr[cx[4]];
  }
  __syncthreads();
  const int y = y0 + ty;
  if (x >= a.dw || y >= a.dh) return;
  const int b = 2 * ty;  // local row of source row 2*y-2
  int sl = hL[b][tx] + 4 * hL[b + 1][tx] + 6 * hL[b + 2][tx] + 4 * hL[b + 3][tx] + hL[b + 4][tx];
  int sr = hR[b][tx] + 4 * hR[b + 1][tx] + 6 * hR[b + 2][tx] + 4 * hR[b + 3][tx] + hR[b + 4][tx];
  a.dstL[(size_t)y * a.dw + x] = (uint8_t)((sl + 128) >> 8);
  a.dstR[(size_t)y * a.dw + x] = (uint8_t)((sr + 128) >> 8);
}

}  // namespace

hipError_t launch_pyramid_u8(const PyrArgs& a, hipStream_t s) {
  dim3 grid((a.dw + kTx - 1) / kTx, (a.dh + kTy - 1) / kTy);
  hipLaunchKernelGGL(k_pyr_u8, grid, dim3(kTx * kTy), 0, s, a);
  return hipGetLastError();
}

}  // namespace bdis
