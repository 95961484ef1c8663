// Optical-flow form of the search: the 2-D dense inverse search that BDIS
// builds on (Sec. III-A: Eq. 1 with the displacement u a 2-vector) and the
// DIS fusion of Eq. 2, on the same pyramid, patch grid and job table as the
// stereo path.
//
//   search  per patch, a group of lanes (one per patch row): template T,
//           J = (Sobel-x / 8, Sobel-y / 8) minus their patch means (reflect-101),
//           H = sum J J^T (2 x 2, group sums); K iterations of
//           (u, v) <- (u, v) - H^-1 sum J (I1(x + u, y + v) - T), bilinear in
//           both axes with indices clamped to the level; no update when
//           det H < 1e-3; reset to the start when the step from it exceeds P.
//   fuse    per pixel, over the covering patches: weight 1 / max(1, r^2),
//           r = I1(x + u_k) - I0(x); the fused (u, v) initialises the next
//           finer level (2 x bilinear at the patch centre / 2) or is the output.
//
// Per-patch flow lives in the patch arrays u (horizontal) and uinit
// (vertical); the fused level maps in ubar (horizontal) and qmap (vertical).
#include "bdis_internal.h"

#include <climits>

namespace bdis {

namespace {

// Bilinear sample of a uint8 level image at (x, y), indices clamped.
BDIS_DEV double bilinear_u8(const uint8_t* img, int pitch, int w, int h, double x, double y) {
  const double fx0 = floor(x), fy0 = floor(y);
  const double ax = x - fx0, ay = y - fy0;
  const int ix = (int)fx0, iy = (int)fy0;
  const int x0 = clampi(ix, 0, w - 1), x1 = clampi(ix + 1, 0, w - 1);
  const int y0 = clampi(iy, 0, h - 1), y1 = clampi(iy + 1, 0, h - 1);
  const auto g = gbl(img);
  const double top = (1.0 - ax) * (double)g[(size_t)y0 * pitch + x0] + ax * (double)g[(size_t)y0 * pitch + x1];
  const double bot = (1.0 - ax) * (double)g[(size_t)y1 * pitch + x0] + ax * (double)g[(size_t)y1 * pitch + x1];
  return (1.0 - ay) * top + ay * bot;
}

template <int P>
__global__ __launch_bounds__(kSearchF64Threads) void k_flow_search(const PairLevel* tab, int npairs, LevelParams lp) {
  constexpr int G = group_lanes(P);
  constexpr int NPB = kSearchF64Threads / G;
  constexpr int N = P * P;
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
  const int ox = grid_origin(i, W, P, S), oy = grid_origin(j, Hh, P, S);
  const bool row_live = r < P;
  const int rr = row_live ? r : P - 1;
  const auto I0 = gbl(a.L);
  const int pitch = a.pitch;
  const int y = oy + rr, ym = reflect101(y - 1, Hh), yp = reflect101(y + 1, Hh);
  auto px = [&](int yy, int xx) { return (double)I0[(size_t)yy * pitch + xx]; };

  double T[P], gx[P], gy[P];
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const int x = ox + c, xm = reflect101(x - 1, W), xp = reflect101(x + 1, W);
    T[c] = px(y, x);
    gx[c] = ((px(ym, xp) - px(ym, xm)) + 2.0 * (px(y, xp) - px(y, xm)) + (px(yp, xp) - px(yp, xm))) / 8.0;
    gy[c] = ((px(yp, xm) - px(ym, xm)) + 2.0 * (px(yp, x) - px(ym, x)) + (px(yp, xp) - px(ym, xp))) / 8.0;
    sx += gx[c];
    sy += gy[c];
  }
  const double mx = group_sum_d<G>(row_live ? sx : 0.0) / (double)N;
  const double my = group_sum_d<G>(row_live ? sy : 0.0) / (double)N;
  double hxx = 0.0, hxy = 0.0, hyy = 0.0;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    gx[c] -= mx;
    gy[c] -= my;
    hxx += gx[c] * gx[c];
    hxy += gx[c] * gy[c];
    hyy += gy[c] * gy[c];
  }
  hxx = group_sum_d<G>(row_live ? hxx : 0.0);
  hxy = group_sum_d<G>(row_live ? hxy : 0.0);
  hyy = group_sum_d<G>(row_live ? hyy : 0.0);
  const double det = hxx * hyy - hxy * hxy;

  double u0 = 0.0, v0 = 0.0;
  if (a.par_ubar) {  // the parent's fused flow at the patch centre, in this level's pixels
    const double cx = (double)ox + 0.5 * (double)(P - 1), cy = (double)oy + 0.5 * (double)(P - 1);
    u0 = 2.0 * bilinear(a.par_ubar, a.pw, a.ph, 0.5 * cx, 0.5 * cy);
    v0 = 2.0 * bilinear(a.par_q, a.pw, a.ph, 0.5 * cx, 0.5 * cy);
  }
  double u = u0, v = v0;
  if (det >= kEpsH) {
    // The warped row of this lane reads I1 rows y + n, y + n + 1 at columns
    // ox + m + c (c = 0..P), (m, n) = floor(u, v), all with the same bilinear
    // fractions; the 2 (P + 1) samples are kept while (m, n) stays the same.
    const auto I1 = gbl(a.R);
    double S0[P + 1], S1[P + 1];
    int mc = INT_MIN, nc = INT_MIN;
    for (int t = 0; t < lp.K; ++t) {
      const double fu = floor(u), fv = floor(v);
      const int m = (int)fu, n = (int)fv;
      const double ax = u - fu, ay = v - fv;
      if (m != mc || n != nc) {
        const size_t r0 = (size_t)clampi(y + n, 0, Hh - 1) * pitch, r1 = (size_t)clampi(y + n + 1, 0, Hh - 1) * pitch;
#pragma unroll
        for (int c = 0; c <= P; ++c) {
          const int xc = clampi(ox + m + c, 0, W - 1);
          S0[c] = (double)I1[r0 + xc];
          S1[c] = (double)I1[r1 + xc];
        }
        mc = m;
        nc = n;
      }
      double bx = 0.0, by = 0.0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const double top = (1.0 - ax) * S0[c] + ax * S0[c + 1];
        const double bot = (1.0 - ax) * S1[c] + ax * S1[c + 1];
        const double e = (1.0 - ay) * top + ay * bot - T[c];
        bx += gx[c] * e;
        by += gy[c] * e;
      }
      bx = group_sum_d<G>(row_live ? bx : 0.0);
      by = group_sum_d<G>(row_live ? by : 0.0);
      u -= (hyy * bx - hxy * by) / det;
      v -= (hxx * by - hxy * bx) / det;
    }
  }
  if ((u - u0) * (u - u0) + (v - v0) * (v - v0) > (double)P * (double)P) {
    u = u0;
    v = v0;
  }
  if (r == 0 && live) {
    gbl(a.pa.u)[k] = u;
    gbl(a.pa.uinit)[k] = v;
    gbl(a.pa.hess)[k] = (float)det;
  }
}

// Per pixel (fusion tiles of lp.fuse_ty rows): Eq. 2 fusion of the covering
// patches' flows.
__global__ __launch_bounds__(512) void k_flow_fuse(const PairLevel* tab, int npairs, LevelParams lp) {
  const int lb = xcd_block();
  const PairLevel& a = tab[find_pair<3>(tab, npairs, lb)];
  const int tid = threadIdx.x;
  const int P = lp.P, S = lp.S;
  const int tiles_x = (a.g.w + kFuseTx - 1) / kFuseTx;
  const int t = lb - a.fuse0;
  const int x = (t % tiles_x) * kFuseTx + tid % kFuseTx;
  if (x >= a.g.w) return;
  int ilo, ihi, iex;
  cover_range(x, a.g.w, P, S, a.g.nx, ilo, ihi, iex);
  const int iend = iex >= 0 ? ihi + 1 : ihi;
  const int ty = lp.fuse_ty, lanes_y = (int)blockDim.x / kFuseTx;
  for (int y = (t / tiles_x) * ty + tid / kFuseTx, yn = 0; yn < ty / lanes_y; ++yn, y += lanes_y) {
    if (y >= a.g.h) break;
    int jlo, jhi, jex;
    cover_range(y, a.g.h, P, S, a.g.ny, jlo, jhi, jex);
    const double l0 = (double)gbl(a.L)[(size_t)y * a.pitch + x];
    double z = 0.0, zu = 0.0, zv = 0.0;
    const int jend = jex >= 0 ? jhi + 1 : jhi;
    for (int jj = jlo; jj <= jend; ++jj) {
      const int j = jj <= jhi ? jj : jex;
      for (int ii = ilo; ii <= iend; ++ii) {
        const int i = ii <= ihi ? ii : iex;
        const size_t k = (size_t)j * a.g.nx + i;
        const double uk = gbl(a.pa.u)[k], vk = gbl(a.pa.uinit)[k];
        const double rres = bilinear_u8(a.R, a.pitch, a.g.w, a.g.h, (double)x + uk, (double)y + vk) - l0;
        const double wk = 1.0 / fmax(1.0, rres * rres);
        z += wk;
        zu += wk * uk;
        zv += wk * vk;
      }
    }
    const size_t idx = (size_t)y * a.g.w + x;
    const double fu = zu / z, fv = zv / z;  // every pixel is covered
    if (lp.level > lp.finest) {
      gbl(a.ubar)[idx] = fu;
      gbl(a.qmap)[idx] = fv;
    } else {
      gbl(a.flow_u)[idx] = (float)fu;
      gbl(a.flow_v)[idx] = (float)fv;
    }
  }
}

}  // namespace

hipError_t launch_flow_search(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  return by_patch(lp.P, [&](auto pc) {
    constexpr int P = decltype(pc)::value;
    bdis_launch(k_flow_search<P>, dim3(nblocks), dim3(kSearchF64Threads), 0, s, tab, npairs, lp);
    return hipGetLastError();
  });
}

hipError_t launch_flow_fuse(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (!fuse_ty_ok(lp.fuse_ty)) return hipErrorInvalidValue;
  bdis_launch(k_flow_fuse, dim3(nblocks), dim3(fuse_threads(lp.fuse_ty)), 0, s, tab, npairs, lp);
  return hipGetLastError();
}

}  // namespace bdis
