// Internal declarations shared by the gfx950 kernels and the C-ABI runtime.
// Nothing here is part of the public interface (include/bdis.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdis {

constexpr int kThreads = 256;    // threads per workgroup of the patch kernels (4 waves)
constexpr int kWinRow = 512;     // columns of the right-image row window staged in LDS
constexpr double kEpsH = 1e-3;   // smallest Hessian that is inverted
constexpr double kEpsSigma = 1e-6;
constexpr int kMaxPatch = 16;    // largest patch side
constexpr int kMaxLevels = 8;

// Lanes that cooperate on one patch: one lane per patch row, rounded up to a
// power of two so that the group is a DPP quad / half-row / row.
constexpr int group_lanes(int P) { return P <= 8 ? 8 : 16; }

// Geometry of one pyramid level and its patch grid.  Origins along x are
// min(i*S, w-P), count ceil((w-P)/S)+1 (same along y).
struct LevelGeom {
  int w, h, nx, ny;
};

__host__ __device__ inline int grid_count(int n, int P, int S) { return (n - P + S - 1) / S + 1; }
__host__ __device__ inline int grid_origin(int i, int n, int P, int S) {
  int o = i * S;
  return o < n - P ? o : n - P;
}

// Four doubles (window SSD differences, or the fusion record of a patch).
struct alignas(16) D4 {
  double x, y, z, w;
};

// Per-level patch arrays (structure of arrays, one entry per patch).  The
// per-patch scalars are FP64: the method is ill-conditioned at patches whose
// iteration does not contract, and rounding this state to FP32 alone moves
// ~0.3% of output pixels by more than 1e-3 px.
struct PatchArrays {
  double* uinit;  // initial displacement (from the parent level)
  double* pipar;  // probability propagated from the parent level
  double* u;      // final displacement
  double* ssd0;   // window SSD at the centre
  D4* dssd;       // SSD(d) - SSD(0), d = -1, -1/2, +1/2, +1
  float* rho;     // in-bounds ratio (exact in FP32: a multiple of 1/P)
  int* acc;       // 1 accepted
  float* hess;    // Gauss-Newton Hessian of the patch
  D4* dens;       // (u, weight: pi if accepted else -1, sigma_k^2, post)
};

struct SearchArgs {
  const uint8_t* L;     // left level image
  const uint8_t* R;     // right level image
  int pitch;            // row pitch of both level images (elements)
  LevelGeom g;
  int S, K;
  float valid_ratio;
  const double* par_ubar;  // parent fused displacement (nullptr at the coarsest level)
  const double* par_q;     // parent fused confidence
  int pw, ph;              // parent level size
  PatchArrays pa;
  // level reduction for sigma_r: per-workgroup partials, reduced by the last
  // workgroup to finish (counter returns to 0 afterwards)
  double* part_sum;
  int* part_cnt;
  unsigned* counter;
  double* scal;           // out: [sigma_r^2, tau]
  int sigma_r_dynamic;
  float sigma_r;
};

struct ProbArgs {
  PatchArrays pa;
  int np;                 // patches in the level
  const double* scal;     // [sigma_r^2, tau]
  float omega[kMaxLevels];  // level weights; Gamma_n = omega_n / sum_{m=f}^{L-1} omega_m
  int level, finest, levels;
  int variance;           // compute sigma_k^2 (finest level)
  int P;
  float var_fit_thresh;
  float var_fail_sigma;   // <= 0 means P
};

struct DensifyArgs {
  const D4* dens;
  LevelGeom g;
  int P, S;
  float sigma_s;
  const double* par_ubar;  // parent maps for holes (nullptr at the coarsest level)
  const double* par_q;
  int pw, ph;
  int finest;              // 1: write the user outputs
  double* ubar;            // level maps (levels above the finest)
  double* qmap;
  float* disparity;       // user outputs (finest level)
  float* variance;        // nullable
  float* confidence;      // nullable
  int variance_on;
  float prob_thresh;
};

struct PyrArgs {
  const uint8_t* srcL;
  const uint8_t* srcR;
  int spitch, sw, sh;
  uint8_t* dstL;
  uint8_t* dstR;
  int dw, dh;
};

// Launchers (each returns the hipError_t of its launch).
hipError_t launch_pyramid_u8(const PyrArgs& a, hipStream_t s);
hipError_t launch_search_u8(int P, const SearchArgs& a, hipStream_t s);
hipError_t launch_prob(const ProbArgs& a, hipStream_t s);
hipError_t launch_densify(const DensifyArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#ifdef __HIP_DEVICE_COMPILE__
#define BDIS_DEV __device__ __forceinline__
#else
#define BDIS_DEV __device__ inline
#endif

// All-reduce (sum) of an int over an aligned group of G lanes (G = 8 or 16)
// with DPP lane permutations: quad swaps, then half-row and row mirrors.
template <int G>
BDIS_DEV int group_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
  if constexpr (G == 16) v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row_mirror
  return v;
}

// Reflect-101 index for |overshoot| < n (the only case the kernels produce).
BDIS_DEV int reflect101(int i, int n) {
  i = i < 0 ? -i : i;
  return i >= n ? 2 * (n - 1) - i : i;
}

BDIS_DEV int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bilinear sample of a w x h map at (x, y), indices clamped to the map.
BDIS_DEV double bilinear(const double* m, int w, int h, double x, double y) {
  const double fx0 = floor(x), fy0 = floor(y);
  const double ax = x - fx0, ay = y - fy0;
  const int ix = (int)fx0, iy = (int)fy0;
  const int x0 = clampi(ix, 0, w - 1), x1 = clampi(ix + 1, 0, w - 1);
  const int y0 = clampi(iy, 0, h - 1), y1 = clampi(iy + 1, 0, h - 1);
  const double top = (1.0 - ax) * m[(size_t)y0 * w + x0] + ax * m[(size_t)y0 * w + x1];
  const double bot = (1.0 - ax) * m[(size_t)y1 * w + x0] + ax * m[(size_t)y1 * w + x1];
  return (1.0 - ay) * top + ay * bot;
}

}  // namespace bdis
