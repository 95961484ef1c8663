// Internal declarations shared by the gfx950 kernels and the C-ABI runtime.
// Nothing here is part of the public interface (include/bdis.h).
//
// Every kernel works on a batch: a launch covers one phase (pyramid level,
// patch search, patch probability or fusion) of one pyramid level for every
// pair of the batch that has that level.  Per-pair geometry and pointers live
// in a device-resident job table (one PairLevel per pair and level); each
// workgroup finds its pair by a binary search over the table's workgroup
// offsets, so uneven sizes and pyramid depths share one launch.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

namespace bdis {

constexpr double kEpsH = 1e-3;   // smallest Hessian that is inverted
constexpr double kEpsSigma = 1e-6;
constexpr int kMaxPatch = 16;    // largest patch side
constexpr int kMaxLevels = 8;
constexpr int kWin = 5;          // samples of the Bayesian window

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
  double* uinit;  // initial displacement (from the parent level)           [kept]
  double* pipar;  // probability propagated from the parent level
  double* u;      // final displacement
  double* ssd0;   // window SSD at the centre                               [kept]
  D4* dssd;       // SSD(d) - SSD(0), d = -1, -1/2, +1/2, +1
  float* rho;     // in-bounds ratio (exact in FP32: a multiple of 1/P)     [kept]
  int* acc;       // 1 accepted
  float* hess;    // Gauss-Newton Hessian of the patch                      [kept]
  D4* dens;       // (u, weight: pi if accepted else -1, sigma_k^2, post)  [kept on
                  // levels whose records the fusion computes itself]
};
// [kept]: written only when the launch stores every intermediate (LevelParams::keep).

// One pair at one pyramid level: everything a workgroup of any phase needs.
struct PairLevel {
  // pyramid phase: level n from level n-1 (unused at n = 0)
  const uint8_t* srcL;
  const uint8_t* srcR;
  int spitch, sw, sh;
  // this level's images (level 0: the caller's inputs)
  const uint8_t* L;
  const uint8_t* R;
  int pitch;       // row pitch of L and R (level images in the workspace: 64-byte rows)
  uint8_t* dstL;   // == L for n >= 1 (written by the pyramid phase, row pitch `pitch`)
  uint8_t* dstR;
  LevelGeom g;
  int levels;      // the pair's pyramid depth
  // parent maps (nullptr at the pair's coarsest level)
  const double* par_ubar;
  const double* par_q;
  int pw, ph;
  PatchArrays pa;
  // sigma_r reduction of this pair and level, one partial per search
  // workgroup: the sum of SSD(0) over its accepted patches (uint8 path: the
  // exact fixed-point sums of the low and high 32-bit halves as two uint64 at
  // 2 b and 2 b + 1; float path: a double at b) and their count
  double* part_sum;
  int* part_cnt;
  double* scal;    // [sigma_r^2, tau, pooled residual, accepted count, d loss / d tau, SSD(0) adjoint share]
  // fusion outputs: level maps above the finest, user outputs at the finest
  double* ubar;
  double* qmap;
  float* disparity;
  float* variance;
  float* confidence;
  // finest level f > 0, on the level-0 entry: the level-f output maps (dense
  // fw x fh) that are upsampled into the outputs above
  const float* fdisp;
  const float* fvar;
  const float* fconf;
  int fw, fh, fshift;
  // optical-flow form, finest level: the flow outputs (dense w x h)
  float* flow_u;
  float* flow_v;
  // workgroup offsets of this pair in each flattened launch
  int pyr0, search0, prob0, fuse0, up0;
  int search_nbx;  // search workgroups per patch row

  // ---- float (differentiable) path: FP64 level images, pitch in elements
  const float* src32L;   // level 0 only: the caller's float images
  const float* src32R;
  int src32pitch;
  const double* srcdL;   // level n-1 (n >= 1)
  const double* srcdR;
  int srcdpitch;
  double* Ld;            // this level
  double* Rd;
  int dpitch;
  // state kept for the backward pass (training contexts)
  double* uhist;         // per patch: u_0 .. u_K of the iterations (K + 1 values)
  int* reset;            // per patch: 1 if the search threshold reset u to u_0
  double* zmap;          // per pixel: sum W (0 marks a hole)
  double* smmap;         // per pixel: sum M over accepted covering patches
  double* vmap;          // per pixel (finest level): variance
  double* ubar_keep;     // finest level: fused displacement and confidence
  double* qmap_keep;
  // adjoints (training contexts)
  double* Lbar;          // d loss / d level image
  double* Rbar;
  const double* upLbar;  // d loss / d level n+1 images (nullptr at the coarsest level)
  const double* upRbar;
  int upw, uph, updpitch;
  double* Gbar;          // d loss / d template gradient (Sobel / 8) image
  double* ubar_adj;      // d loss / d fused maps of this level
  double* qmap_adj;
  double* par_ubar_adj;  // d loss / d parent maps (nullptr at the coarsest level)
  double* par_qmap_adj;
  double* pu_adj;        // per patch: d loss / d u, d pi, d sigma_k^2
  double* ppi_adj;
  double* psig_adj;
  double* pssd_adj;      // per patch: d loss / d SSD(d), 5 values
  const float* grad_disp;  // finest level: caller's d loss / d disparity, variance
  const float* grad_var;
  float* grad_left;        // level 0: caller's image gradients (dense W x H)
  float* grad_right;
  double* hyper_adj;       // [sigma_s, sigma_r or alpha_r, omega_0 .. omega_7] (atomically summed)
};

// Parameters shared by all pairs of a launch.
struct LevelParams {
  int level;        // n
  int finest;       // f
  int P, S, K;
  float valid_ratio;
  int sigma_r_dynamic;
  float sigma_r;
  float omega[kMaxLevels];
  int variance;
  float var_fit_thresh;
  float var_fail_sigma;  // <= 0 means P
  float sigma_s;
  float prob_thresh;
  int fusion;       // 0 Eq. 13, 1 Eq. 2 (DIS), 2 Eq. 13 with a uniform mask
  int propagate;    // 1: add the parent confidence (Eq. 11)
  int inline_prob;  // 1: the fusion computes the level scalars and patch records itself (small levels)
  int fuse_ty;      // fusion tile height (kFuseTyShort, kFuseTyTall or kFuseTyHuge)
  int fuse_rec;     // patch records a fusion workgroup stages (<= kFuseMaxRec), fuse_lds_bytes
  int fuse_sep;     // staged patch rows with separable column sums (<= fuse_sep_rows(fuse_ty))
  int keep;         // 1: store every per-patch intermediate (debug dumps, training), else
                    // only what the later phases read
  int f64_sums;     // 1: the float path's search partials (doubles), else the exact sums
  int wide_win;     // 1: the search stages its whole right window (small launches), else
                    // only the columns around its patches' starting range
  // 1-D mixture mask m(a) = sum_c exp(-(a - c)^2 / (2 sigma_s^2)), a = 0..P-1
  // (Eq. 9-10), and its derivative in sigma_s, evaluated once on the host
  double mask[kMaxPatch];
  double dmask[kMaxPatch];
};

// Tile shapes of the flattened launches.
// Pyramid tiles: 64 x 4 output pixels (small levels) or 120 x 12 (levels of at
// least kPyrTallPixels pixels over the batch).
constexpr int kPyrSmallTx = 64, kPyrSmallTy = 4, kPyrTallTx = 120, kPyrTallTy = 12;
constexpr long kPyrTallPixels = 1 << 18;
constexpr int kProbThreads = 256;           // probability: patches per workgroup
// Levels with at most this many patches (over the batch) have their level
// scalars (sigma_r, tau) and patch records computed inside the fusion (no
// reduction or probability launch); larger levels compute each once in
// launches of their own.
constexpr long kInlineProbPatches = 1 << 16;
// Fusion tiles: 64 x 4 pixels, one per lane of 256 (small levels, many
// workgroups), 64 x 16, two per lane of 512 (levels of at least
// kFuseTallPixels pixels over the batch: fewer re-staged patch records), or
// 64 x 32, four per lane of 512 (levels of at least kFuseHugePixels).
constexpr int kFuseTx = 64, kFuseTyShort = 4, kFuseTyTall = 16, kFuseTyHuge = 32;
constexpr long kFuseTallPixels = 1 << 18, kFuseHugePixels = 1 << 22;
__host__ __device__ constexpr int fuse_threads(int ty) { return ty == kFuseTyShort ? 256 : 512; }
__host__ __device__ constexpr bool fuse_ty_ok(int ty) {
  return ty == kFuseTyShort || ty == kFuseTyTall || ty == kFuseTyHuge;
}
// Patch records a fusion workgroup stages, and the staged patch rows whose
// column sums the separable form keeps, per tile height.
constexpr int kFuseMaxRec = 512;
__host__ __device__ constexpr int fuse_sep_rows(int ty) {
  return ty == kFuseTyHuge ? 16 : (ty == kFuseTyTall ? 12 : 8);
}
// Dynamic LDS of a fusion workgroup: three record arrays, then the column sums.
__host__ __device__ constexpr int fuse_lds_bytes(int rec, int sep) {
  return 8 * (3 * rec + 4 * kFuseTx * sep);
}
// Whether the patches covering any tile of height ty (at most (ty + P - 1) / S
// + 1 grid rows plus the border patch, likewise for the 64 columns) fit both.
__host__ __device__ constexpr bool fuse_tile_fits(int ty, int P, int S) {
  return (ty + P - 1) / S + 2 <= fuse_sep_rows(ty) &&
         ((kFuseTx + P - 1) / S + 2) * ((ty + P - 1) / S + 2) <= kFuseMaxRec;
}

// Workgroups of the float-path search (fixed size) and of per-pixel adjoint launches.
constexpr int kSearchF64Threads = 256;
// Columns of the float-path search's staged right-image window: the patch
// origins' span, a margin of P + 4 each side and 128 columns of disparity
// spread, capped at 40 KB of LDS for the P rows.
__host__ __device__ inline int f64_window_cols(int P, int S) {
  const int npb = kSearchF64Threads / group_lanes(P);
  const int want = (npb - 1) * S + P + 2 * (P + 4) + 2 + 128;
  const int cap = 40 * 1024 / (8 * P);
  return want < cap ? want : cap;
}
constexpr size_t kAdjTileBytes = 64 * 1024;  // LDS accumulation tiles of the search adjoint
constexpr int kPixThreads = 256;

// Uint8 search configurations the tuner may pick per level: a lane mapping
// (kind) and a workgroup size.  Kind k puts G = search_lanes(P, k) lanes on a
// patch, each lane holding R = ceil(P / G) consecutive patch rows: kind 0 one
// row per lane (short per-lane chains, for latency-bound small levels), kinds
// 1 and 2 two and three-to-four rows per lane (the per-patch iteration logic
// repeated on fewer lanes, for throughput-bound large levels).
constexpr int kSearchKinds = 3;
constexpr int kNumSearchThreads = 4;
constexpr int kSearchThreadOptions[kNumSearchThreads] = {64, 128, 256, 512};
constexpr int kNumSearchOptions = kSearchKinds * kNumSearchThreads;

__host__ __device__ constexpr int search_lanes(int P, int kind) {
  return kind == 0 ? (P <= 8 ? 8 : 16) : kind == 1 ? (P <= 8 ? 4 : 8) : (P <= 8 ? 2 : (P <= 12 ? 4 : 8));
}
__host__ __device__ inline int search_option_threads(int opt) { return kSearchThreadOptions[opt % kNumSearchThreads]; }
__host__ __device__ inline int search_option_kind(int opt) { return opt / kNumSearchThreads; }
__host__ __device__ inline int search_patches_per_block(int P, int opt) {
  return search_option_threads(opt) / search_lanes(P, search_option_kind(opt));
}

// Columns of disparity spread among a workgroup's patches that the staged
// right-image window absorbs; samples beyond it are read from global memory.
constexpr int kWinSpread = 384;
constexpr int kSearchMaxLds = 64 * 1024;

// LDS layout of a uint8 search workgroup of `npb` patches at stride S: the left
// tile holds P + 2 rows of `ltw` bytes (patch columns plus the Sobel border,
// from a 4-aligned start), the right window P rows of `rwb` bytes.
__host__ __device__ inline void search_lds_layout(int P, int npb, int S, int& ltw, int& rwb) {
  const int span = (npb - 1) * S + P;  // columns covered by the patch origins
  ltw = (span + 8) / 4 * 4;
  rwb = (span + 2 * (P + 4) + 8 + kWinSpread + 15) / 16 * 16;
}
__host__ __device__ inline int search_lds_bytes(int P, int opt, int S) {
  int ltw, rwb;
  search_lds_layout(P, search_patches_per_block(P, opt), S, ltw, rwb);
  return (P + 2) * ltw + P * rwb;
}

// The level sum behind sigma_r (Sec. III-B) on the uint8 path is exact: each
// accepted patch's SSD(0) is rounded once to a multiple of 2^-36 (an integer
// below 2^63: SSD(0) <= (2 * 255)^2 P^2 < 2^27), split into its high and low
// 32-bit halves, and the halves are summed separately in 64 bits (below 2^55
// for any level of up to 2^23 patches, so no carries), so the sum does not
// depend on how patches are grouped into workgroups or in which order partials
// are added (search configuration, batch composition, reduction shape).  The
// rounding is far below the FP64 rounding of a sequential sum of the values.
constexpr double kSumScale = 68719476736.0;          // 2^36
constexpr double kSumInvScale = 1.0 / 68719476736.0;  // exact
// An SSD(0) value as the fixed-point integer of the level sum (negative
// rounding residue of the closed form clamped to 0).
__host__ __device__ inline unsigned long long ssd_fixed(double ssd) {
  const double v = ssd > 0.0 ? ssd * kSumScale : 0.0;
  return v < 9.2e18 ? (unsigned long long)llrint(v) : 9200000000000000000ull;
}
// The sum from its half sums: (sum of high halves) 2^32 + (sum of low halves),
// scaled back (two roundings of an exact integer: the same bits every time).
__host__ __device__ inline double fixed_sum_value(unsigned long long hi_sum, unsigned long long lo_sum) {
  return ((double)hi_sum * 4294967296.0 + (double)lo_sum) * kSumInvScale;
}
// Upper bound of the search workgroups of a level (every configuration puts at
// least four patches of one row in a workgroup): sizes the partial arrays.
__host__ __device__ inline int max_partials(const LevelGeom& g) { return (g.nx + 3) / 4 * g.ny; }

// Launchers over a device table of `npairs` entries (each returns the launch status).
hipError_t launch_pyramid(const PairLevel* tab, int npairs, int nblocks, bool tall, hipStream_t s);
// Small pyramid levels n0 + 1 .. n0 + m in one launch (tiles of the top one;
// each workgroup stages the level-n0 region its tile depends on).
struct PyrChain {
  int first[kMaxLevels];  // first table entry of each level
  int n0, m;              // built from level n0: levels n0 + 1 .. n0 + m
  int tile;               // top-level tile edge
  int lds_half, lds;      // dynamic LDS: two halves (0: does not fit)
};
PyrChain pyr_chain_shape(int n0, int m, int tile_top);
hipError_t launch_pyr_chain(const PairLevel* tab, int npairs, int nblocks, const PyrChain& ca, hipStream_t s);
hipError_t launch_search(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp,
                         int opt, hipStream_t s);
hipError_t launch_reduce(const PairLevel* tab, int npairs, const LevelParams& lp, hipStream_t s);
hipError_t launch_prob(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s);
hipError_t launch_fuse(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp,
                       hipStream_t s);
hipError_t launch_upsample(const PairLevel* tab, int npairs, int nblocks, hipStream_t s);
// The coarsest level of each pair in one workgroup (pyramid step, search, level
// scalars, records and fusion of that level): lanes per patch (0: the level
// takes the per-phase launches) and the dynamic LDS layout in bytes.
struct TopShape {
  int g;                  // lanes per patch
  int sw4, src_rows;      // row stride and rows of one staged view of the level below
  int img_px;             // bytes of one plain level image
  int ltw, rwb;           // row strides of the search's left (rows -1 .. h) and right views
  int np_max;             // patches of the largest pair of the launch
  int off_img, off_left, off_right, off_pat;
  int lds;
};
TopShape top_shape(int P, int S, int maxw, int maxh, int maxsw, int maxsh, int maxnp);
hipError_t launch_top(const PairLevel* tab, int npairs, const LevelParams& lp, const TopShape& ts, hipStream_t s);
hipError_t launch_coverage(const float* disp, const float* var, const float* ref, const uint8_t* valid, int w,
                           int h, int pitch, double k, unsigned long long* counts, hipStream_t s);
hipError_t launch_flow_search(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s);
hipError_t launch_flow_fuse(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp, hipStream_t s);
hipError_t launch_depth(const float* disp, const float* var, int w, int h, int pitch, float fb, float* depth,
                        float* dvar, hipStream_t s);

// Float (differentiable) path: FP64 pyramid and search, and the adjoint kernels.
hipError_t launch_pyramid_f64(const PairLevel* tab, int npairs, int nblocks, int level, hipStream_t s);
hipError_t launch_search_f64(const PairLevel* tab, int npairs, int nblocks, const LevelParams& lp,
                             hipStream_t s);
// sobel_in_pyramid: the level's transposed template gradient is left to the
// pyramid adjoint launch of the same level (launch_pyramid_adj with sobel).
hipError_t launch_backward_level(const PairLevel* tab, int npairs, const int* blocks, const LevelParams& lp,
                                 bool sobel_in_pyramid, hipStream_t s);
hipError_t launch_pyramid_adj(const PairLevel* tab, int npairs, int nblocks, bool sobel, hipStream_t s);
hipError_t launch_grad_out(const PairLevel* tab, int npairs, int nblocks, hipStream_t s);

// Per-kernel timing (bdis_timing_enable): the runtime hands the events of a
// timed launch to bdis_launch, which lets the kernel dispatch record them
// itself (hipExtLaunchKernelGGL): the first kernel of the launch records the
// start, every kernel the stop.  A timed span is then the kernels' own
// execution, as a profiler's kernel trace reports it, without the cost of
// separate event records.  Thread-local; set and cleared by the runtime.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool used = false;  // a kernel has recorded the start
};
LaunchEvents& launch_events();

template <typename F, typename... Args>
void bdis_launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
  LaunchEvents& ev = launch_events();
  if (ev.stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, ev.used ? nullptr : ev.start, ev.stop, 0u, args...);
    ev.used = true;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#ifdef __HIP_DEVICE_COMPILE__
#define BDIS_DEV __device__ __forceinline__
#else
#define BDIS_DEV __device__ inline
#endif

// Index of the table entry whose [first, next first) workgroup range holds
// workgroup `b` of a launch; Field selects the offset (0 pyramid, 1 search,
// 2 probability, 3 fusion).  Entries are stored in increasing offset order.
// Workgroups of a launch are handed to the 8 XCDs round-robin (workgroup b runs
// on XCD b mod 8, each XCD with its own L2).  The kernels whose neighbouring
// tiles share image rows index their work by this logical number instead, so
// that each XCD takes one contiguous range of tiles and the shared rows stay
// in its L2.  A bijection on [0, gridDim.x).
constexpr int kXcds = 8;
BDIS_DEV int xcd_block() {
  const int b = (int)blockIdx.x, n = (int)gridDim.x;
  const int x = b % kXcds, r = b / kXcds;
  return x * (n / kXcds) + min(x, n % kXcds) + r;
}

template <int Field>
BDIS_DEV int find_pair(const PairLevel* tab, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    int off;
    if constexpr (Field == 0) off = tab[mid].pyr0;
    else if constexpr (Field == 1) off = tab[mid].search0;
    else if constexpr (Field == 2) off = tab[mid].prob0;
    else if constexpr (Field == 3) off = tab[mid].fuse0;
    else off = tab[mid].up0;
    if (off <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// All-reduce (sum) of an int over an aligned group of G lanes (G = 1, 2, 4, 8
// or 16) with DPP lane permutations: quad swaps, then half-row and row mirrors.
template <int G>
BDIS_DEV int group_sum(int v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 2) v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
  if constexpr (G >= 16) v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);  // row_mirror
  return v;
}

// Global-address-space view of a pointer taken from the job table, so loads
// and stores compile to global_* rather than flat_* instructions (flat
// accesses also count against the LDS wait counter).
template <typename T>
BDIS_DEV __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Global loads / stores of a D4 record.
BDIS_DEV D4 ld4(const D4* p) {
  const auto q = gbl(reinterpret_cast<const double*>(p));
  return D4{q[0], q[1], q[2], q[3]};
}
BDIS_DEV void st4(D4* p, const D4& v) {
  auto q = gbl(reinterpret_cast<double*>(p));
  q[0] = v.x;
  q[1] = v.y;
  q[2] = v.z;
  q[3] = v.w;
}

// All-reduce (sum) of a double over an aligned group of G lanes (two 32-bit DPP moves per step).
template <int Ctrl>
BDIS_DEV double dpp_move_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), Ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Ctrl, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int G>
BDIS_DEV double group_sum_d(double v) {
  v += dpp_move_d<0xB1>(v);
  v += dpp_move_d<0x4E>(v);
  v += dpp_move_d<0x141>(v);
  if constexpr (G == 16) v += dpp_move_d<0x140>(v);
  return v;
}

// Sum over the 64 lanes of a wavefront of a 64-bit integer: DPP butterflies
// within each row of 16 lanes (no LDS round trips), then the four row sums
// read from lanes 0, 16, 32, 48.  Every lane returns the total.
template <int Ctrl>
BDIS_DEV unsigned long long dpp_move_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffull), Ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), Ctrl, 0xF, 0xF, true);
  return ((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo;
}
BDIS_DEV unsigned long long wave_sum_u64(unsigned long long v) {
  v += dpp_move_u64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move_u64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move_u64<0x141>(v);  // row_half_mirror
  v += dpp_move_u64<0x140>(v);  // row_mirror
  unsigned long long t = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(v & 0xffffffffull), 16 * r);
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(v >> 32), 16 * r);
    t += ((unsigned long long)hi << 32) | lo;
  }
  return t;
}
BDIS_DEV int wave_sum_i32(int v) {
  v = group_sum<16>(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
         __builtin_amdgcn_readlane(v, 48);
}

// Hardware FP64 atomic add on global memory (accumulation of adjoints).
BDIS_DEV void atomic_add_d(double* p, double v) { (void)__builtin_amdgcn_global_atomic_fadd_f64(gbl(p), v); }

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
  const auto g = gbl(m);
  const double top = (1.0 - ax) * g[(size_t)y0 * w + x0] + ax * g[(size_t)y0 * w + x1];
  const double bot = (1.0 - ax) * g[(size_t)y1 * w + x0] + ax * g[(size_t)y1 * w + x1];
  return (1.0 - ay) * top + ay * bot;
}

// The level scalars from the level sum of SSD(0) over the accepted patches
// and their count (Sec. III-B, Eq. 6): sigma_r^2 (the pooled per-pixel variance
// of the mean-normalised residual scaled by alpha_r^2 and floored, or the
// fixed alpha_r^2), tau = 2 sigma_r^2 s^2, the pooled residual, the count.
BDIS_DEV void level_scalars(const LevelParams& lp, double sum, long long cnt, double out[4]) {
  const double alpha2 = (double)lp.sigma_r * (double)lp.sigma_r;
  const double pooled = cnt > 0 ? sum / ((double)cnt * (double)(lp.P * lp.P)) : 0.0;
  const double sr2 = lp.sigma_r_dynamic ? alpha2 * (pooled > kEpsSigma ? pooled : kEpsSigma) : alpha2;
  out[0] = sr2;
  out[1] = 2.0 * sr2 * (double)(kWin * kWin);
  out[2] = pooled;
  out[3] = (double)cnt;
}

// sigma_r^(n) of one pair (called by a whole workgroup), read from Sec. III-B
// as the pooled per-pixel variance of the mean-normalised residual over the
// accepted patches of the level, scaled by alpha_r^2 and floored; or the fixed
// sigma_r.  tau = 2 sigma_r^2 s^2 (Eq. 6).  The search partials are summed in
// a fixed order (strided per thread, then a fixed tree), so every workgroup
// that calls this for a pair gets the same bits.  out: sigma_r^2, tau, pooled
// residual, accepted count.  Every thread returns the values.
BDIS_DEV void pair_scalars(const PairLevel& a, const LevelParams& lp, double* s_red, long long* s_redc,
                           double out[4]) {
  const int tid = threadIdx.x, nt = (int)blockDim.x;
  const int nblocks = a.search_nbx * a.g.ny;
  double sum;
  long long cnt;
  if (!lp.f64_sums) {
    // exact integer sums: any split and order give the same value, so every
    // thread strides over the partials, waves reduce by DPP and one barrier
    // combines the waves
    unsigned long long lo = 0, hi = 0;
    int c = 0;
    const auto ps = gbl(reinterpret_cast<const unsigned long long*>(a.part_sum));
    for (int b = tid; b < nblocks; b += nt) {
      lo += ps[2 * b];
      hi += ps[2 * b + 1];
      c += gbl(a.part_cnt)[b];
    }
    lo = wave_sum_u64(lo);
    hi = wave_sum_u64(hi);
    c = wave_sum_i32(c);
    unsigned long long* s_w = reinterpret_cast<unsigned long long*>(s_red);
    const int wave = tid / 64, nw = (nt + 63) / 64;
    if (tid % 64 == 0) {
      s_w[2 * wave] = lo;
      s_w[2 * wave + 1] = hi;
      s_redc[wave] = c;
    }
    __syncthreads();
    unsigned long long tlo = 0, thi = 0;
    cnt = 0;
    for (int w = 0; w < nw; ++w) {
      tlo += s_w[2 * w];
      thi += s_w[2 * w + 1];
      cnt += s_redc[w];
    }
    sum = fixed_sum_value(thi, tlo);
  } else {
    // float path: 256 virtual lanes (each thread takes every nt-th one when the
    // workgroup is smaller), the same sums in the same order at any size
    for (int vt = tid; vt < 256; vt += nt) {
      double ps = 0.0;
      long long pc = 0;
      for (int b = vt; b < nblocks; b += 256) {
        ps += gbl(a.part_sum)[b];
        pc += gbl(a.part_cnt)[b];
      }
      s_red[vt] = ps;
      s_redc[vt] = pc;
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      for (int vt = tid; vt < off; vt += nt) {
        s_red[vt] += s_red[vt + off];
        s_redc[vt] += s_redc[vt + off];
      }
      __syncthreads();
    }
    sum = s_red[0];
    cnt = s_redc[0];
  }
  __syncthreads();  // the buffers may be reused by the caller
  level_scalars(lp, sum, cnt, out);
}

// floor(a / d) for 0 <= a < 2^22 and 1 <= d <= 2^10: a float reciprocal
// estimate (error well below 1) corrected by one step each way, so exact; a
// few instructions instead of the generic integer division.
BDIS_DEV int div_small(int a, int d) {
  int q = (int)((float)a * __builtin_amdgcn_rcpf((float)d));
  q += (q + 1) * d <= a ? 1 : 0;
  q -= q * d > a ? 1 : 0;
  return q;
}

// Covering patches along one axis: indices lo..hi (origin i*S), plus the last
// patch (origin n-P) when it covers x but lies past hi.
BDIS_DEV void cover_range(int x, int n, int P, int S, int cnt, int& lo, int& hi, int& extra) {
  const int t = x - P;  // origin must exceed x - P
  lo = t >= 0 ? div_small(t, S) + 1 : 0;
  hi = min(div_small(x, S), cnt - 1);
  extra = (x >= n - P && cnt - 1 > hi) ? cnt - 1 : -1;
}

// Calls f(std::integral_constant<int, P>) for the runtime patch size.
template <typename F>
hipError_t by_patch(int P, F&& f) {
  switch (P) {
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 9: return f(std::integral_constant<int, 9>{});
    case 10: return f(std::integral_constant<int, 10>{});
    case 11: return f(std::integral_constant<int, 11>{});
    case 12: return f(std::integral_constant<int, 12>{});
    case 13: return f(std::integral_constant<int, 13>{});
    case 14: return f(std::integral_constant<int, 14>{});
    case 15: return f(std::integral_constant<int, 15>{});
    case 16: return f(std::integral_constant<int, 16>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdis
