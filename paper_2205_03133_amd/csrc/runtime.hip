// C-ABI runtime of the BDIS library: parameter validation, the device
// workspace, the per-level job tables and the launch sequence of one
// coarse-to-fine pass (Fig. 1) over a batch of pairs:
//   pyramid levels 1 .. L-1 of both views, then for n = L-1 .. f:
//     patch search (+ per-pair sigma_r reduction), patch probability, fusion,
// each phase one launch covering every pair that has level n.  The sequence
// is captured once per batch shape into a hipGraph and replayed; the job
// table (pointers) lives in device memory and is re-uploaded only when it
// changes.  Nothing here synchronises the host except bdis_create,
// bdis_destroy, bdis_debug_dump, the first call of a new batch shape (tuning)
// and bdis_timing_read.
#include <bdis.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "bdis_internal.h"

using namespace bdis;

namespace bdis {
LaunchEvents& launch_events() {
  static thread_local LaunchEvents ev;
  return ev;
}
}  // namespace bdis

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Host wall-clock time in ms (tuning and capture times).
double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Byte offsets of every array of one pair within its workspace slot.
struct Layout {
  int levels = 0;
  LevelGeom g[kMaxLevels]{};
  int lpitch[kMaxLevels]{};      // row pitch of the level images (64-byte rows)
  int sum_parts[kMaxLevels]{};
  size_t lvl_l[kMaxLevels]{}, lvl_r[kMaxLevels]{};
  size_t uinit[kMaxLevels]{}, pipar[kMaxLevels]{}, u[kMaxLevels]{}, ssd0[kMaxLevels]{},
      dssd[kMaxLevels]{}, rho[kMaxLevels]{}, acc[kMaxLevels]{}, hess[kMaxLevels]{},
      dens[kMaxLevels]{};
  size_t ubar[kMaxLevels]{}, qmap[kMaxLevels]{};
  size_t odisp = 0, ovar = 0, oconf = 0;  // finest level f > 0: outputs before upsampling
  size_t part_sum[kMaxLevels]{}, part_cnt[kMaxLevels]{}, scal[kMaxLevels]{};
  // training contexts: FP64 level images, saved state, adjoints (one region)
  bool train = false;
  int dpitch[kMaxLevels]{};
  size_t ld[kMaxLevels]{}, rd[kMaxLevels]{}, uhist[kMaxLevels]{}, reset[kMaxLevels]{}, zmap[kMaxLevels]{},
      smmap[kMaxLevels]{}, vmap = 0, ubar_keep = 0, qmap_keep = 0;
  size_t adj_begin = 0, adj_end = 0;
  size_t lbar[kMaxLevels]{}, rbar[kMaxLevels]{}, gbar[kMaxLevels]{}, ubar_adj[kMaxLevels]{},
      qmap_adj[kMaxLevels]{}, pu_adj[kMaxLevels]{}, ppi_adj[kMaxLevels]{},
      psig_adj[kMaxLevels]{}, pssd_adj[kMaxLevels]{};
  size_t total = 0;
};

int search_nbx(const LevelGeom& g, int npb) { return (g.nx + npb - 1) / npb; }

// Patches per search workgroup: the uint8 search in a tuned configuration
// (option index), or the fixed float-path / optical-flow search.
int search_npb(int P, int opt, bool f64_search) {
  return f64_search ? kSearchF64Threads / group_lanes(P) : search_patches_per_block(P, opt);
}

// Level sizes W_n = ceil(W_{n-1} / 2); the patch grid exists on processed levels.
bool level_geometry(const bdis_params& p, int w, int h, int levels, LevelGeom* g) {
  int lw = w, lh = h;
  for (int n = 0; n < levels; ++n) {
    g[n].w = lw;
    g[n].h = lh;
    if (n >= p.finest_level) {
      if (lw < p.patch || lh < p.patch) return false;
      g[n].nx = grid_count(lw, p.patch, p.stride);
      g[n].ny = grid_count(lh, p.patch, p.stride);
    } else {
      g[n].nx = g[n].ny = 0;
    }
    lw = (lw + 1) >> 1;
    lh = (lh + 1) >> 1;
  }
  return true;
}

bool make_layout(const bdis_params& p, int w, int h, int levels, Layout* lay, bool train = false) {
  Layout L;
  L.levels = levels;
  L.train = train;
  if (!level_geometry(p, w, h, levels, L.g)) return false;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  for (int n = 0; n < levels; ++n) {
    const size_t npx = (size_t)L.g[n].w * L.g[n].h;
    L.lpitch[n] = (L.g[n].w + 63) / 64 * 64;
    if (n >= 1) {
      L.lvl_l[n] = take((size_t)L.lpitch[n] * L.g[n].h);
      L.lvl_r[n] = take((size_t)L.lpitch[n] * L.g[n].h);
    }
    if (n < p.finest_level) continue;
    const size_t np = (size_t)L.g[n].nx * L.g[n].ny;
    L.uinit[n] = take(np * 8);
    L.pipar[n] = take(np * 8);
    L.u[n] = take(np * 8);
    L.ssd0[n] = take(np * 8);
    L.dssd[n] = take(np * sizeof(D4));
    L.rho[n] = take(np * 4);
    L.acc[n] = take(np * 4);
    L.hess[n] = take(np * 4);
    L.dens[n] = take(np * sizeof(D4));
    if (n > p.finest_level) {
      L.ubar[n] = take(npx * 8);
      L.qmap[n] = take(npx * 8);
    }
    if (n == p.finest_level && n > 0) {
      L.odisp = take(npx * 4);
      L.ovar = take(npx * 4);
      L.oconf = take(npx * 4);
    }
    // partials of the sigma_r reduction: one per search workgroup (16 bytes)
    L.sum_parts[n] = max_partials(L.g[n]);
    L.part_sum[n] = take((size_t)L.sum_parts[n] * 16);
    L.part_cnt[n] = take((size_t)L.sum_parts[n] * 4);
    L.scal[n] = take(64);
  }
  if (train) {
    const int f = p.finest_level;
    for (int n = 0; n < levels; ++n) {
      const size_t np = (size_t)L.g[n].nx * L.g[n].ny, npx = (size_t)L.g[n].w * L.g[n].h;
      L.dpitch[n] = (L.g[n].w + 7) / 8 * 8;
      const size_t nd = (size_t)L.dpitch[n] * L.g[n].h;
      L.ld[n] = take(nd * 8);
      L.rd[n] = take(nd * 8);
      if (n < f) continue;
      L.uhist[n] = take(np * (size_t)(p.iters + 1) * 8);
      L.reset[n] = take(np * 4);
      L.zmap[n] = take(npx * 8);
      L.smmap[n] = take(npx * 8);
      if (n == f) {
        L.vmap = take(npx * 8);
        L.ubar_keep = take(npx * 8);
        L.qmap_keep = take(npx * 8);
      }
    }
    L.adj_begin = off;
    for (int n = 0; n < levels; ++n) {
      const size_t np = (size_t)L.g[n].nx * L.g[n].ny, npx = (size_t)L.g[n].w * L.g[n].h;
      const size_t nd = (size_t)L.dpitch[n] * L.g[n].h;
      L.lbar[n] = take(nd * 8);
      L.rbar[n] = take(nd * 8);
      L.gbar[n] = take(nd * 8);
      if (n < f) continue;
      // the finest level's map adjoints are formed from the caller's output
      // gradients where they are read (the fusion adjoint): no buffers
      if (n > f) {
        L.ubar_adj[n] = take(npx * 8);
        L.qmap_adj[n] = take(npx * 8);
      }
      L.pu_adj[n] = take(np * 8);
      L.ppi_adj[n] = take(np * 8);
      L.psig_adj[n] = take(np * 8);
      L.pssd_adj[n] = take(np * kWin * 8);
    }
    L.adj_end = off;
  }
  L.total = off;
  *lay = L;
  return true;
}

bool finite_f(float v) { return std::isfinite(v); }

// One pair of a call, as validated.
struct PairSpec {
  const uint8_t* left;
  const uint8_t* right;
  int w, h, pitch, levels;
  float* disp;
  float* var;
  float* conf;
  // float path
  const float* left32 = nullptr;
  const float* right32 = nullptr;
  // backward
  const float* grad_disp = nullptr;
  const float* grad_var = nullptr;
  float* grad_left = nullptr;
  float* grad_right = nullptr;
  // optical-flow form
  float* flow_u = nullptr;
  float* flow_v = nullptr;
};

// Job-table entries of a plan: inline storage for the levels of one pair (a
// single-pair plan touches no heap), a heap vector beyond that.
struct PlanTab {
  PairLevel fixed[kMaxLevels];
  std::vector<PairLevel> heap;
  size_t n = 0;
  void push_back(const PairLevel& e) {
    if (heap.empty() && n < (size_t)kMaxLevels) {
      fixed[n++] = e;
      return;
    }
    if (heap.empty()) heap.assign(fixed, fixed + n);
    heap.push_back(e);
    ++n;
  }
  size_t size() const { return n; }
  PairLevel* data() { return heap.empty() ? fixed : heap.data(); }
  const PairLevel* data() const { return heap.empty() ? fixed : heap.data(); }
  PairLevel& operator[](size_t i) { return data()[i]; }
  const PairLevel& operator[](size_t i) const { return data()[i]; }
};

// Untuned plans run the coarsest level in k_top from this many pairs on (one
// workgroup per pair at once beats the level's launches there).
constexpr int kTopMinPairs = 8;

// Launch plan of one call: level-major job table and workgroup counts.
struct Plan {
  int max_levels = 0;
  int finest = 0;
  int tab_first[kMaxLevels]{};   // first table entry of level n
  int tab_count[kMaxLevels]{};   // entries (pairs having level n)
  int pyr_blocks[kMaxLevels]{}, search_blocks[kMaxLevels]{}, prob_blocks[kMaxLevels]{},
      fuse_blocks[kMaxLevels]{};
  bool flow = false;             // optical-flow search (fixed workgroups like the float path)
  int search_opt[kMaxLevels]{};  // uint8 search configuration per level (lane mapping, workgroup size)
  int up_blocks = 0;             // finest level f > 0: upsampling workgroups (level 0)
  int inline_prob[kMaxLevels]{}; // 1: the fusion computes the patch records (small levels)
  int fuse_ty[kMaxLevels]{};     // fusion tile height per level
  bool keep = false;             // store every per-patch intermediate (LevelParams::keep)
  bool pyr_tall[kMaxLevels]{};   // pyramid level built with the large-tile kernel
  bool f32 = false;              // float (FP64) path: per-pixel pyramid blocks, fixed search size
  int top_level = -1;            // level whose pyramid step, search and fusion run in k_top (-1: none)
  int top_fits = -1;             // the level k_top could take (-1: none)
  TopShape top{};                // its launch shape
  PyrChain chain{};              // small pyramid levels built by one launch (chain.m == 0: none)
  int chain_blocks = 0;
  PlanTab tab;
};

// HIP events recorded by the timed launches while timing is enabled.
struct TimingMark {
  int kernel, level;
  size_t idx;  // index of the start event (the stop event follows it)
};
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> pool;   // reused events
  size_t used = 0;                // events handed out since enable
  std::vector<TimingMark> marks;
};

// Launch shapes the tuner picked for one level shape (-1 / 0: not tuned, the
// size thresholds decide).
struct TuneChoice {
  int search = -1;   // uint8 search configuration (option index)
  int fuse_ty = 0;   // fusion tile height
  int pyr_tall = -1; // pyramid form: 1 staged 120 x 12 tiles, 0 gather 64 x 4 tiles
  int top = -1;      // coarsest level: 1 one workgroup per pair (k_top), 0 the per-phase launches
  int chain = -1;    // highest level of a pyramid chain: 1 one launch for the chained levels, 0 one each
};

// A captured launch sequence for one batch shape.
struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long used = 0;  // the context's launch count at its last launch
};
// Captured launch sequences a context keeps (one per batch shape and set of
// launch choices); beyond this the least recently launched one is destroyed.
constexpr size_t kMaxGraphs = 32;

}  // namespace

struct bdis_ctx {
  bdis_params p{};
  Timing tm;
  int max_w = 0, max_h = 0, max_batch = 0;
  size_t slot_bytes = 0;
  char* ws = nullptr;
  int device = 0;
  // device job table + pinned staging, uploaded only when its contents change
  PairLevel* tab_dev = nullptr;
  PairLevel* tab_host = nullptr;
  size_t tab_cap = 0;             // entries
  std::vector<PairLevel> tab_last;
  hipEvent_t tab_evt = nullptr;   // completion of the last upload
  bool tab_evt_live = false;
  hipEvent_t done_evt = nullptr;  // end of the last call's work (orders calls on other streams)
  hipStream_t done_stream = nullptr;
  bool done_live = false;
  bool multi_stream = false;      // calls have come on more than one stream
  hipStream_t capture_stream = nullptr;
  std::map<std::string, GraphEntry> graphs;
  unsigned long long graph_launches = 0;
  std::map<std::string, TuneChoice> tuned;  // level shape key -> tuned launch shapes of the level
  std::string arch;                  // gcnArchName of the device (part of the tuning keys)
  std::string tune_cache;            // file the tuned choices persist in ("" = none)
  double last_tune_ms = 0.0, last_capture_ms = 0.0;  // host time of the last call's tuning / capture
  int forced_opt = -1;               // BDIS_SEARCH_CONFIG: one configuration for every level, no tuning
  int top_mode = -1;                 // BDIS_TOP: 0 the coarsest level in per-phase launches, 1 in k_top
                                     // where it fits, unset: timed by the tuner
  int chain_mode = -1;               // BDIS_CHAIN: 0 one pyramid launch per level, 1 chained small
                                     // levels where possible, unset: timed by the tuner
  int use_graph = 1;
  bool train = false;                // created with BDIS_TRAIN
  bool keep = false;                 // created with BDIS_KEEP
  std::vector<PairSpec> last_f32;    // pairs of the last float-path call (backward state)
  double* hyper_dev = nullptr;       // d loss / d hyperparameters accumulator (2 + 8)
  // geometry of the last single-pair compute (slot 0), for debug dumps
  int last_w = 0, last_h = 0;
  bool have_last = false;
  char err[512] = {0};
};

namespace {

char g_create_err[512] = {0};

// Zeroes `n` bytes at `p` (16-byte stores for the aligned body, bytes at the
// ends): a kernel rather than a memset node, so that a call a caller captures
// into a graph replays correctly.
// Up to kZeroJobs byte ranges zeroed by one launch (blockIdx.y picks the range).
constexpr int kZeroJobs = 32;
struct ZeroJobs {
  unsigned char* p[kZeroJobs];
  size_t n[kZeroJobs];
};
__global__ __launch_bounds__(256) void k_zero_bytes(ZeroJobs jobs) {
  unsigned char* const p = jobs.p[blockIdx.y];
  const size_t n = jobs.n[blockIdx.y];
  const size_t head = std::min(n, (size_t)((16 - ((uintptr_t)p & 15)) & 15));
  const size_t n16 = (n - head) / 16;
  const size_t tail = head + 16 * n16;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4* body = reinterpret_cast<uint4*>(p + head);
  for (size_t i = t; i < n16; i += stride) body[i] = make_uint4(0u, 0u, 0u, 0u);
  if (t < head) p[t] = 0;
  if (t < n - tail) p[tail + t] = 0;
}
// The adjoint scalars of every entry of a job table (d loss / d tau, its share
// per accepted SSD(0), d loss / d Gamma): zeroed once per backward pass.
__global__ __launch_bounds__(64) void k_adj_scal_zero(const PairLevel* tab, int n) {
  const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= n) return;
  double* sc = tab[e].scal;
  sc[4] = 0.0;
  sc[5] = 0.0;
  sc[6] = 0.0;
}
// Zeroes the byte ranges (p[i], n[i]), i < count, kZeroJobs ranges per launch.
hipError_t zero_ranges(unsigned char* const* p, const size_t* n, int count, hipStream_t st) {
  for (int b = 0; b < count; b += kZeroJobs) {
    ZeroJobs jobs{};
    const int m = std::min(kZeroJobs, count - b);
    size_t most = 0;
    for (int i = 0; i < m; ++i) {
      jobs.p[i] = p[b + i];
      jobs.n[i] = n[b + i];
      most = std::max(most, n[b + i]);
    }
    if (most == 0) continue;
    const size_t n16 = most / 16 + 1;
    const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 4096);
    bdis_launch(k_zero_bytes, dim3(blocks, (unsigned)m), dim3(256), 0, st, jobs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

bdis_status fail(bdis_ctx* c, bdis_status st, const char* fmt, ...) {
  char* dst = c ? c->err : g_create_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return st;
}

bdis_status check_params_msg(const bdis_params* p, char* msg, size_t n) {
  if (!p) return snprintf(msg, n, "params is NULL"), BDIS_E_ARG;
  if (p->levels < 1 || p->levels > BDIS_MAX_LEVELS)
    return snprintf(msg, n, "levels %d outside 1..%d", p->levels, BDIS_MAX_LEVELS), BDIS_E_ARG;
  if (p->finest_level < 0 || p->finest_level >= p->levels)
    return snprintf(msg, n, "finest_level %d outside 0..levels-1", p->finest_level), BDIS_E_ARG;
  if (p->patch < 3 || p->patch > BDIS_MAX_PATCH)
    return snprintf(msg, n, "patch %d outside 3..%d", p->patch, BDIS_MAX_PATCH), BDIS_E_ARG;
  if (p->stride < 1 || p->stride > p->patch)
    return snprintf(msg, n, "stride %d outside 1..patch", p->stride), BDIS_E_ARG;
  if (p->iters < 1 || p->iters > 256) return snprintf(msg, n, "iters %d outside 1..256", p->iters), BDIS_E_ARG;
  if (p->float_pyramid != 0 && p->float_pyramid != 1) return snprintf(msg, n, "float_pyramid must be 0 or 1"), BDIS_E_ARG;
  if (p->fusion < 0 || p->fusion > 2) return snprintf(msg, n, "fusion %d outside 0..2", p->fusion), BDIS_E_ARG;
  if (p->propagate != 0 && p->propagate != 1) return snprintf(msg, n, "propagate must be 0 or 1"), BDIS_E_ARG;
  if (!finite_f(p->sigma_s) || !(p->sigma_s > 0.0f)) return snprintf(msg, n, "sigma_s must be > 0"), BDIS_E_ARG;
  if (!finite_f(p->sigma_r) || !(p->sigma_r > 0.0f)) return snprintf(msg, n, "sigma_r must be > 0"), BDIS_E_ARG;
  if (!finite_f(p->valid_ratio) || !(p->valid_ratio > 0.0f) || p->valid_ratio > 1.0f)
    return snprintf(msg, n, "valid_ratio %g outside (0, 1]", (double)p->valid_ratio), BDIS_E_ARG;
  if (!finite_f(p->var_fail_sigma) || !finite_f(p->var_fit_thresh) || !finite_f(p->prob_thresh))
    return snprintf(msg, n, "variance/threshold parameters not finite"), BDIS_E_ARG;
  float wsum = 0.0f;
  for (int k = p->finest_level; k < p->levels; ++k) {
    if (!finite_f(p->level_weight[k]) || p->level_weight[k] < 0.0f)
      return snprintf(msg, n, "level_weight[%d] must be finite and >= 0", k), BDIS_E_ARG;
    wsum += p->level_weight[k];
  }
  if (!(wsum > 0.0f)) return snprintf(msg, n, "level weights sum to 0"), BDIS_E_ARG;
  return BDIS_OK;
}

bdis_status hip_fail(bdis_ctx* c, hipError_t e, const char* what) {
  return fail(c, BDIS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- timing ---------------------------------------------------------------

hipEvent_t next_event(bdis_ctx* c) {
  if (c->tm.used == c->tm.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->tm.pool.push_back(e);
  }
  return c->tm.pool[c->tm.used++];
}

// Hands a pair of events to the launches that follow (recorded by their
// dispatches); timing_stop takes them back and drops the mark when nothing was
// launched (a phase a level skips).
long timing_start(bdis_ctx* c, int kernel, hipStream_t, int level = -1) {
  if (!c->tm.on) return -1;
  const size_t idx = c->tm.used;
  hipEvent_t a = next_event(c);
  hipEvent_t b = next_event(c);
  if (!a || !b) return -1;
  c->tm.marks.push_back(TimingMark{kernel, level, idx});
  LaunchEvents& ev = launch_events();
  ev.start = a;
  ev.stop = b;
  ev.used = false;
  return (long)idx;
}

void timing_stop(bdis_ctx* c, long mark, hipStream_t) {
  if (mark < 0) return;
  LaunchEvents& ev = launch_events();
  const bool used = ev.used;
  ev = LaunchEvents{};
  if (!used) {
    c->tm.marks.pop_back();
    c->tm.used -= 2;
  }
}

// ---- planning ---------------------------------------------------------------

LevelParams level_params(const bdis_params& p, int n) {
  LevelParams lp{};
  lp.level = n;
  lp.finest = p.finest_level;
  lp.P = p.patch;
  lp.S = p.stride;
  lp.K = p.iters;
  lp.valid_ratio = p.valid_ratio;
  lp.sigma_r_dynamic = p.sigma_r_dynamic;
  lp.sigma_r = p.sigma_r;
  for (int k = 0; k < kMaxLevels; ++k) lp.omega[k] = p.level_weight[k];
  lp.variance = p.variance;
  lp.var_fit_thresh = p.var_fit_thresh;
  lp.var_fail_sigma = p.var_fail_sigma;
  lp.sigma_s = p.sigma_s;
  lp.prob_thresh = p.prob_thresh;
  lp.fusion = p.fusion;
  lp.propagate = p.propagate;
  const double sg = (double)p.sigma_s;
  for (int a = 0; a < kMaxPatch; ++a) {
    double acc = 0.0, dacc = 0.0;
    for (int c = 0; c < p.patch && a < p.patch; ++c) {
      const double d2 = (double)((a - c) * (a - c));
      const double e = std::exp(-d2 / (2.0 * sg * sg));
      acc += e;
      dacc += e * d2 / (sg * sg * sg);
    }
    lp.mask[a] = acc;
    lp.dmask[a] = dacc;
  }
  return lp;
}

// Level parameters of a launch of level n under plan pl.
// Search launches of at most this many workgroups stage the whole right
// window (latency-bound levels: patches that wander past the start range still
// read LDS); larger ones stage only the start range and its margins (the extra
// columns would cost more traffic than they save).
constexpr int kWideWindowBlocks = 4096;

LevelParams plan_level_params(const bdis_params& p, const Plan& pl, int n) {
  LevelParams lp = level_params(p, n);
  lp.inline_prob = pl.inline_prob[n];
  lp.fuse_ty = pl.fuse_ty[n];
  // largest covering-patch block of a tile (bound of cover_range's counts)
  const int nj = (lp.fuse_ty + p.patch - 1) / p.stride + 2, ni = (kFuseTx + p.patch - 1) / p.stride + 2;
  lp.fuse_rec = std::min(ni * nj, kFuseMaxRec);
  lp.fuse_sep = std::min(nj, fuse_sep_rows(lp.fuse_ty));
  lp.keep = pl.keep ? 1 : 0;
  lp.f64_sums = pl.f32 ? 1 : 0;
  lp.wide_win = pl.search_blocks[n] <= kWideWindowBlocks ? 1 : 0;
  return lp;
}

// Tuning key of a level: the device architecture, the library version and the
// level's workload shape across the batch (patch, stride, iterations, pairs, patches, pixels,
// widest level image, and what changes the fusion's work).
std::string level_key(const bdis_ctx* c, const Plan& pl, int n) {
  const bdis_params& p = c->p;
  long np = 0, npx = 0;
  int maxw = 0;
  for (int e = 0; e < pl.tab_count[n]; ++e) {
    const PairLevel& q = pl.tab[pl.tab_first[n] + e];
    np += (long)q.g.nx * q.g.ny;
    npx += (long)q.g.w * q.g.h;
    maxw = std::max(maxw, q.g.w);
  }
  // the library version is part of the key: a build whose kernels changed
  // times its choices again instead of reusing another build's
  char buf[320];
  snprintf(buf, sizeof buf, "%s %s P%d S%d K%d n%d f%d pairs%d patches%ld pixels%ld w%d fusion%d var%d",
           c->arch.c_str(), bdis_version(), p.patch, p.stride, p.iters, n, p.finest_level, pl.tab_count[n], np,
           npx, maxw, p.fusion, p.variance);
  return buf;
}

// Default search configuration (untuned): one patch row per lane, the largest
// workgroup that still gives every compute unit (256 on MI355X) two
// workgroups; else the smallest workgroup.
int default_search_opt(const Plan& pl, int n, int P, int S) {
  for (int o = 2; o >= 0; --o) {  // kind 0 at 256, 128, 64 threads
    if (search_lds_bytes(P, o, S) > kSearchMaxLds) continue;
    long blocks = 0;
    for (int e = 0; e < pl.tab_count[n]; ++e) {
      const PairLevel& q = pl.tab[pl.tab_first[n] + e];
      blocks += (long)search_nbx(q.g, search_npb(P, o, false)) * q.g.ny;
    }
    if (blocks >= 512) return o;
  }
  return 0;
}

// Assigns workgroup offsets for the given per-level search workgroup sizes.
void assign_offsets(const bdis_params& p, Plan& pl) {
  int up = 0;
  for (int e = 0; p.finest_level > 0 && e < pl.tab_count[0]; ++e) {
    PairLevel& q = pl.tab[pl.tab_first[0] + e];
    q.up0 = up;
    up += (q.g.w * q.g.h + kPixThreads - 1) / kPixThreads;
  }
  pl.up_blocks = up;
  for (int n = 0; n < pl.max_levels; ++n) {
    int pyr = 0, se = 0, pr = 0, fu = 0;
    const bool patches = n >= p.finest_level;
    const int opt = pl.search_opt[n];
    for (int e = 0; e < pl.tab_count[n]; ++e) {
      PairLevel& q = pl.tab[pl.tab_first[n] + e];
      q.pyr0 = pyr;
      if (pl.f32)  // one lane per pixel, every level (conversion at level 0; adjoint launches)
        pyr += (q.g.w * q.g.h + kPixThreads - 1) / kPixThreads;
      else
        pyr += n >= 1 ? (pl.pyr_tall[n] ? ((q.g.w + kPyrTallTx - 1) / kPyrTallTx) * ((q.g.h + kPyrTallTy - 1) / kPyrTallTy)
                                         : ((q.g.w + kPyrSmallTx - 1) / kPyrSmallTx) * ((q.g.h + kPyrSmallTy - 1) / kPyrSmallTy))
                      : 0;
      q.search_nbx = patches ? search_nbx(q.g, search_npb(p.patch, opt, pl.f32 || pl.flow)) : 0;
      q.search0 = se;
      se += patches ? q.search_nbx * q.g.ny : 0;
      q.prob0 = pr;
      pr += patches ? (q.g.nx * q.g.ny + kProbThreads - 1) / kProbThreads : 0;
      q.fuse0 = fu;
      fu += patches ? ((q.g.w + kFuseTx - 1) / kFuseTx) * ((q.g.h + pl.fuse_ty[n] - 1) / pl.fuse_ty[n]) : 0;
    }
    pl.pyr_blocks[n] = pyr;
    pl.search_blocks[n] = se;
    pl.prob_blocks[n] = pr;
    pl.fuse_blocks[n] = fu;
  }
  // the pyramid chain's workgroups: tiles of its top level (through that level's pyr0)
  pl.chain_blocks = 0;
  if (pl.chain.m > 0) {
    const int top = pl.chain.n0 + pl.chain.m, tile = pl.chain.tile;
    for (int e = 0; e < pl.tab_count[top]; ++e) {
      PairLevel& q = pl.tab[pl.tab_first[top] + e];
      q.pyr0 = pl.chain_blocks;
      pl.chain_blocks += ((q.g.w + tile - 1) / tile) * ((q.g.h + tile - 1) / tile);
    }
  }
}

// The pyramid chain of a plan: the longest run of small (gather-form) levels
// below the coarsest level the pyramid launches build (the k_top level builds
// its own), present for every pair of the run, above level 1 (built from the
// caller's images by its own launch), of two to four levels.
void plan_chain(Plan& pl) {
  pl.chain = PyrChain{};
  const int last = pl.top_level >= 0 ? pl.top_level - 1 : pl.max_levels - 1;
  if (last < 3) return;
  int first = last;
  while (first - 1 >= 2 && !pl.pyr_tall[first - 1] && pl.tab_count[first - 1] == pl.tab_count[last]) --first;
  if (pl.pyr_tall[last] || pl.tab_count[last] == 0) return;
  for (int k = first; k <= last; ++k)
    if (pl.pyr_tall[k] || pl.tab_count[k] != pl.tab_count[last]) return;
  const int m = std::min(last - first + 1, 4);
  if (m < 2) return;
  const int n0 = last - m;
  const int tile = 16 >> m;  // small tiles: many workgroups, each a short chain
  PyrChain ca = pyr_chain_shape(n0, m, tile);
  if (ca.lds <= 0 || ca.lds > 64 * 1024) return;
  for (int k = 0; k < kMaxLevels; ++k) ca.first[k] = pl.tab_first[k];
  pl.chain = ca;
}

bdis_status build_plan(bdis_ctx* c, const PairSpec* pairs, size_t npairs, Plan* out, bool f32 = false,
                       bool flow = false) {
  const bdis_params& p = c->p;
  Plan& pl = *out;
  pl = Plan();
  pl.finest = p.finest_level;
  pl.f32 = f32;
  pl.flow = flow;
  pl.keep = c->keep || f32;  // the backward pass reads the records
  // a single pair's layout lives on the stack (no heap use)
  Layout lay_one;
  std::vector<Layout> lay_many;
  if (npairs > 1) lay_many.resize(npairs);
  Layout* lays = npairs > 1 ? lay_many.data() : &lay_one;
  for (size_t i = 0; i < npairs; ++i) {
    const PairSpec& q = pairs[i];
    if (!make_layout(p, q.w, q.h, q.levels, &lays[i], c->train))
      return fail(c, BDIS_E_SIZE, "pair %zu: a level of %dx%d with %d levels is smaller than patch %d", i, q.w,
                  q.h, q.levels, p.patch);
    if (lays[i].total > c->slot_bytes)
      return fail(c, BDIS_E_CAPACITY, "pair %zu (%dx%d, %d levels) needs %zu workspace bytes > %zu", i, q.w, q.h,
                  q.levels, lays[i].total, c->slot_bytes);
    pl.max_levels = std::max(pl.max_levels, q.levels);
  }
  for (int n = 0; n < pl.max_levels; ++n) {
    pl.tab_first[n] = (int)pl.tab.size();
    for (size_t i = 0; i < npairs; ++i) {
      const PairSpec& q = pairs[i];
      if (q.levels <= n) continue;
      const Layout& lay = lays[i];
      char* base = c->ws + i * c->slot_bytes;
      auto B8 = [&](size_t o) { return reinterpret_cast<uint8_t*>(base + o); };
      auto BD = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
      PairLevel e;
      std::memset(&e, 0, sizeof e);
      e.g = lay.g[n];
      e.levels = q.levels;
      if (n >= 1) {
        e.srcL = n == 1 ? q.left : B8(lay.lvl_l[n - 1]);
        e.srcR = n == 1 ? q.right : B8(lay.lvl_r[n - 1]);
        e.spitch = n == 1 ? q.pitch : lay.lpitch[n - 1];
        e.sw = lay.g[n - 1].w;
        e.sh = lay.g[n - 1].h;
        e.dstL = B8(lay.lvl_l[n]);
        e.dstR = B8(lay.lvl_r[n]);
      }
      e.L = n == 0 ? q.left : B8(lay.lvl_l[n]);
      e.R = n == 0 ? q.right : B8(lay.lvl_r[n]);
      e.pitch = n == 0 ? q.pitch : lay.lpitch[n];
      if (n == 0 && p.finest_level > 0) {
        e.fdisp = reinterpret_cast<const float*>(base + lay.odisp);
        e.fvar = reinterpret_cast<const float*>(base + lay.ovar);
        e.fconf = reinterpret_cast<const float*>(base + lay.oconf);
        e.fw = lay.g[p.finest_level].w;
        e.fh = lay.g[p.finest_level].h;
        e.fshift = p.finest_level;
        e.disparity = q.disp;
        e.variance = q.var;
        e.confidence = q.conf;
      }
      if (n >= p.finest_level) {
        const bool has_par = n + 1 < q.levels;
        e.par_ubar = has_par ? BD(lay.ubar[n + 1]) : nullptr;
        e.par_q = has_par ? BD(lay.qmap[n + 1]) : nullptr;
        e.pw = has_par ? lay.g[n + 1].w : 0;
        e.ph = has_par ? lay.g[n + 1].h : 0;
        e.pa.uinit = BD(lay.uinit[n]);
        e.pa.pipar = BD(lay.pipar[n]);
        e.pa.u = BD(lay.u[n]);
        e.pa.ssd0 = BD(lay.ssd0[n]);
        e.pa.dssd = reinterpret_cast<D4*>(base + lay.dssd[n]);
        e.pa.rho = reinterpret_cast<float*>(base + lay.rho[n]);
        e.pa.acc = reinterpret_cast<int*>(base + lay.acc[n]);
        e.pa.hess = reinterpret_cast<float*>(base + lay.hess[n]);
        e.pa.dens = reinterpret_cast<D4*>(base + lay.dens[n]);
        e.part_sum = BD(lay.part_sum[n]);
        e.part_cnt = reinterpret_cast<int*>(base + lay.part_cnt[n]);
        e.scal = BD(lay.scal[n]);
        if (n > p.finest_level) {
          e.ubar = BD(lay.ubar[n]);
          e.qmap = BD(lay.qmap[n]);
        } else if (n > 0) {  // level-f maps, upsampled afterwards
          e.disparity = reinterpret_cast<float*>(base + lay.odisp);
          e.variance = reinterpret_cast<float*>(base + lay.ovar);
          e.confidence = reinterpret_cast<float*>(base + lay.oconf);
        } else {
          e.disparity = q.disp;
          e.variance = q.var;
          e.confidence = q.conf;
          e.flow_u = q.flow_u;
          e.flow_v = q.flow_v;
        }
      }
      if (f32) {
        const int f = p.finest_level;
        if (n == 0) {
          e.src32L = q.left32;
          e.src32R = q.right32;
          e.src32pitch = q.pitch;
        } else {
          e.srcdL = BD(lay.ld[n - 1]);
          e.srcdR = BD(lay.rd[n - 1]);
          e.srcdpitch = lay.dpitch[n - 1];
        }
        if (n + 1 < q.levels) {
          e.upLbar = BD(lay.lbar[n + 1]);
          e.upRbar = BD(lay.rbar[n + 1]);
          e.upw = lay.g[n + 1].w;
          e.uph = lay.g[n + 1].h;
          e.updpitch = lay.dpitch[n + 1];
        }
        e.Ld = BD(lay.ld[n]);
        e.Rd = BD(lay.rd[n]);
        e.dpitch = lay.dpitch[n];
        e.Lbar = BD(lay.lbar[n]);
        e.Rbar = BD(lay.rbar[n]);
        e.Gbar = BD(lay.gbar[n]);
        if (n >= f) {
          const bool has_par = n + 1 < q.levels;
          e.uhist = BD(lay.uhist[n]);
          e.reset = reinterpret_cast<int*>(base + lay.reset[n]);
          e.zmap = BD(lay.zmap[n]);
          e.smmap = BD(lay.smmap[n]);
          e.ubar_adj = n > f ? BD(lay.ubar_adj[n]) : nullptr;
          e.qmap_adj = n > f ? BD(lay.qmap_adj[n]) : nullptr;
          e.par_ubar_adj = has_par ? BD(lay.ubar_adj[n + 1]) : nullptr;
          e.par_qmap_adj = has_par ? BD(lay.qmap_adj[n + 1]) : nullptr;
          e.pu_adj = BD(lay.pu_adj[n]);
          e.ppi_adj = BD(lay.ppi_adj[n]);
          e.psig_adj = BD(lay.psig_adj[n]);
          e.pssd_adj = BD(lay.pssd_adj[n]);
          if (n == f) {
            e.vmap = BD(lay.vmap);
            e.ubar_keep = BD(lay.ubar_keep);
            e.qmap_keep = BD(lay.qmap_keep);
            e.grad_disp = q.grad_disp;
            e.grad_var = q.grad_var;
          }
        }
        if (n == 0) {
          e.grad_left = q.grad_left;
          e.grad_right = q.grad_right;
        }
        e.hyper_adj = c->hyper_dev;
      }
      pl.tab.push_back(e);
    }
    pl.tab_count[n] = (int)pl.tab.size() - pl.tab_first[n];
  }
  for (int n = 0; n < pl.max_levels; ++n) {
    if (f32 || flow || n < p.finest_level || pl.tab_count[n] == 0) {
      pl.search_opt[n] = 0;
      continue;
    }
    pl.search_opt[n] = default_search_opt(pl, n, p.patch, p.stride);
  }
  for (int n = 0; n < pl.max_levels; ++n) {
    long np = 0, npx = 0;
    for (int e = 0; e < pl.tab_count[n]; ++e) {
      const LevelGeom& g = pl.tab[pl.tab_first[n] + e].g;
      np += (long)g.nx * g.ny;
      npx += (long)g.w * g.h;
    }
    pl.inline_prob[n] = np <= kInlineProbPatches ? 1 : 0;
    const bool huge = npx >= kFuseHugePixels && fuse_tile_fits(kFuseTyHuge, p.patch, p.stride);
    pl.fuse_ty[n] = flow                      ? kFuseTyShort
                    : huge                    ? kFuseTyHuge
                    : npx >= kFuseTallPixels ? kFuseTyTall
                                              : kFuseTyShort;
    pl.pyr_tall[n] = npx >= kPyrTallPixels;
  }
  // tuned choices of this batch shape (uint8 stereo path; the key is a string,
  // so it is built only when something was tuned or loaded)
  bool top_tuned_off = false, top_tuned_on = false, chain_tuned_off = false;
  if (!f32 && !flow && !c->tuned.empty()) {
    for (int n = 0; n < pl.max_levels; ++n) {
      if (pl.tab_count[n] == 0) continue;
      auto it = c->tuned.find(level_key(c, pl, n));
      if (it == c->tuned.end()) continue;
      const TuneChoice& tc = it->second;
      if (n >= p.finest_level && tc.search >= 0 && tc.search < kNumSearchOptions &&
          search_lds_bytes(p.patch, tc.search, p.stride) <= kSearchMaxLds)
        pl.search_opt[n] = tc.search;
      if (n >= p.finest_level && fuse_ty_ok(tc.fuse_ty) &&
          (tc.fuse_ty != kFuseTyHuge || fuse_tile_fits(kFuseTyHuge, p.patch, p.stride)))
        pl.fuse_ty[n] = tc.fuse_ty;
      if (n >= 1 && (tc.pyr_tall == 0 || tc.pyr_tall == 1)) pl.pyr_tall[n] = tc.pyr_tall == 1;
      if (tc.top == 0) top_tuned_off = true;
      if (tc.top == 1) top_tuned_on = true;
      if (tc.chain == 0) chain_tuned_off = true;
    }
  }
  if (!f32 && !flow && c->forced_opt >= 0)
    for (int n = p.finest_level; n < pl.max_levels; ++n) pl.search_opt[n] = c->forced_opt;
  // the coarsest level of the deepest pairs (every entry there is a pair's
  // coarsest level) in one workgroup per pair, when it is above the finest
  // level, uses the mask weights and fits
  const int top = pl.max_levels - 1;
  if (!f32 && !flow && c->top_mode != 0 && top >= 1 && top > p.finest_level && p.fusion != 1 && pl.tab_count[top] > 0) {
    int mw = 0, mh = 0, msw = 0, msh = 0, mnp = 0;
    for (int e = 0; e < pl.tab_count[top]; ++e) {
      const PairLevel& q = pl.tab[pl.tab_first[top] + e];
      mw = std::max(mw, q.g.w);
      mh = std::max(mh, q.g.h);
      msw = std::max(msw, q.sw);
      msh = std::max(msh, q.sh);
      mnp = std::max(mnp, q.g.nx * q.g.ny);
    }
    pl.top = top_shape(p.patch, p.stride, mw, mh, msw, msh, mnp);
    if (pl.top.g > 0) {
      pl.top_fits = top;
      // forced, tuned, or (untuned) for batches of many pairs, where one
      // workgroup per pair at once beats the level's launches
      const bool use = c->top_mode == 1 || top_tuned_on || (!top_tuned_off && pl.tab_count[top] >= kTopMinPairs);
      if (use) pl.top_level = top;
    }
  }
  if (!f32 && !flow && c->chain_mode != 0 && (c->chain_mode == 1 || !chain_tuned_off)) plan_chain(pl);
  assign_offsets(p, pl);
  return BDIS_OK;
}

// Uploads the job table when it differs from the one on the device.
bdis_status upload_table(bdis_ctx* c, const Plan& pl, hipStream_t st) {
  const size_t n = pl.tab.size();
  if (n == c->tab_last.size() && std::memcmp(pl.tab.data(), c->tab_last.data(), n * sizeof(PairLevel)) == 0)
    return BDIS_OK;
  hipError_t e;
  if (n > c->tab_cap) {
    // the old table may still be read by queued work: drain before freeing it
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "table resize");
    if (c->tab_dev) (void)hipFree(c->tab_dev);
    if (c->tab_host) (void)hipHostFree(c->tab_host);
    c->tab_dev = nullptr;
    c->tab_host = nullptr;
    c->tab_cap = 0;
    c->tab_last.clear();
    c->tab_evt_live = false;
    for (auto& kv : c->graphs) {  // graphs hold the old table address
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    c->graphs.clear();
    if ((e = hipMalloc(reinterpret_cast<void**>(&c->tab_dev), n * sizeof(PairLevel))) != hipSuccess)
      return fail(c, BDIS_E_NOMEM, "job table: %s", hipGetErrorString(e));
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&c->tab_host), n * sizeof(PairLevel))) != hipSuccess)
      return fail(c, BDIS_E_NOMEM, "job table staging: %s", hipGetErrorString(e));
    c->tab_cap = n;
  }
  // the staging buffer may still feed the previous (async) upload
  if (c->tab_evt_live && (e = hipEventSynchronize(c->tab_evt)) != hipSuccess) return hip_fail(c, e, "table event");
  std::memcpy(c->tab_host, pl.tab.data(), n * sizeof(PairLevel));
  if ((e = hipMemcpyAsync(c->tab_dev, c->tab_host, n * sizeof(PairLevel), hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(c, e, "job table upload");
  if ((e = hipEventRecord(c->tab_evt, st)) != hipSuccess) return hip_fail(c, e, "table event");
  c->tab_evt_live = true;
  c->tab_last.assign(pl.tab.data(), pl.tab.data() + n);
  return BDIS_OK;
}

// The pyramid launch of level n under plan pl.
hipError_t launch_pyramid_level(const PairLevel* tab_dev, const Plan& pl, int n, hipStream_t st) {
  return launch_pyramid(tab_dev + pl.tab_first[n], pl.tab_count[n], pl.pyr_blocks[n], pl.pyr_tall[n], st);
}

// The launch sequence of a plan (eager; optionally timed per kernel).
bdis_status launch_all(bdis_ctx* c, const Plan& pl, hipStream_t st) {
  const bdis_params& p = c->p;
  hipError_t e;
  for (int n = 1; n < pl.max_levels; ++n) {
    if (n == pl.top_level) continue;  // built inside k_top
    const bool chained = pl.chain.m > 0 && n > pl.chain.n0 && n <= pl.chain.n0 + pl.chain.m;
    if (chained && n > pl.chain.n0 + 1) continue;  // built by the chain launch
    const long tmk = timing_start(c, BDIS_K_PYRAMID, st, n);
    e = chained ? launch_pyr_chain(c->tab_dev, pl.tab_count[n], pl.chain_blocks, pl.chain, st)
                : launch_pyramid_level(c->tab_dev, pl, n, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "pyramid launch");
  }
  for (int n = pl.max_levels - 1; n >= p.finest_level; --n) {
    const PairLevel* tab = c->tab_dev + pl.tab_first[n];
    const int cnt = pl.tab_count[n];
    const LevelParams lp = plan_level_params(p, pl, n);
    if (n == pl.top_level) {  // pyramid step, search, scalars, records and fusion in one launch
      const long tmk = timing_start(c, BDIS_K_TOP, st, n);
      e = launch_top(tab, cnt, lp, pl.top, st);
      timing_stop(c, tmk, st);
      if (e != hipSuccess) return hip_fail(c, e, "top-level launch");
      continue;
    }
    long tmk = timing_start(c, BDIS_K_SEARCH, st, n);
    e = launch_search(tab, cnt, pl.search_blocks[n], lp, pl.search_opt[n], st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "search launch");
    tmk = timing_start(c, BDIS_K_REDUCE, st, n);
    e = launch_reduce(tab, cnt, lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "reduction launch");
    tmk = timing_start(c, BDIS_K_PROB, st, n);
    e = launch_prob(tab, cnt, pl.prob_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "probability launch");
    tmk = timing_start(c, BDIS_K_FUSE, st, n);
    e = launch_fuse(tab, cnt, pl.fuse_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "fusion launch");
  }
  if (p.finest_level > 0) {
    const long tmk = timing_start(c, BDIS_K_FUSE, st);
    e = launch_upsample(c->tab_dev + pl.tab_first[0], pl.tab_count[0], pl.up_blocks, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "upsampling launch");
  }
  return BDIS_OK;
}

// Graph key: everything that shapes the launch sequence (not the pointers).
std::string graph_key(const bdis_params& p, const Plan& pl) {
  std::string k(reinterpret_cast<const char*>(&p), sizeof p);
  auto add = [&](const void* ptr, size_t n) { k.append(reinterpret_cast<const char*>(ptr), n); };
  add(pl.tab_first, sizeof pl.tab_first);
  add(pl.tab_count, sizeof pl.tab_count);
  add(pl.pyr_blocks, sizeof pl.pyr_blocks);
  add(pl.search_blocks, sizeof pl.search_blocks);
  add(pl.prob_blocks, sizeof pl.prob_blocks);
  add(pl.fuse_blocks, sizeof pl.fuse_blocks);
  add(pl.search_opt, sizeof pl.search_opt);
  add(&pl.up_blocks, sizeof pl.up_blocks);
  add(pl.inline_prob, sizeof pl.inline_prob);
  add(pl.fuse_ty, sizeof pl.fuse_ty);
  add(pl.pyr_tall, sizeof pl.pyr_tall);
  add(&pl.max_levels, sizeof pl.max_levels);
  add(&pl.top_level, sizeof pl.top_level);
  add(&pl.top, sizeof pl.top);
  add(&pl.chain, sizeof pl.chain);
  add(&pl.chain_blocks, sizeof pl.chain_blocks);
  return k;
}

bdis_status run_graph(bdis_ctx* c, const Plan& pl, hipStream_t st) {
  const std::string key = graph_key(c->p, pl);
  auto it = c->graphs.find(key);
  hipError_t e;
  if (it == c->graphs.end()) {
    const double t0 = wall_ms();
    if (c->graphs.size() >= kMaxGraphs) {
      // the least recently launched graph goes; the device is synchronised
      // first, so that no launch of it is still in flight when it is destroyed
      auto lru = c->graphs.begin();
      for (auto g = c->graphs.begin(); g != c->graphs.end(); ++g)
        if (g->second.used < lru->second.used) lru = g;
      if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "graph eviction");
      if (lru->second.exec) (void)hipGraphExecDestroy(lru->second.exec);
      if (lru->second.graph) (void)hipGraphDestroy(lru->second.graph);
      c->graphs.erase(lru);
    }
    GraphEntry ge;
    if ((e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(c, e, "graph capture begin");
    bdis_status s2 = launch_all(c, pl, c->capture_stream);
    e = hipStreamEndCapture(c->capture_stream, &ge.graph);
    if (s2 != BDIS_OK) {
      if (ge.graph) (void)hipGraphDestroy(ge.graph);
      return s2;
    }
    if (e != hipSuccess) return hip_fail(c, e, "graph capture end");
    if ((e = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(ge.graph);
      return hip_fail(c, e, "graph instantiate");
    }
    it = c->graphs.emplace(key, ge).first;
    c->last_capture_ms = wall_ms() - t0;
  }
  if ((e = hipGraphLaunch(it->second.exec, st)) != hipSuccess) return hip_fail(c, e, "graph launch");
  it->second.used = ++c->graph_launches;
  return BDIS_OK;
}

// ---- tuning cache file --------------------------------------------------------
// One JSON object; each tuned level shape is one line
//   "<key>": {"search": S, "fuse_ty": T, "pyr_tall": Y},
// where the key starts with the device architecture.  Read at bdis_create
// (entries of the context's architecture), rewritten after each tuning with
// the entries of every architecture (written to a temporary file, then
// renamed).  A missing or unreadable file only means tuning again.

// Entries of the cache file (every architecture).
std::map<std::string, TuneChoice> read_tune_cache(const std::string& path) {
  std::map<std::string, TuneChoice> out;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return out;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char* q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char* q1 = std::strchr(q0 + 1, '"');
    if (!q1) continue;
    TuneChoice tc;
    if (std::sscanf(q1 + 1, " : {\"search\": %d, \"fuse_ty\": %d, \"pyr_tall\": %d, \"top\": %d, \"chain\": %d}",
                    &tc.search, &tc.fuse_ty, &tc.pyr_tall, &tc.top, &tc.chain) == 5)
      out[std::string(q0 + 1, q1)] = tc;
  }
  std::fclose(f);
  return out;
}

bdis_status save_tune_cache(bdis_ctx* c) {
  if (c->tune_cache.empty()) return BDIS_OK;
  std::map<std::string, TuneChoice> all = read_tune_cache(c->tune_cache);
  for (const auto& kv : c->tuned) all[kv.first] = kv.second;
  // the directory of the file (one level created if missing)
  const size_t slash = c->tune_cache.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    const std::string dir = c->tune_cache.substr(0, slash);
    const size_t up = dir.rfind('/');
    if (up != std::string::npos && up > 0) (void)mkdir(dir.substr(0, up).c_str(), 0755);
    (void)mkdir(dir.c_str(), 0755);
  }
  char tmp_suffix[64];
  std::snprintf(tmp_suffix, sizeof tmp_suffix, ".tmp%ld", (long)getpid());
  const std::string tmp = c->tune_cache + tmp_suffix;
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return BDIS_OK;  // the cache is an optimisation: an unwritable file is not an error
  std::fprintf(f, "{\n\"bdis_tune_cache\": 1,\n\"entries\": {\n");
  size_t k = 0;
  for (const auto& kv : all)
    std::fprintf(f, "\"%s\": {\"search\": %d, \"fuse_ty\": %d, \"pyr_tall\": %d, \"top\": %d, \"chain\": %d}%s\n",
                 kv.first.c_str(), kv.second.search, kv.second.fuse_ty, kv.second.pyr_tall, kv.second.top,
                 kv.second.chain, ++k < all.size() ? "," : "");
  std::fprintf(f, "}\n}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), c->tune_cache.c_str()) != 0) (void)std::remove(tmp.c_str());
  return BDIS_OK;
}

// The cache file: BDIS_TUNE_CACHE if set ("" disables it), else
// $HOME/.cache/bdis/tune.json.
std::string tune_cache_path() {
  if (const char* e = std::getenv("BDIS_TUNE_CACHE")) return e;
  const char* home = std::getenv("HOME");
  if (!home || !*home) return "";
  return std::string(home) + "/.cache/bdis/tune.json";
}

// Picks the launch shapes of every level of a new batch shape by timing the
// options over full passes (every phase rewrites its outputs, so trial passes
// leave nothing behind; every option gives identical results):
//   1. the search configuration (lane mapping and workgroup size),
//   2. the fusion tile height (64 x 4, 64 x 16, 64 x 32 where its covering
//      patches fit the staged form), with the searches at their best,
//   3. the pyramid form (gather 64 x 4 or staged 120 x 12 tiles).
// Each timed launch records its events from its own dispatch.  Timed passes
// per option: the first one only warms caches and code, the best of the
// others counts.  The choices are kept per level shape and written to the
// tuning cache file.
constexpr int kTuneReps = 5;
constexpr int kTuneGraphReps = 10;  // replays per captured combination of the structural choices

bdis_status save_tune_cache(bdis_ctx* c);

bdis_status tune(bdis_ctx* c, Plan& pl, hipStream_t st) {
  const bdis_params& p = c->p;
  bool need = false;
  for (int n = 0; n < pl.max_levels; ++n)
    if (pl.tab_count[n] && !c->tuned.count(level_key(c, pl, n))) need = true;
  if (!need) return BDIS_OK;
  const char* env = std::getenv("BDIS_TUNE");
  const bool enabled = !(env && std::strcmp(env, "0") == 0) && c->forced_opt < 0;
  const double t0 = wall_ms();
  TuneChoice best[kMaxLevels];
  for (int n = 0; n < pl.max_levels; ++n) {
    best[n].search = pl.search_opt[n];
    best[n].fuse_ty = pl.fuse_ty[n];
    best[n].pyr_tall = pl.pyr_tall[n] ? 1 : 0;
    best[n].top = n == pl.top_fits ? (pl.top_level == n ? 1 : 0) : -1;
  }
  const int top_cand = pl.top_fits;   // the level k_top could take (-1: none)
  int chain_hi = -1;                  // top level of the pyramid chain, where its choice is kept
  if (enabled) {
    std::vector<hipEvent_t> ev(2 * kMaxLevels, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
      if (e == hipSuccess) e = hipEventCreate(&x);
    bdis_status s2 = BDIS_OK;
    // Times `trial` over kTuneReps passes; phase 0 search, 1 fusion, 2 pyramid.
    // best_ms[n] / pick(n) record a level whose timed launch beat its best.
    auto run_trial = [&](Plan& trial, int phase, float* best_ms, auto&& pick) {
      assign_offsets(p, trial);
      if ((s2 = upload_table(c, trial, st)) != BDIS_OK) return;
      bool rec[kMaxLevels] = {};  // levels whose timed phase launched a kernel (recorded its events)
      auto timed = [&](int n, int ph, auto&& launch) {
        if (ph != phase) return launch();
        LaunchEvents& le = launch_events();
        le.start = ev[2 * n];
        le.stop = ev[2 * n + 1];
        le.used = false;
        const hipError_t r = launch();
        rec[n] = le.used;
        le = LaunchEvents{};
        return r;
      };
      for (int rep = 0; rep < kTuneReps && e == hipSuccess; ++rep) {
        for (int n = 1; n < trial.max_levels && e == hipSuccess; ++n) {
          if (n == trial.top_level) continue;
          const bool chained = trial.chain.m > 0 && n > trial.chain.n0 && n <= trial.chain.n0 + trial.chain.m;
          if (chained) {
            if (n == trial.chain.n0 + 1)
              e = launch_pyr_chain(c->tab_dev, trial.tab_count[n], trial.chain_blocks, trial.chain, st);
          } else {
            e = timed(n, 2, [&] { return launch_pyramid_level(c->tab_dev, trial, n, st); });
          }
        }
        for (int n = trial.max_levels - 1; n >= p.finest_level && e == hipSuccess; --n) {
          const PairLevel* tab = c->tab_dev + trial.tab_first[n];
          const int cnt = trial.tab_count[n];
          const LevelParams lp = plan_level_params(p, trial, n);
          if (n == trial.top_level) {
            e = launch_top(tab, cnt, lp, trial.top, st);
          } else {
            e = timed(n, 0, [&] { return launch_search(tab, cnt, trial.search_blocks[n], lp, trial.search_opt[n], st); });
            if (e == hipSuccess) e = launch_reduce(tab, cnt, lp, st);
            if (e == hipSuccess) e = launch_prob(tab, cnt, trial.prob_blocks[n], lp, st);
            if (e == hipSuccess) e = timed(n, 1, [&] { return launch_fuse(tab, cnt, trial.fuse_blocks[n], lp, st); });
          }
        }
        if (p.finest_level > 0 && e == hipSuccess)
          e = launch_upsample(c->tab_dev + trial.tab_first[0], trial.tab_count[0], trial.up_blocks, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || rep == 0) continue;  // the first pass warms caches and code
        const int lo = phase == 2 ? 1 : p.finest_level;
        for (int n = lo; n < trial.max_levels; ++n) {
          if (!trial.tab_count[n] || !rec[n]) continue;  // nothing launched at this level
          float ms = 0.0f;
          if (hipEventElapsedTime(&ms, ev[2 * n], ev[2 * n + 1]) == hipSuccess && ms < best_ms[n]) {
            best_ms[n] = ms;
            pick(n);
          }
        }
      }
    };
    // 1. search configurations
    float bs[kMaxLevels];
    std::fill(bs, bs + kMaxLevels, 1e30f);
    for (int o = 0; o < kNumSearchOptions && e == hipSuccess && s2 == BDIS_OK; ++o) {
      if (search_lds_bytes(p.patch, o, p.stride) > kSearchMaxLds) continue;
      const int kind = search_option_kind(o);
      if (kind > 0 && search_lanes(p.patch, kind) == search_lanes(p.patch, kind - 1)) continue;  // same mapping
      Plan trial = pl;
      trial.top_level = -1;
      trial.chain.m = 0;
      for (int n = 0; n < trial.max_levels; ++n) trial.search_opt[n] = o;
      run_trial(trial, 0, bs, [&](int n) { best[n].search = o; });
    }
    // 2. fusion tile heights (searches at their best)
    float bf[kMaxLevels];
    std::fill(bf, bf + kMaxLevels, 1e30f);
    const int tys[3] = {kFuseTyShort, kFuseTyTall, kFuseTyHuge};
    for (int ty : tys) {
      if (e != hipSuccess || s2 != BDIS_OK) break;
      if (ty == kFuseTyHuge && !fuse_tile_fits(kFuseTyHuge, p.patch, p.stride)) continue;
      Plan trial = pl;
      trial.top_level = -1;
      trial.chain.m = 0;
      for (int n = 0; n < trial.max_levels; ++n) {
        if (n >= p.finest_level) trial.search_opt[n] = best[n].search;
        trial.fuse_ty[n] = ty;
      }
      run_trial(trial, 1, bf, [&](int n) { best[n].fuse_ty = ty; });
    }
    // 3. pyramid forms
    float bp[kMaxLevels];
    std::fill(bp, bp + kMaxLevels, 1e30f);
    for (int tall = 0; tall <= 1 && e == hipSuccess && s2 == BDIS_OK; ++tall) {
      Plan trial = pl;
      trial.top_level = -1;
      trial.chain.m = 0;
      for (int n = 0; n < trial.max_levels; ++n) {
        if (n >= p.finest_level) {
          trial.search_opt[n] = best[n].search;
          trial.fuse_ty[n] = best[n].fuse_ty;
        }
        trial.pyr_tall[n] = tall == 1;
      }
      run_trial(trial, 2, bp, [&](int n) { best[n].pyr_tall = tall; });
    }
    // 4. the structural choices: the coarsest level in one workgroup per pair
    // or in its per-phase launches, and one launch for a run of small pyramid
    // levels or one each.  They change the number of launches, whose cost is
    // the graph's node overhead, so each combination (the rest at its best)
    // is captured as a graph and its replays are timed.
    if ((top_cand >= 0 && c->top_mode < 0) || c->chain_mode < 0) {
      Plan base = pl;
      for (int n = 0; n < base.max_levels; ++n) {
        if (n >= p.finest_level) {
          base.search_opt[n] = best[n].search;
          base.fuse_ty[n] = best[n].fuse_ty;
        }
        if (n >= 1) base.pyr_tall[n] = best[n].pyr_tall == 1;
      }
      const bool was_timing = c->tm.on;
      c->tm.on = false;  // captured launches record no timing events
      float best_ms = 1e30f;
      int best_top = top_cand >= 0 ? 1 : -1, best_chain = -1;
      for (int top = 1; top >= 0 && e == hipSuccess && s2 == BDIS_OK; --top) {
        if (top == 1 && top_cand < 0) continue;
        if (c->top_mode >= 0 && top != c->top_mode && top_cand >= 0) continue;
        for (int ch = 1; ch >= 0 && e == hipSuccess && s2 == BDIS_OK; --ch) {
          Plan trial = base;
          trial.top_level = top ? top_cand : -1;
          trial.chain.m = 0;
          if (ch) {
            if (c->chain_mode == 0) continue;
            plan_chain(trial);
            if (trial.chain.m == 0) continue;
          } else if (c->chain_mode == 1) {
            Plan probe = trial;
            plan_chain(probe);
            if (probe.chain.m > 0) continue;
          }
          assign_offsets(p, trial);
          if ((s2 = upload_table(c, trial, st)) != BDIS_OK) break;
          hipGraph_t g = nullptr;
          hipGraphExec_t ge = nullptr;
          if ((e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) break;
          const bdis_status s3 = launch_all(c, trial, c->capture_stream);
          e = hipStreamEndCapture(c->capture_stream, &g);
          if (s3 != BDIS_OK) {
            if (g) (void)hipGraphDestroy(g);
            s2 = s3;
            break;
          }
          if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
          for (int r = 0; r < 2 && e == hipSuccess; ++r) e = hipGraphLaunch(ge, st);  // warm-up
          if (e == hipSuccess) e = hipEventRecord(ev[0], st);
          for (int r = 0; r < kTuneGraphReps && e == hipSuccess; ++r) e = hipGraphLaunch(ge, st);
          if (e == hipSuccess) e = hipEventRecord(ev[1], st);
          if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
          if (ge) (void)hipGraphExecDestroy(ge);
          if (g) (void)hipGraphDestroy(g);
          if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best_top = top_cand >= 0 ? top : -1;
            best_chain = ch;
            // the level that keeps the chain choice: the top of the chain this
            // top-level choice allows
            Plan probe = trial;
            plan_chain(probe);
            chain_hi = probe.chain.m > 0 ? probe.chain.n0 + probe.chain.m : -1;
          }
        }
      }
      c->tm.on = was_timing;
      if (top_cand >= 0) best[top_cand].top = best_top;
      if (chain_hi >= 0 && best_chain >= 0) best[chain_hi].chain = best_chain;
    }
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    if (s2 != BDIS_OK) return s2;
    if (e != hipSuccess) return hip_fail(c, e, "tuning");
  }
  for (int n = 0; n < pl.max_levels; ++n) {
    if (!pl.tab_count[n]) continue;
    TuneChoice tc = best[n];
    if (n < p.finest_level) tc.search = -1, tc.fuse_ty = 0;
    if (n == 0) tc.pyr_tall = -1;
    c->tuned[level_key(c, pl, n)] = tc;
    if (n >= p.finest_level) {
      pl.search_opt[n] = best[n].search;
      pl.fuse_ty[n] = best[n].fuse_ty;
    }
    if (n >= 1) pl.pyr_tall[n] = best[n].pyr_tall == 1;
    if (n == top_cand) pl.top_level = best[n].top == 1 ? n : -1;
  }
  pl.chain.m = 0;
  if (c->chain_mode == 1 || (c->chain_mode < 0 && !(chain_hi >= 0 && best[chain_hi].chain == 0))) plan_chain(pl);
  assign_offsets(p, pl);
  c->last_tune_ms = wall_ms() - t0;
  if (enabled) return save_tune_cache(c);
  return BDIS_OK;
}

// Every call reuses the context's workspace and job table, so the work of a
// call must not start before the previous call's work ends.  On one stream
// that holds by stream order and costs nothing.  The first time a call comes
// on another stream the device is drained once; from then on every call
// records an event at its end and a call on a different stream waits for it
// (no host wait).
bdis_status order_after_last(bdis_ctx* c, hipStream_t st) {
  if (!c->done_live || c->done_stream == st) return BDIS_OK;
  hipError_t e;
  if (!c->multi_stream) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, "ordering after the previous call");
    c->multi_stream = true;
    return BDIS_OK;
  }
  e = hipStreamWaitEvent(st, c->done_evt, 0);
  return e == hipSuccess ? BDIS_OK : hip_fail(c, e, "ordering after the previous call");
}

bdis_status mark_done(bdis_ctx* c, hipStream_t st, bdis_status s) {
  if (s != BDIS_OK) return s;
  c->done_stream = st;
  c->done_live = true;
  if (!c->multi_stream) return BDIS_OK;
  const hipError_t e = hipEventRecord(c->done_evt, st);
  return e == hipSuccess ? BDIS_OK : hip_fail(c, e, "call completion event");
}

// The workspace lives on the device current at bdis_create: calls must keep it current.
bdis_status check_device(bdis_ctx* c) {
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  if (dev != c->device)
    return fail(c, BDIS_E_STATE, "current device %d is not the context's device %d", dev, c->device);
  return BDIS_OK;
}

template <typename F>
bdis_status ordered(bdis_ctx* c, hipStream_t st, F&& run) {
  bdis_status s = check_device(c);
  if (s != BDIS_OK) return s;
  s = order_after_last(c, st);
  if (s != BDIS_OK) return s;
  return mark_done(c, st, run(st));
}

bdis_status run_pairs(bdis_ctx* c, const std::vector<PairSpec>& pairs, hipStream_t st) {
  c->last_tune_ms = c->last_capture_ms = 0.0;
  Plan pl;
  bdis_status s = build_plan(c, pairs.data(), pairs.size(), &pl);
  if (s != BDIS_OK) return s;
  if ((s = tune(c, pl, st)) != BDIS_OK) return s;
  if ((s = upload_table(c, pl, st)) != BDIS_OK) return s;
  if (c->tm.on || !c->use_graph) return launch_all(c, pl, st);
  return run_graph(c, pl, st);
}

// Float path forward: FP64 pyramid (level 0 converted from float), then the
// usual per-level phases; training state is written as it goes.
bdis_status run_pairs_f32(bdis_ctx* c, const std::vector<PairSpec>& pairs, hipStream_t st) {
  Plan pl;
  bdis_status s = build_plan(c, pairs.data(), pairs.size(), &pl, true);
  if (s != BDIS_OK) return s;
  if ((s = upload_table(c, pl, st)) != BDIS_OK) return s;
  const bdis_params& p = c->p;
  hipError_t e;
  for (int n = 0; n < pl.max_levels; ++n) {
    const long tmk = timing_start(c, BDIS_K_PYRAMID, st, n);
    e = launch_pyramid_f64(c->tab_dev + pl.tab_first[n], pl.tab_count[n], pl.pyr_blocks[n], n, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "pyramid launch");
  }
  for (int n = pl.max_levels - 1; n >= p.finest_level; --n) {
    const PairLevel* tab = c->tab_dev + pl.tab_first[n];
    const int cnt = pl.tab_count[n];
    const LevelParams lp = plan_level_params(p, pl, n);
    long tmk = timing_start(c, BDIS_K_SEARCH, st, n);
    e = launch_search_f64(tab, cnt, pl.search_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "search launch");
    tmk = timing_start(c, BDIS_K_REDUCE, st, n);
    e = launch_reduce(tab, cnt, lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "reduction launch");
    tmk = timing_start(c, BDIS_K_PROB, st, n);
    e = launch_prob(tab, cnt, pl.prob_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "probability launch");
    tmk = timing_start(c, BDIS_K_FUSE, st, n);
    e = launch_fuse(tab, cnt, pl.fuse_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "fusion launch");
  }
  if (p.finest_level > 0) {
    const long tmk = timing_start(c, BDIS_K_FUSE, st);
    e = launch_upsample(c->tab_dev + pl.tab_first[0], pl.tab_count[0], pl.up_blocks, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "upsampling launch");
  }
  return BDIS_OK;
}

// Optical-flow form: the same pyramid, then per level the 2-D search and the
// Eq. 2 fusion (no probability, no reduction).
bdis_status run_flow(bdis_ctx* c, const std::vector<PairSpec>& pairs, hipStream_t st) {
  Plan pl;
  bdis_status s = build_plan(c, pairs.data(), pairs.size(), &pl, false, true);
  if (s != BDIS_OK) return s;
  if ((s = upload_table(c, pl, st)) != BDIS_OK) return s;
  const bdis_params& p = c->p;
  hipError_t e;
  for (int n = 1; n < pl.max_levels; ++n) {
    const long tmk = timing_start(c, BDIS_K_PYRAMID, st, n);
    e = launch_pyramid_level(c->tab_dev, pl, n, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "pyramid launch");
  }
  for (int n = pl.max_levels - 1; n >= 0; --n) {
    const PairLevel* tab = c->tab_dev + pl.tab_first[n];
    const LevelParams lp = plan_level_params(p, pl, n);
    long tmk = timing_start(c, BDIS_K_SEARCH, st, n);
    e = launch_flow_search(tab, pl.tab_count[n], pl.search_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "flow search launch");
    tmk = timing_start(c, BDIS_K_FUSE, st, n);
    e = launch_flow_fuse(tab, pl.tab_count[n], pl.fuse_blocks[n], lp, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "flow fusion launch");
  }
  return BDIS_OK;
}

// Backward pass of the last float-path call: adjoints level by level from the
// finest to the coarsest, then the transposed pyramid down to the images.
bdis_status run_backward(bdis_ctx* c, std::vector<PairSpec> pairs, double* grad_hyper, hipStream_t st) {
  if (c->p.finest_level != 0)
    return fail(c, BDIS_E_ARG, "backward needs finest_level 0 (no adjoint of the upsampling)");
  if (c->p.fusion != 0 || c->p.propagate != 1)
    return fail(c, BDIS_E_ARG, "backward needs fusion 0 and propagate 1 (the method's own weights)");
  Plan pl;
  bdis_status s = build_plan(c, pairs.data(), pairs.size(), &pl, true);
  if (s != BDIS_OK) return s;
  if ((s = upload_table(c, pl, st)) != BDIS_OK) return s;
  const bdis_params& p = c->p;
  hipError_t e;
  // every pair's adjoint buffers and the hyper-gradient sums start from zero
  std::vector<unsigned char*> zp;
  std::vector<size_t> zn;
  for (size_t i = 0; i < pairs.size(); ++i) {
    Layout lay;
    make_layout(p, pairs[i].w, pairs[i].h, pairs[i].levels, &lay, true);
    zp.push_back(reinterpret_cast<unsigned char*>(c->ws + i * c->slot_bytes + lay.adj_begin));
    zn.push_back(lay.adj_end - lay.adj_begin);
  }
  zp.push_back(reinterpret_cast<unsigned char*>(c->hyper_dev));
  zn.push_back(sizeof(double) * (2 + kMaxLevels));
  if ((e = zero_ranges(zp.data(), zn.data(), (int)zp.size(), st)) != hipSuccess)
    return hip_fail(c, e, "adjoint clear");
  const int ntab = (int)pl.tab.size();
  bdis_launch(k_adj_scal_zero, dim3((ntab + 63) / 64), dim3(64), 0, st, c->tab_dev, ntab);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "adjoint clear");
  // with more than one level, level 0's transposed template gradient is taken
  // by its pyramid adjoint launch (one per-pixel pass over level 0 fewer)
  const bool sobel0_in_pyramid = pl.max_levels >= 2;
  for (int n = p.finest_level; n < pl.max_levels; ++n) {
    const int blocks[3] = {pl.pyr_blocks[n], pl.search_blocks[n], pl.prob_blocks[n]};
    const long tmk = timing_start(c, BDIS_K_BACKWARD, st, n);
    e = launch_backward_level(c->tab_dev + pl.tab_first[n], pl.tab_count[n], blocks, level_params(p, n),
                              n == 0 && sobel0_in_pyramid, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "backward launch");
  }
  for (int n = pl.max_levels - 2; n >= 0; --n) {  // level n+1 -> level n
    const long tmk = timing_start(c, BDIS_K_BACKWARD, st, n);
    e = launch_pyramid_adj(c->tab_dev + pl.tab_first[n], pl.tab_count[n], pl.pyr_blocks[n],
                           n == 0 && sobel0_in_pyramid, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "pyramid adjoint launch");
  }
  // the level-0 pyramid adjoint writes the image gradients; with one level, a
  // launch of its own does
  if (pl.max_levels < 2 &&
      (e = launch_grad_out(c->tab_dev + pl.tab_first[0], pl.tab_count[0], pl.pyr_blocks[0], st)) != hipSuccess)
    return hip_fail(c, e, "gradient output launch");
  if (grad_hyper) {
    e = hipMemcpyAsync(grad_hyper, c->hyper_dev, sizeof(double) * (2 + pl.max_levels), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "hyper-gradient copy");
  }
  return BDIS_OK;
}

// ---- allocation-free single-pair path ----------------------------------------
// bdis_compute_static runs the same launch sequence as bdis_compute on a
// workspace that lives in the static device array `scratch` (job table first,
// then the pair's workspace slot): no allocation, no graph, no tuning (the
// default search configuration per level).  The array's host-side name is not
// a device address: its address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = (size_t)48 << 20;
constexpr int kMaxStaticDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxStaticDevices] = {nullptr};

// Address of `scratch` on device `dev` (the current device).
hipError_t static_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kMaxStaticDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Job-table entries written by a kernel from its arguments (captured by value,
// so the call can sit under graph capture), kTabChunk entries per launch.
constexpr int kTabChunk = 4;
struct TabChunk {
  PairLevel e[kTabChunk];
};
__global__ __launch_bounds__(64) void k_put_table(PairLevel* dst, int count, TabChunk ch) {
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int i = 0; i < kTabChunk; ++i)
    if (i < count) dst[i] = ch.e[i];
}

// Copies a transient context's error text to the context-free error buffer.
bdis_status static_fail(const bdis_ctx& sc, bdis_status s) {
  if (s != BDIS_OK) std::snprintf(g_create_err, sizeof g_create_err, "%s", sc.err);
  return s;
}

}  // namespace

extern "C" {

bdis_status bdis_params_default(bdis_params* p) {
  if (!p) return BDIS_E_ARG;
  std::memset(p, 0, sizeof(*p));
  p->levels = 5;
  p->finest_level = 0;
  p->patch = 10;
  p->stride = 4;
  p->iters = 12;
  p->sigma_r_dynamic = 1;
  p->variance = 0;
  p->float_pyramid = 0;
  p->sigma_s = 4.0f;
  p->sigma_r = 1.0f;
  p->valid_ratio = 0.75f;
  p->var_fail_sigma = 0.0f;
  p->var_fit_thresh = 0.1f;
  p->prob_thresh = 0.0f;
  p->fusion = 0;
  p->propagate = 1;
  for (int n = 0; n < BDIS_MAX_LEVELS; ++n) p->level_weight[n] = (float)(1 << n);
  return BDIS_OK;
}

bdis_status bdis_params_check(const bdis_params* p) {
  char msg[256];
  return check_params_msg(p, msg, sizeof msg);
}

bdis_status bdis_create(bdis_ctx** out, const bdis_params* p, int max_w, int max_h, int max_batch,
                        unsigned flags) {
  if (!out) return fail(nullptr, BDIS_E_ARG, "out is NULL");
  *out = nullptr;
  char msg[256];
  bdis_status st = check_params_msg(p, msg, sizeof msg);
  if (st != BDIS_OK) return fail(nullptr, st, "%s", msg);
  if (max_w < 1 || max_h < 1 || max_batch < 1 || (flags & ~(BDIS_TRAIN | BDIS_KEEP)) != 0)
    return fail(nullptr, BDIS_E_ARG, "max_w/max_h/max_batch must be >= 1 and flags a combination of BDIS_TRAIN, BDIS_KEEP");
  const bool train = (flags & BDIS_TRAIN) != 0;
  Layout lay;
  if (!make_layout(*p, max_w, max_h, p->levels, &lay, train))
    return fail(nullptr, BDIS_E_SIZE, "%dx%d with %d levels is smaller than patch %d", max_w, max_h,
                p->levels, p->patch);
  const char* fault = std::getenv("BDIS_FAULT");
  if (fault && std::strcmp(fault, "alloc") == 0)
    return fail(nullptr, BDIS_E_NOMEM, "workspace allocation failed (injected by BDIS_FAULT=alloc)");
  bdis_ctx* c = new (std::nothrow) bdis_ctx;
  if (!c) return fail(nullptr, BDIS_E_NOMEM, "host allocation failed");
  c->p = *p;
  c->max_w = max_w;
  c->max_h = max_h;
  c->max_batch = max_batch;
  c->slot_bytes = lay.total;
  c->train = train;
  c->keep = (flags & BDIS_KEEP) != 0;
  const char* g = std::getenv("BDIS_GRAPH");
  c->use_graph = !(g && std::strcmp(g, "0") == 0);
  auto mode = [](const char* v) { return !v ? -1 : std::strcmp(v, "0") == 0 ? 0 : std::strcmp(v, "1") == 0 ? 1 : -1; };
  c->top_mode = mode(std::getenv("BDIS_TOP"));
  c->chain_mode = mode(std::getenv("BDIS_CHAIN"));
  if (const char* so = std::getenv("BDIS_SEARCH_CONFIG")) {
    char* end = nullptr;
    const long v = std::strtol(so, &end, 10);
    if (end == so || *end != '\0' || v < 0 || v >= kNumSearchOptions ||
        search_lds_bytes(p->patch, (int)v, p->stride) > kSearchMaxLds) {
      delete c;
      return fail(nullptr, BDIS_E_ARG, "BDIS_SEARCH_CONFIG=%s: not a search configuration 0..%d for this patch and stride",
                  so, kNumSearchOptions - 1);
    }
    c->forced_opt = (int)v;
  }
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, BDIS_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, BDIS_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  }
  c->arch = prop.gcnArchName;
  for (char& ch : c->arch)
    if (ch == '"' || ch == ' ') ch = '_';
  c->tune_cache = tune_cache_path();
  if (!c->tune_cache.empty() && c->forced_opt < 0)
    for (const auto& kv : read_tune_cache(c->tune_cache))
      if (kv.first.compare(0, c->arch.size() + 1, c->arch + " ") == 0) c->tuned.insert(kv);
  e = hipMalloc(reinterpret_cast<void**>(&c->ws), c->slot_bytes * (size_t)max_batch);
  if (e != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return fail(nullptr, BDIS_E_NOMEM, "hipMalloc of %zu bytes: %s", lay.total * (size_t)max_batch,
                hipGetErrorString(e));
  }
  // zero the workspace once (every array is rewritten before it is read)
  e = hipMemset(c->ws, 0, c->slot_bytes * (size_t)max_batch);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->tab_evt, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done_evt, hipEventDisableTiming);
  if (e == hipSuccess && train) e = hipMalloc(reinterpret_cast<void**>(&c->hyper_dev), sizeof(double) * (2 + kMaxLevels));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->tab_evt) (void)hipEventDestroy(c->tab_evt);
    if (c->done_evt) (void)hipEventDestroy(c->done_evt);
    if (c->hyper_dev) (void)hipFree(c->hyper_dev);
    (void)hipFree(c->ws);
    delete c;
    return fail(nullptr, BDIS_E_HIP, "workspace init: %s", hipGetErrorString(e));
  }
  *out = c;
  return BDIS_OK;
}

bdis_status bdis_set_params(bdis_ctx* c, const bdis_params* p) {
  if (!c) return BDIS_E_ARG;
  char msg[256];
  bdis_status st = check_params_msg(p, msg, sizeof msg);
  if (st != BDIS_OK) return fail(c, st, "%s", msg);
  Layout lay;
  if (!make_layout(*p, c->max_w, c->max_h, p->levels, &lay, c->train) || lay.total > c->slot_bytes)
    return fail(c, BDIS_E_CAPACITY, "parameters need more workspace than the context holds");
  c->p = *p;
  c->have_last = false;
  c->last_f32.clear();
  return BDIS_OK;
}

bdis_status bdis_compute(bdis_ctx* c, const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                         float* disp, float* var, float* conf, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!left || !right || !disp) return fail(c, BDIS_E_ARG, "left, right and disparity are required");
  if (w < 1 || h < 1 || pitch < w) return fail(c, BDIS_E_ARG, "bad image size %dx%d pitch %d", w, h, pitch);
  if (var && !c->p.variance) return fail(c, BDIS_E_ARG, "variance output given but params.variance is 0");
  if (c->p.float_pyramid) return fail(c, BDIS_E_ARG, "uint8 input needs params.float_pyramid = 0");
  if (w > c->max_w || h > c->max_h)
    return fail(c, BDIS_E_CAPACITY, "image %dx%d exceeds the context's %dx%d", w, h, c->max_w, c->max_h);
  c->have_last = false;
  std::vector<PairSpec> v{PairSpec{left, right, w, h, pitch, c->p.levels, disp, var, conf}};
  bdis_status st = ordered(c, reinterpret_cast<hipStream_t>(stream), [&](hipStream_t ss) { return run_pairs(c, v, ss); });
  if (st == BDIS_OK) {
    c->last_w = w;
    c->last_h = h;
    c->have_last = true;
  }
  return st;
}

bdis_status bdis_compute_static(const bdis_params* p, const uint8_t* left, const uint8_t* right, int w, int h,
                                int pitch, float* disp, float* var, float* conf, void* stream) {
  char msg[256];
  bdis_status s = check_params_msg(p, msg, sizeof msg);
  if (s != BDIS_OK) return fail(nullptr, s, "%s", msg);
  if (!left || !right || !disp) return fail(nullptr, BDIS_E_ARG, "left, right and disparity are required");
  if (w < 1 || h < 1 || pitch < w) return fail(nullptr, BDIS_E_ARG, "bad image size %dx%d pitch %d", w, h, pitch);
  if (var && !p->variance) return fail(nullptr, BDIS_E_ARG, "variance output given but params.variance is 0");
  if (p->float_pyramid) return fail(nullptr, BDIS_E_ARG, "uint8 input needs params.float_pyramid = 0");
  Layout lay;
  if (!make_layout(*p, w, h, p->levels, &lay))
    return fail(nullptr, BDIS_E_SIZE, "a level of %dx%d with %d levels is smaller than patch %d", w, h, p->levels,
                p->patch);
  const size_t tab_bytes = align_up(sizeof(PairLevel) * kMaxLevels);
  if (tab_bytes + lay.total > kStaticScratchBytes)
    return fail(nullptr, BDIS_E_CAPACITY, "%dx%d with these parameters needs %zu bytes of the %zu-byte static scratch",
                w, h, tab_bytes + lay.total, kStaticScratchBytes);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, BDIS_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  char* base = nullptr;
  if ((e = static_scratch(dev, &base)) != hipSuccess)
    return fail(nullptr, BDIS_E_HIP, "static scratch address on device %d: %s", dev, hipGetErrorString(e));
  // a transient context on the stack whose workspace and job table are the scratch
  bdis_ctx sc;
  sc.p = *p;
  sc.max_w = w;
  sc.max_h = h;
  sc.max_batch = 1;
  sc.slot_bytes = lay.total;
  sc.ws = base + tab_bytes;
  sc.device = dev;
  sc.use_graph = 0;
  sc.tab_dev = reinterpret_cast<PairLevel*>(base);
  const PairSpec q{left, right, w, h, pitch, p->levels, disp, var, conf};
  Plan pl;
  if ((s = build_plan(&sc, &q, 1, &pl)) != BDIS_OK) return static_fail(sc, s);
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (size_t i0 = 0; i0 < pl.tab.size(); i0 += kTabChunk) {
    TabChunk ch;
    const int cnt = (int)std::min(pl.tab.size() - i0, (size_t)kTabChunk);
    std::memset(&ch, 0, sizeof ch);
    std::memcpy(ch.e, pl.tab.data() + i0, sizeof(PairLevel) * (size_t)cnt);
    hipLaunchKernelGGL(k_put_table, dim3(1), dim3(64), 0, st, sc.tab_dev + i0, cnt, ch);
    if ((e = hipGetLastError()) != hipSuccess) return fail(nullptr, BDIS_E_HIP, "job table: %s", hipGetErrorString(e));
  }
  return static_fail(sc, launch_all(&sc, pl, st));
}

bdis_status bdis_compute_batch(bdis_ctx* c, int n, const bdis_pair* pairs, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (n < 0 || (n > 0 && !pairs)) return fail(c, BDIS_E_ARG, "bad batch");
  if (n > c->max_batch) return fail(c, BDIS_E_CAPACITY, "batch of %d exceeds max_batch %d", n, c->max_batch);
  std::vector<PairSpec> v;
  v.reserve((size_t)n);
  for (int i = 0; i < n; ++i) {
    const bdis_pair& q = pairs[i];
    if (!q.left || !q.right || !q.disparity) return fail(c, BDIS_E_ARG, "pair %d: null pointer", i);
    if (q.w < 1 || q.h < 1 || q.pitch < q.w) return fail(c, BDIS_E_ARG, "pair %d: bad size", i);
    if (q.variance && !c->p.variance)
      return fail(c, BDIS_E_ARG, "pair %d: variance output without params.variance", i);
    if (q.levels < 0) return fail(c, BDIS_E_ARG, "pair %d: negative levels", i);
    const int lv = q.levels > 0 ? q.levels : c->p.levels;
    if (lv > c->p.levels) return fail(c, BDIS_E_CAPACITY, "pair %d: %d levels > %d", i, lv, c->p.levels);
    if (lv <= c->p.finest_level)
      return fail(c, BDIS_E_ARG, "pair %d: %d levels do not reach finest_level %d", i, lv, c->p.finest_level);
    if (q.w > c->max_w || q.h > c->max_h) return fail(c, BDIS_E_CAPACITY, "pair %d: %dx%d too large", i, q.w, q.h);
    v.push_back(PairSpec{q.left, q.right, q.w, q.h, q.pitch, lv, q.disparity, q.variance, q.confidence});
  }
  if (c->p.float_pyramid) return fail(c, BDIS_E_ARG, "uint8 input needs params.float_pyramid = 0");
  c->have_last = false;
  if (n == 0) return BDIS_OK;
  return ordered(c, reinterpret_cast<hipStream_t>(stream), [&](hipStream_t ss) { return run_pairs(c, v, ss); });
}

bdis_status bdis_compute_f32_batch(bdis_ctx* c, int n, const bdis_pair_f32* pairs, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!c->train) return fail(c, BDIS_E_STATE, "the float path needs a context created with BDIS_TRAIN");
  if (!c->p.float_pyramid) return fail(c, BDIS_E_ARG, "float input needs params.float_pyramid = 1");
  if (n < 1 || !pairs) return fail(c, BDIS_E_ARG, "bad batch");
  if (n > c->max_batch) return fail(c, BDIS_E_CAPACITY, "batch of %d exceeds max_batch %d", n, c->max_batch);
  std::vector<PairSpec> v;
  for (int i = 0; i < n; ++i) {
    const bdis_pair_f32& q = pairs[i];
    if (!q.left || !q.right || !q.disparity) return fail(c, BDIS_E_ARG, "pair %d: null pointer", i);
    if (q.w < 1 || q.h < 1 || q.pitch < q.w || q.levels < 0) return fail(c, BDIS_E_ARG, "pair %d: bad size", i);
    if (q.variance && !c->p.variance)
      return fail(c, BDIS_E_ARG, "pair %d: variance output without params.variance", i);
    const int lv = q.levels > 0 ? q.levels : c->p.levels;
    if (lv > c->p.levels) return fail(c, BDIS_E_CAPACITY, "pair %d: %d levels > %d", i, lv, c->p.levels);
    if (lv <= c->p.finest_level)
      return fail(c, BDIS_E_ARG, "pair %d: %d levels do not reach finest_level %d", i, lv, c->p.finest_level);
    if (q.w > c->max_w || q.h > c->max_h) return fail(c, BDIS_E_CAPACITY, "pair %d: %dx%d too large", i, q.w, q.h);
    PairSpec ps{nullptr, nullptr, q.w, q.h, q.pitch, lv, q.disparity, q.variance, q.confidence};
    ps.left32 = q.left;
    ps.right32 = q.right;
    v.push_back(ps);
  }
  c->have_last = false;
  c->last_f32.clear();
  bdis_status st =
      ordered(c, reinterpret_cast<hipStream_t>(stream), [&](hipStream_t ss) { return run_pairs_f32(c, v, ss); });
  if (st == BDIS_OK) c->last_f32 = v;
  return st;
}

bdis_status bdis_compute_f32(bdis_ctx* c, const float* left, const float* right, int w, int h, int pitch,
                             float* disp, float* var, float* conf, void* stream) {
  if (!c) return BDIS_E_ARG;
  bdis_pair_f32 q{left, right, w, h, pitch, 0, disp, var, conf};
  return bdis_compute_f32_batch(c, 1, &q, stream);
}

bdis_status bdis_backward_batch(bdis_ctx* c, int n, const bdis_pair_grad* grads, double* grad_hyper,
                                void* stream) {
  if (!c) return BDIS_E_ARG;
  if (c->last_f32.empty()) return fail(c, BDIS_E_STATE, "backward needs a preceding float-path compute");
  if (n != (int)c->last_f32.size() || !grads)
    return fail(c, BDIS_E_ARG, "backward batch of %d after a compute of %zu pairs", n, c->last_f32.size());
  std::vector<PairSpec> v = c->last_f32;
  for (int i = 0; i < n; ++i) {
    if (!grads[i].grad_disparity && !grads[i].grad_variance)
      return fail(c, BDIS_E_ARG, "pair %d: no output gradient", i);
    if (grads[i].grad_variance && !c->p.variance)
      return fail(c, BDIS_E_ARG, "pair %d: variance gradient without params.variance", i);
    v[i].grad_disp = grads[i].grad_disparity;
    v[i].grad_var = grads[i].grad_variance;
    v[i].grad_left = grads[i].grad_left;
    v[i].grad_right = grads[i].grad_right;
  }
  return ordered(c, reinterpret_cast<hipStream_t>(stream),
                 [&](hipStream_t ss) { return run_backward(c, v, grad_hyper, ss); });
}

bdis_status bdis_backward(bdis_ctx* c, const float* grad_disparity, const float* grad_variance, float* grad_left,
                          float* grad_right, double* grad_hyper, void* stream) {
  bdis_pair_grad g{grad_disparity, grad_variance, grad_left, grad_right};
  return bdis_backward_batch(c, 1, &g, grad_hyper, stream);
}

bdis_status bdis_debug_dump(bdis_ctx* c, int level, int what, void* host_dst, size_t bytes, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!c->have_last) return fail(c, BDIS_E_STATE, "no single-pair compute to dump");
  if (!host_dst || level < 0 || level >= c->p.levels) return fail(c, BDIS_E_ARG, "bad dump request");
  Layout lay;
  make_layout(c->p, c->last_w, c->last_h, c->p.levels, &lay, c->train);
  const LevelGeom& g = lay.g[level];
  const size_t npx = (size_t)g.w * g.h, np = (size_t)g.nx * g.ny;
  size_t off = 0, n = 0;
  const bool patch_level = level >= c->p.finest_level;
  switch (what) {
    case BDIS_DBG_LEFT: off = lay.lvl_l[level]; n = npx; break;
    case BDIS_DBG_RIGHT: off = lay.lvl_r[level]; n = npx; break;
    case BDIS_DBG_UINIT: off = lay.uinit[level]; n = np * 8; break;
    case BDIS_DBG_PIPAR: off = lay.pipar[level]; n = np * 8; break;
    case BDIS_DBG_U: off = lay.u[level]; n = np * 8; break;
    case BDIS_DBG_SSD0: off = lay.ssd0[level]; n = np * 8; break;
    case BDIS_DBG_DSSD: off = lay.dssd[level]; n = np * 32; break;
    case BDIS_DBG_RHO: off = lay.rho[level]; n = np * 4; break;
    case BDIS_DBG_ACC: off = lay.acc[level]; n = np * 4; break;
    case BDIS_DBG_HESS: off = lay.hess[level]; n = np * 4; break;
    case BDIS_DBG_DENS: off = lay.dens[level]; n = np * 32; break;
    case BDIS_DBG_UBAR: off = lay.ubar[level]; n = npx * 8; break;
    case BDIS_DBG_QMAP: off = lay.qmap[level]; n = npx * 8; break;
    case BDIS_DBG_SCAL: off = lay.scal[level]; n = 16; break;
    default: return fail(c, BDIS_E_ARG, "unknown dump %d", what);
  }
  if ((what == BDIS_DBG_LEFT || what == BDIS_DBG_RIGHT) && level == 0)
    return fail(c, BDIS_E_ARG, "level 0 images are the caller's inputs");
  if (!c->keep && (what == BDIS_DBG_UINIT || what == BDIS_DBG_SSD0 || what == BDIS_DBG_RHO ||
                   what == BDIS_DBG_HESS || what == BDIS_DBG_DENS))
    return fail(c, BDIS_E_STATE, "dump %d is stored only by contexts created with BDIS_KEEP", what);
  if ((what >= BDIS_DBG_UINIT && what <= BDIS_DBG_DENS) && !patch_level)
    return fail(c, BDIS_E_ARG, "level %d has no patches", level);
  if ((what == BDIS_DBG_UBAR || what == BDIS_DBG_QMAP) && level <= c->p.finest_level)
    return fail(c, BDIS_E_ARG, "the finest level writes the outputs, not level maps");
  if (bytes < n) return fail(c, BDIS_E_ARG, "buffer of %zu bytes < %zu", bytes, n);
  bdis_status so = check_device(c);
  if (so == BDIS_OK) so = order_after_last(c, reinterpret_cast<hipStream_t>(stream));
  if (so != BDIS_OK) return so;
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e == hipSuccess) {
    if (what == BDIS_DBG_LEFT || what == BDIS_DBG_RIGHT)  // padded rows -> dense W x H
      e = hipMemcpy2D(host_dst, g.w, c->ws + off, lay.lpitch[level], g.w, g.h, hipMemcpyDeviceToHost);
    else
      e = hipMemcpy(host_dst, c->ws + off, n, hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) return hip_fail(c, e, "debug dump");
  return BDIS_OK;
}

bdis_status bdis_depth(bdis_ctx* c, const float* disp, const float* var, int w, int h, int pitch, float fb,
                       float* depth, float* dvar, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!disp || !depth) return fail(c, BDIS_E_ARG, "disparity and depth are required");
  if ((var == nullptr) != (dvar == nullptr))
    return fail(c, BDIS_E_ARG, "variance and depth_variance go together");
  if (w < 1 || h < 1 || pitch < w || (long)w * h > (long)INT32_MAX)
    return fail(c, BDIS_E_ARG, "bad map size %dx%d pitch %d", w, h, pitch);
  if (!finite_f(fb) || !(fb > 0.0f)) return fail(c, BDIS_E_ARG, "fb must be finite and > 0");
  const hipError_t e = launch_depth(disp, var, w, h, pitch, fb, depth, dvar, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BDIS_OK : hip_fail(c, e, "depth launch");
}

bdis_status bdis_coverage(bdis_ctx* c, const float* disp, const float* var, const float* ref, const uint8_t* valid,
                          int w, int h, int pitch, float k, long long* counts, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!disp || !var || !ref || !counts) return fail(c, BDIS_E_ARG, "disparity, variance, reference and counts are required");
  if (w < 1 || h < 1 || pitch < w || (long)w * h > (long)INT32_MAX)
    return fail(c, BDIS_E_ARG, "bad map size %dx%d pitch %d", w, h, pitch);
  if (!finite_f(k) || k < 0.0f) return fail(c, BDIS_E_ARG, "k must be finite and >= 0");
  const hipError_t e = launch_coverage(disp, var, ref, valid, w, h, pitch, (double)k,
                                       reinterpret_cast<unsigned long long*>(counts),
                                       reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? BDIS_OK : hip_fail(c, e, "coverage launch");
}

bdis_status bdis_flow(bdis_ctx* c, const uint8_t* i0, const uint8_t* i1, int w, int h, int pitch, float* flow_u,
                      float* flow_v, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!i0 || !i1 || !flow_u || !flow_v) return fail(c, BDIS_E_ARG, "frames and both flow outputs are required");
  if (w < 1 || h < 1 || pitch < w) return fail(c, BDIS_E_ARG, "bad image size %dx%d pitch %d", w, h, pitch);
  if (c->p.float_pyramid) return fail(c, BDIS_E_ARG, "uint8 frames need params.float_pyramid = 0");
  if (c->p.finest_level != 0) return fail(c, BDIS_E_ARG, "the flow form needs finest_level 0");
  if (w > c->max_w || h > c->max_h)
    return fail(c, BDIS_E_CAPACITY, "image %dx%d exceeds the context's %dx%d", w, h, c->max_w, c->max_h);
  c->have_last = false;
  PairSpec ps{i0, i1, w, h, pitch, c->p.levels, nullptr, nullptr, nullptr};
  ps.flow_u = flow_u;
  ps.flow_v = flow_v;
  std::vector<PairSpec> v{ps};
  const bdis_status st =
      ordered(c, reinterpret_cast<hipStream_t>(stream), [&](hipStream_t ss) { return run_flow(c, v, ss); });
  if (st == BDIS_OK) {  // per-patch flow stays readable through bdis_debug_dump (u: BDIS_DBG_U, v: BDIS_DBG_UINIT)
    c->last_w = w;
    c->last_h = h;
    c->have_last = true;
  }
  return st;
}

bdis_status bdis_level_dims(const bdis_params* p, int w, int h, int level, int* lw, int* lh, int* nx, int* ny) {
  char msg[256];
  if (check_params_msg(p, msg, sizeof msg) != BDIS_OK) return BDIS_E_ARG;
  if (level < 0 || level >= p->levels || w < 1 || h < 1) return BDIS_E_ARG;
  LevelGeom g[kMaxLevels];
  if (!level_geometry(*p, w, h, p->levels, g)) return BDIS_E_SIZE;
  if (lw) *lw = g[level].w;
  if (lh) *lh = g[level].h;
  if (nx) *nx = g[level].nx;
  if (ny) *ny = g[level].ny;
  return BDIS_OK;
}

bdis_status bdis_timing_enable(bdis_ctx* c, int enable) {
  if (!c) return BDIS_E_ARG;
  c->tm.on = enable != 0;
  c->tm.used = 0;
  c->tm.marks.clear();
  return BDIS_OK;
}

bdis_status bdis_setup_time(bdis_ctx* c, double* tune_ms, double* capture_ms) {
  if (!c || !tune_ms || !capture_ms) return BDIS_E_ARG;
  *tune_ms = c->last_tune_ms;
  *capture_ms = c->last_capture_ms;
  return BDIS_OK;
}

bdis_status bdis_timing_read(bdis_ctx* c, int kernel, double* total_ms, long* launches) {
  return bdis_timing_read_level(c, kernel, -1, total_ms, launches);
}

bdis_status bdis_timing_read_level(bdis_ctx* c, int kernel, int level, double* total_ms, long* launches) {
  if (!c || kernel < 0 || kernel >= BDIS_K_COUNT || level < -1 || level >= kMaxLevels || !total_ms || !launches)
    return BDIS_E_ARG;
  double tot = 0.0;
  long n = 0;
  for (const auto& m : c->tm.marks) {
    if (m.kernel != kernel || (level >= 0 && m.level != level)) continue;
    hipError_t e = hipEventSynchronize(c->tm.pool[m.idx + 1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->tm.pool[m.idx], c->tm.pool[m.idx + 1]);
    if (e != hipSuccess) return hip_fail(c, e, "timing read");
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return BDIS_OK;
}

void bdis_destroy(bdis_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : c->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  for (hipEvent_t e : c->tm.pool) (void)hipEventDestroy(e);
  if (c->tab_evt) (void)hipEventDestroy(c->tab_evt);
  if (c->done_evt) (void)hipEventDestroy(c->done_evt);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->tab_dev) (void)hipFree(c->tab_dev);
  if (c->tab_host) (void)hipHostFree(c->tab_host);
  if (c->hyper_dev) (void)hipFree(c->hyper_dev);
  if (c->ws) (void)hipFree(c->ws);
  delete c;
}

const char* bdis_last_error(const bdis_ctx* c) { return c ? c->err : g_create_err; }

const char* bdis_version(void) { return "bdis-gfx950 0.4"; }

}  // extern "C"
