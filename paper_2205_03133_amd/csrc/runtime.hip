// C-ABI runtime of the BDIS library: parameter validation, the device
// workspace, and the launch sequence of one coarse-to-fine pass (Fig. 1):
//   pyramid of both views, then for n = L-1 .. f:
//     patch search (+ sigma_r reduction), patch probability, fusion.
// Every launch goes to the caller's stream; nothing here synchronises the host
// except bdis_create, bdis_destroy and bdis_debug_dump.
#include <bdis.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

#include "bdis_internal.h"

using namespace bdis;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of every array of one pair within its workspace slot.
struct Layout {
  int levels = 0;
  LevelGeom g[kMaxLevels]{};
  int nblocks[kMaxLevels]{};
  size_t lvl_l[kMaxLevels]{}, lvl_r[kMaxLevels]{};
  size_t uinit[kMaxLevels]{}, pipar[kMaxLevels]{}, u[kMaxLevels]{}, ssd0[kMaxLevels]{},
      dssd[kMaxLevels]{}, rho[kMaxLevels]{}, acc[kMaxLevels]{}, hess[kMaxLevels]{},
      dens[kMaxLevels]{};
  size_t ubar[kMaxLevels]{}, qmap[kMaxLevels]{};
  size_t part_sum[kMaxLevels]{}, part_cnt[kMaxLevels]{}, counter[kMaxLevels]{}, scal[kMaxLevels]{};
  size_t total = 0;
};

int search_blocks(const LevelGeom& g, int P) {
  const int npb = kThreads / group_lanes(P);
  return (g.nx + npb - 1) / npb * g.ny;
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

bool make_layout(const bdis_params& p, int w, int h, int levels, Layout* lay) {
  Layout L;
  L.levels = levels;
  if (!level_geometry(p, w, h, levels, L.g)) return false;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  for (int n = 0; n < levels; ++n) {
    const size_t npx = (size_t)L.g[n].w * L.g[n].h;
    if (n >= 1) {
      L.lvl_l[n] = take(npx);
      L.lvl_r[n] = take(npx);
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
    L.nblocks[n] = search_blocks(L.g[n], p.patch);
    L.part_sum[n] = take((size_t)L.nblocks[n] * 8);
    L.part_cnt[n] = take((size_t)L.nblocks[n] * 4);
    L.counter[n] = take(64);
    L.scal[n] = take(64);
  }
  L.total = off;
  *lay = L;
  return true;
}

bool finite_f(float v) { return std::isfinite(v); }

}  // namespace

// HIP events recorded around each launch while timing is enabled.
struct Timing {
  bool on = false;
  std::vector<hipEvent_t> pool;                 // reused events
  size_t used = 0;                              // events handed out since enable
  std::vector<std::pair<int, size_t>> marks;    // (kernel, index of start event)
};

struct bdis_ctx {
  bdis_params p{};
  Timing tm;
  int max_w = 0, max_h = 0, max_batch = 0;
  size_t slot_bytes = 0;
  char* ws = nullptr;
  int device = 0;
  // geometry of the last single-pair compute (slot 0), for debug dumps
  int last_w = 0, last_h = 0;
  bool have_last = false;
  char err[512] = {0};
};

namespace {

char g_create_err[512] = {0};

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
  if (p->finest_level != 0)
    return snprintf(msg, n, "finest_level %d unsupported (only 0)", p->finest_level), BDIS_E_ARG;
  if (p->patch < 3 || p->patch > BDIS_MAX_PATCH)
    return snprintf(msg, n, "patch %d outside 3..%d", p->patch, BDIS_MAX_PATCH), BDIS_E_ARG;
  if (p->stride < 1 || p->stride > p->patch)
    return snprintf(msg, n, "stride %d outside 1..patch", p->stride), BDIS_E_ARG;
  if (p->iters < 1 || p->iters > 256) return snprintf(msg, n, "iters %d outside 1..256", p->iters), BDIS_E_ARG;
  if (p->float_pyramid != 0) return snprintf(msg, n, "float_pyramid must be 0 for uint8 input"), BDIS_E_ARG;
  if (!finite_f(p->sigma_s) || !(p->sigma_s > 0.0f)) return snprintf(msg, n, "sigma_s must be > 0"), BDIS_E_ARG;
  if (!finite_f(p->sigma_r) || !(p->sigma_r > 0.0f)) return snprintf(msg, n, "sigma_r must be > 0"), BDIS_E_ARG;
  if (!finite_f(p->valid_ratio)) return snprintf(msg, n, "valid_ratio not finite"), BDIS_E_ARG;
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

hipEvent_t next_event(bdis_ctx* c) {
  if (c->tm.used == c->tm.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->tm.pool.push_back(e);
  }
  return c->tm.pool[c->tm.used++];
}

// Records a start event for `kernel` (no-op unless timing is on); returns the mark index.
long timing_start(bdis_ctx* c, int kernel, hipStream_t st) {
  if (!c->tm.on) return -1;
  const size_t idx = c->tm.used;
  hipEvent_t a = next_event(c);
  hipEvent_t b = next_event(c);
  if (!a || !b) return -1;
  (void)hipEventRecord(a, st);
  c->tm.marks.emplace_back(kernel, idx);
  return (long)idx;
}

void timing_stop(bdis_ctx* c, long mark, hipStream_t st) {
  if (mark < 0) return;
  (void)hipEventRecord(c->tm.pool[(size_t)mark + 1], st);
}

// Launch sequence of one pair in slot `slot`.  Inputs were validated.
bdis_status run_pair(bdis_ctx* c, int slot, const uint8_t* left, const uint8_t* right, int w, int h,
                     int pitch, int levels, float* disp, float* var, float* conf, hipStream_t st) {
  const bdis_params& p = c->p;
  Layout lay;
  if (!make_layout(p, w, h, levels, &lay))
    return fail(c, BDIS_E_SIZE, "a level of %dx%d with %d levels is smaller than patch %d", w, h, levels, p.patch);
  if (lay.total > c->slot_bytes)
    return fail(c, BDIS_E_CAPACITY, "pair %dx%d (%d levels) needs %zu workspace bytes > %zu", w, h, levels,
                lay.total, c->slot_bytes);
  char* base = c->ws + (size_t)slot * c->slot_bytes;
  auto P8 = [&](size_t o) { return reinterpret_cast<uint8_t*>(base + o); };
  auto PF = [&](size_t o) { return reinterpret_cast<float*>(base + o); };
  auto PD = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
  hipError_t e;

  // pyramid of both views (levels 1 .. L-1)
  for (int n = 1; n < levels; ++n) {
    PyrArgs a;
    a.srcL = n == 1 ? left : P8(lay.lvl_l[n - 1]);
    a.srcR = n == 1 ? right : P8(lay.lvl_r[n - 1]);
    a.spitch = n == 1 ? pitch : lay.g[n - 1].w;
    a.sw = lay.g[n - 1].w;
    a.sh = lay.g[n - 1].h;
    a.dstL = P8(lay.lvl_l[n]);
    a.dstR = P8(lay.lvl_r[n]);
    a.dw = lay.g[n].w;
    a.dh = lay.g[n].h;
    const long tmk = timing_start(c, BDIS_K_PYRAMID, st);
    e = launch_pyramid_u8(a, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "pyramid launch");
  }

  for (int n = levels - 1; n >= p.finest_level; --n) {
    const LevelGeom& g = lay.g[n];
    PatchArrays pa;
    pa.uinit = PD(lay.uinit[n]);
    pa.pipar = PD(lay.pipar[n]);
    pa.u = PD(lay.u[n]);
    pa.ssd0 = PD(lay.ssd0[n]);
    pa.dssd = reinterpret_cast<D4*>(base + lay.dssd[n]);
    pa.rho = PF(lay.rho[n]);
    pa.acc = reinterpret_cast<int*>(base + lay.acc[n]);
    pa.hess = PF(lay.hess[n]);
    pa.dens = reinterpret_cast<D4*>(base + lay.dens[n]);
    const bool has_par = n + 1 < levels;
    double* scal = reinterpret_cast<double*>(base + lay.scal[n]);

    SearchArgs sa;
    sa.L = n == 0 ? left : P8(lay.lvl_l[n]);
    sa.R = n == 0 ? right : P8(lay.lvl_r[n]);
    sa.pitch = n == 0 ? pitch : g.w;
    sa.g = g;
    sa.S = p.stride;
    sa.K = p.iters;
    sa.valid_ratio = p.valid_ratio;
    sa.par_ubar = has_par ? PD(lay.ubar[n + 1]) : nullptr;
    sa.par_q = has_par ? PD(lay.qmap[n + 1]) : nullptr;
    sa.pw = has_par ? lay.g[n + 1].w : 0;
    sa.ph = has_par ? lay.g[n + 1].h : 0;
    sa.pa = pa;
    sa.part_sum = reinterpret_cast<double*>(base + lay.part_sum[n]);
    sa.part_cnt = reinterpret_cast<int*>(base + lay.part_cnt[n]);
    sa.counter = reinterpret_cast<unsigned*>(base + lay.counter[n]);
    sa.scal = scal;
    sa.sigma_r_dynamic = p.sigma_r_dynamic;
    sa.sigma_r = p.sigma_r;
    long tmk = timing_start(c, BDIS_K_SEARCH, st);
    e = launch_search_u8(p.patch, sa, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "search launch");

    ProbArgs pr;
    pr.pa = pa;
    pr.np = g.nx * g.ny;
    pr.scal = scal;
    for (int k = 0; k < kMaxLevels; ++k) pr.omega[k] = p.level_weight[k];
    pr.level = n;
    pr.finest = p.finest_level;
    pr.levels = levels;
    pr.variance = p.variance;
    pr.P = p.patch;
    pr.var_fit_thresh = p.var_fit_thresh;
    pr.var_fail_sigma = p.var_fail_sigma;
    tmk = timing_start(c, BDIS_K_PROB, st);
    e = launch_prob(pr, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "probability launch");

    DensifyArgs da;
    da.dens = pa.dens;
    da.g = g;
    da.P = p.patch;
    da.S = p.stride;
    da.sigma_s = p.sigma_s;
    da.par_ubar = sa.par_ubar;
    da.par_q = sa.par_q;
    da.pw = sa.pw;
    da.ph = sa.ph;
    da.finest = n == p.finest_level;
    da.ubar = da.finest ? nullptr : PD(lay.ubar[n]);
    da.qmap = da.finest ? nullptr : PD(lay.qmap[n]);
    da.disparity = disp;
    da.variance = var;
    da.confidence = conf;
    da.variance_on = p.variance;
    da.prob_thresh = p.prob_thresh;
    tmk = timing_start(c, BDIS_K_FUSE, st);
    e = launch_densify(da, st);
    timing_stop(c, tmk, st);
    if (e != hipSuccess) return hip_fail(c, e, "fusion launch");
  }
  return BDIS_OK;
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
  if (max_w < 1 || max_h < 1 || max_batch < 1 || flags != 0)
    return fail(nullptr, BDIS_E_ARG, "max_w/max_h/max_batch must be >= 1 and flags 0");
  Layout lay;
  if (!make_layout(*p, max_w, max_h, p->levels, &lay))
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
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, BDIS_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  e = hipMalloc(reinterpret_cast<void**>(&c->ws), c->slot_bytes * (size_t)max_batch);
  if (e != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return fail(nullptr, BDIS_E_NOMEM, "hipMalloc of %zu bytes: %s", c->slot_bytes * (size_t)max_batch,
                hipGetErrorString(e));
  }
  // zero the workspace once: the reduction counters must start at 0
  e = hipMemset(c->ws, 0, c->slot_bytes * (size_t)max_batch);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
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
  if (!make_layout(*p, c->max_w, c->max_h, p->levels, &lay) || lay.total > c->slot_bytes)
    return fail(c, BDIS_E_CAPACITY, "parameters need more workspace than the context holds");
  c->p = *p;
  c->have_last = false;
  return BDIS_OK;
}

bdis_status bdis_compute(bdis_ctx* c, const uint8_t* left, const uint8_t* right, int w, int h, int pitch,
                         float* disp, float* var, float* conf, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!left || !right || !disp) return fail(c, BDIS_E_ARG, "left, right and disparity are required");
  if (w < 1 || h < 1 || pitch < w) return fail(c, BDIS_E_ARG, "bad image size %dx%d pitch %d", w, h, pitch);
  if (var && !c->p.variance) return fail(c, BDIS_E_ARG, "variance output given but params.variance is 0");
  if (w > c->max_w || h > c->max_h)
    return fail(c, BDIS_E_CAPACITY, "image %dx%d exceeds the context's %dx%d", w, h, c->max_w, c->max_h);
  c->have_last = false;
  bdis_status st = run_pair(c, 0, left, right, w, h, pitch, c->p.levels, disp, var, conf,
                            reinterpret_cast<hipStream_t>(stream));
  if (st == BDIS_OK) {
    c->last_w = w;
    c->last_h = h;
    c->have_last = true;
  }
  return st;
}

bdis_status bdis_compute_batch(bdis_ctx* c, int n, const bdis_pair* pairs, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (n < 0 || (n > 0 && !pairs)) return fail(c, BDIS_E_ARG, "bad batch");
  if (n > c->max_batch) return fail(c, BDIS_E_CAPACITY, "batch of %d exceeds max_batch %d", n, c->max_batch);
  // validate everything before launching anything
  for (int i = 0; i < n; ++i) {
    const bdis_pair& q = pairs[i];
    if (!q.left || !q.right || !q.disparity) return fail(c, BDIS_E_ARG, "pair %d: null pointer", i);
    if (q.w < 1 || q.h < 1 || q.pitch < q.w) return fail(c, BDIS_E_ARG, "pair %d: bad size", i);
    if (q.variance && !c->p.variance) return fail(c, BDIS_E_ARG, "pair %d: variance output without params.variance", i);
    const int lv = q.levels > 0 ? q.levels : c->p.levels;
    if (lv > c->p.levels) return fail(c, BDIS_E_CAPACITY, "pair %d: %d levels > %d", i, lv, c->p.levels);
    if (q.w > c->max_w || q.h > c->max_h) return fail(c, BDIS_E_CAPACITY, "pair %d: %dx%d too large", i, q.w, q.h);
    Layout lay;
    if (!make_layout(c->p, q.w, q.h, lv, &lay)) return fail(c, BDIS_E_SIZE, "pair %d: level smaller than patch", i);
    if (lay.total > c->slot_bytes) return fail(c, BDIS_E_CAPACITY, "pair %d: workspace", i);
  }
  c->have_last = false;
  for (int i = 0; i < n; ++i) {
    const bdis_pair& q = pairs[i];
    const int lv = q.levels > 0 ? q.levels : c->p.levels;
    bdis_status st = run_pair(c, i, q.left, q.right, q.w, q.h, q.pitch, lv, q.disparity, q.variance,
                              q.confidence, reinterpret_cast<hipStream_t>(stream));
    if (st != BDIS_OK) return st;
  }
  return BDIS_OK;
}

bdis_status bdis_debug_dump(bdis_ctx* c, int level, int what, void* host_dst, size_t bytes, void* stream) {
  if (!c) return BDIS_E_ARG;
  if (!c->have_last) return fail(c, BDIS_E_STATE, "no single-pair compute to dump");
  if (!host_dst || level < 0 || level >= c->p.levels) return fail(c, BDIS_E_ARG, "bad dump request");
  Layout lay;
  make_layout(c->p, c->last_w, c->last_h, c->p.levels, &lay);
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
  if ((what >= BDIS_DBG_UINIT && what <= BDIS_DBG_DENS) && !patch_level)
    return fail(c, BDIS_E_ARG, "level %d has no patches", level);
  if ((what == BDIS_DBG_UBAR || what == BDIS_DBG_QMAP) && level <= c->p.finest_level)
    return fail(c, BDIS_E_ARG, "the finest level writes the outputs, not level maps");
  if (bytes < n) return fail(c, BDIS_E_ARG, "buffer of %zu bytes < %zu", bytes, n);
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipMemcpy(host_dst, c->ws + off, n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "debug dump");
  return BDIS_OK;
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

bdis_status bdis_timing_read(bdis_ctx* c, int kernel, double* total_ms, long* launches) {
  if (!c || kernel < 0 || kernel >= BDIS_K_COUNT || !total_ms || !launches)
    return BDIS_E_ARG;
  double tot = 0.0;
  long n = 0;
  for (const auto& m : c->tm.marks) {
    if (m.first != kernel) continue;
    hipError_t e = hipEventSynchronize(c->tm.pool[m.second + 1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->tm.pool[m.second], c->tm.pool[m.second + 1]);
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
  for (hipEvent_t e : c->tm.pool) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
  delete c;
}

const char* bdis_last_error(const bdis_ctx* c) { return c ? c->err : g_create_err; }

const char* bdis_version(void) { return "bdis-gfx950 0.1"; }

}  // extern "C"
