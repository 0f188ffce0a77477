// C ABI of libfga: argument validation, state management and the host loop
// of Alg. 2. Every argument check runs before the first HIP call, so invalid
// requests fail identically with or without a GPU.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <cstdlib>
#include <limits>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "rigid.h"

namespace fga {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

namespace {

// point and node indices are 32-bit inside the kernels and child-block
// indices use 28 bits (a tree has fewer than 2 nodes per point)
constexpr int64_t kMaxPoints = (int64_t)1 << 27;

fga_status check_params(const fga_params* p) {
  if (!p) {
    set_error("params is NULL");
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->G) && p->G > 0)) {
    set_error("G must be finite and > 0 (got %g)", p->G);
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->eps) && p->eps > 0)) {
    set_error("eps must be finite and > 0 (got %g)", p->eps);
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->dt) && p->dt > 0)) {
    set_error("dt must be finite and > 0 (got %g)", p->dt);
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->eta) && p->eta >= 0)) {
    set_error("eta must be finite and >= 0 (got %g)", p->eta);
    return FGA_E_INVALID_ARG;
  }
  if (p->damping != FGA_DAMP_FRACTION && p->damping != FGA_DAMP_LITERAL) {
    set_error("unknown damping mode %d", p->damping);
    return FGA_E_INVALID_ARG;
  }
  if (p->damping == FGA_DAMP_FRACTION && p->eta > 1.0) {
    set_error("fraction damping needs eta in [0, 1] (got %g)", p->eta);
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->theta) && p->theta >= 0)) {
    set_error("theta must be finite and >= 0 (got %g)", p->theta);
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->a) && std::isfinite(p->b) && p->a < p->b)) {
    set_error("normalisation range needs a < b (got [%g, %g])", p->a, p->b);
    return FGA_E_INVALID_ARG;
  }
  if (p->rho < 1 || p->rho > 64) {
    set_error("rho must be in [1, 64] (got %d)", p->rho);
    return FGA_E_INVALID_ARG;
  }
  if (p->max_depth != kQBits) {
    set_error("max_depth %d: only the paper's depth limit 20 is supported", p->max_depth);
    return FGA_E_UNSUPPORTED;
  }
  if (p->max_iter < 0) {
    set_error("max_iter must be >= 0 (got %d)", p->max_iter);
    return FGA_E_INVALID_ARG;
  }
  if (!std::isfinite(p->tol)) {
    set_error("tol must be finite");
    return FGA_E_INVALID_ARG;
  }
  if (p->velocity != FGA_VEL_RIGID && p->velocity != FGA_VEL_PARTICLE) {
    set_error("unknown velocity mode %d", p->velocity);
    return FGA_E_INVALID_ARG;
  }
  if (p->mass_mode != FGA_MASS_NIV && p->mass_mode != FGA_MASS_UNIFORM) {
    set_error("unknown mass mode %d", p->mass_mode);
    return FGA_E_INVALID_ARG;
  }
  if (p->precision < FGA_PREC_FP32 || p->precision > FGA_PREC_FP32_ALL) {
    set_error("unknown precision %d", p->precision);
    return FGA_E_INVALID_ARG;
  }
  if (p->leaf_size < 0 || p->leaf_size > 64) {
    set_error("leaf_size must be in [0, 64] (got %d)", p->leaf_size);
    return FGA_E_INVALID_ARG;
  }
  if (p->group_width != 0 && p->group_width != 1 && p->group_width != 32 &&
      p->group_width != 64 && p->group_width != 128) {
    set_error("group_width must be 0, 1, 32, 64 or 128 (got %d)", p->group_width);
    return FGA_E_INVALID_ARG;
  }
  if (p->tile < 0 || p->tile > 255 || p->check_every < 0) {
    set_error("tile must be in [0, 255] and check_every >= 0");
    return FGA_E_INVALID_ARG;
  }
  if (!(std::isfinite(p->rbf_sigma) && p->rbf_sigma > 0 && std::isfinite(p->rbf_weight) &&
        p->rbf_weight > 0)) {
    set_error("rbf_sigma and rbf_weight must be finite and > 0 (got %g, %g)", p->rbf_sigma,
              p->rbf_weight);
    return FGA_E_INVALID_ARG;
  }
  return FGA_OK;
}

// Landmark indices (host memory): count in [0, 64], every index in [0, n).
fga_status check_landmarks(const int64_t* idx, int count, int64_t n, const char* what) {
  if (count < 0 || count > kMaxLandmarkPairs) {
    set_error("landmark count must be in [0, %d] (got %d)", kMaxLandmarkPairs, count);
    return FGA_E_INVALID_ARG;
  }
  if (count > 0 && !idx) {
    set_error("%s is NULL with %d landmarks", what, count);
    return FGA_E_INVALID_ARG;
  }
  for (int k = 0; k < count; ++k)
    if (idx[k] < 0 || idx[k] >= n) {
      set_error("%s[%d] = %lld is outside [0, %lld)", what, k, (long long)idx[k], (long long)n);
      return FGA_E_INVALID_ARG;
    }
  return FGA_OK;
}

fga_status check_dtype(fga_dtype dt) {
  if (dt != FGA_F32 && dt != FGA_F64) {
    set_error("unknown dtype %d", (int)dt);
    return FGA_E_INVALID_ARG;
  }
  return FGA_OK;
}

fga_status check_count(int64_t n, const char* what) {
  if (n < 1 || n > kMaxPoints) {
    set_error("%s must be in [1, 2^27] (got %lld)", what, (long long)n);
    return FGA_E_INVALID_ARG;
  }
  return FGA_OK;
}

fga_status check_ptr(const void* p, const char* what) {
  if (!p) {
    set_error("%s is NULL", what);
    return FGA_E_INVALID_ARG;
  }
  return FGA_OK;
}

// Device accessibility of a caller pointer (after the host-only checks).
fga_status check_device_ptr(const void* p, const char* what) {
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof at);
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("%s is not device-accessible memory (%s)", what, hipGetErrorString(e));
    return FGA_E_INVALID_ARG;
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged &&
      at.type != hipMemoryTypeUnified && at.type != hipMemoryTypeHost) {
    set_error("%s is not device-accessible memory (memory type %d)", what, (int)at.type);
    return FGA_E_INVALID_ARG;
  }
  return FGA_OK;
}

size_t dsize(fga_dtype dt) { return dt == FGA_F64 ? 8 : 4; }

IterConsts make_iter_consts(const fga_params& p) {
  IterConsts c;
  c.G = p.G;
  c.eps2 = p.eps * p.eps;
  c.dt = p.dt;
  c.theta2 = p.theta * p.theta;
  c.fG = (float)c.G;
  c.feps2 = (float)c.eps2;
  c.fdt = (float)c.dt;
  c.ftheta2 = (float)c.theta2;
  c.damping = p.damping;
  c.velocity = p.velocity;
  c.prec = p.precision;
  c.pad_ = 0;
  return c;
}

// Reference ranges per template tile for the BH iteration: enough waves to
// keep every SIMD busy, few enough that the shared top of the tree is not
// re-walked too often.
int bh_ranges(int64_t m, int64_t n) {
  const int64_t waves = (m + kWave - 1) / kWave;
  int64_t jr = (4096 + waves - 1) / waves;
  if (jr > 8) jr = 8;
  if (jr > (n + 255) / 256) jr = (n + 255) / 256;
  return jr < 1 ? 1 : (int)jr;
}

// ---------------------------------------------------------------- autotuner
// The number of reference ranges per template tile trades parallelism (more
// waves to hide scalar-load latency) against repeated work at the top of the
// tree (BH) or extra partial moments (direct). It is chosen by timing a few
// iterations of the real kernel on a copy of the state, once per shape class;
// results are kept for the process and, if FGA_TUNE_CACHE names a file, on disk.
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(bool bh, bool f64, int64_t m, int64_t n, int prec, int group_width) {
  auto lg = [](int64_t v) {
    int k = 0;
    while ((int64_t(1) << (k + 1)) <= v) ++k;
    return k;
  };
  char buf[96];
  snprintf(buf, sizeof buf, "%s_%s_p%d_g%d_m%d_n%d", bh ? "bh" : "direct", f64 ? "f64" : "f32",
           prec, group_width, lg(m), lg(n));
  return buf;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("FGA_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[128];
  int v;
  while (fscanf(f, " \"%127[^\"]\" : %d ,", key, &v) == 2) g_tune[key] = v;
  fclose(f);
}

void tune_save_locked() {
  const char* path = getenv("FGA_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (auto& kv : g_tune) fprintf(f, "\"%s\": %d,\n", kv.first.c_str(), kv.second);
  fclose(f);
}

void denormalise(const NormInfo& ni, const double* R, const double* tn, double* t) {
  // X = s (Xn - a) + mean(X) + l, Y = s (Yn - a) + mean(Y) + l with
  // s = (r - l)/(b - a) (inverse of Eq. A.3); Xn = R Yn + tn then gives
  // t = mean(X) - R mean(Y) + s (R a1 + tn - a1) + l1 - R l1.
  const double s = (ni.r - ni.l) / (ni.b - ni.a);
  for (int i = 0; i < 3; ++i) {
    double Ra = 0.0, Ry = 0.0, Rl = 0.0;
    for (int j = 0; j < 3; ++j) {
      Ra += R[3 * i + j] * ni.a;
      Ry += R[3 * i + j] * ni.ybar[j];
      Rl += R[3 * i + j] * ni.l;
    }
    t[i] = ni.xbar[i] - Ry + s * (Ra + tn[i] - ni.a) + ni.l - Rl;
  }
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace
}  // namespace fga

using namespace fga;

// ---------------------------------------------------------------- the state
struct fga_state {
  fga_params p;
  fga_dtype dt;
  hipStream_t s;
  bool f64;
  int64_t n, m;
  void* X = nullptr;        // packed reference (Morton-sorted for BH)
  void* Q = nullptr;        // packed template (Morton-sorted)
  BHWide* nodes = nullptr;  // BH tree in child-block layout (the one in use)
  int n_nodes = 0;
  // the trees of the leaf sizes the autotuner may choose from (one entry
  // when the leaf size is given); a work-split code carries the index
  std::vector<BHWide*> trees;
  std::vector<int> tree_nodes, tree_leaf;
  int leaf_used = 0;                    // leaf size of the tree in use
  RigidState* st = nullptr;
  double* partial = nullptr;
  unsigned* done = nullptr;
  void* V = nullptr;
  PairDev pd;
  IterConsts c;
  NormInfo norm;
  int tree_stats[3] = {0, 0, 0};
  struct Groups {
    std::vector<int2> host;             // (first, count) of every group, Morton order
    int n = 0;
    std::vector<unsigned> cost;         // measured list entries per group (empty: not yet)
    std::map<int, std::pair<int4*, int>> items;  // range cap -> wave items, count
  };
  std::map<int, Groups> groups;         // key 16 * tree index + 4 K + tau option
  // group walk whose costs are measured by the first iteration of fga_step
  // (registrations): the K, tau option, part cap and tree of the pending split
  int pend_K = 0, pend_fi = 0, pend_cap = 0, pend_li = 0;
  int run = 0;  // particles per group of the group walk in use (32, 64 or 128)
  int4* ident_items = nullptr;          // one wave item per group, Morton order
};

struct fga_tree {
  int64_t n;
  hipStream_t s = nullptr;
  BHNode* nodes = nullptr;  // preorder (exported)
  BHWide* wide = nullptr;   // child-block layout (traversed)
  int n_nodes = 0;
  int* order = nullptr;
  void* Xs = nullptr;
  int stats[3] = {0, 0, 0};
};

static void state_free(fga_state* S) {
  if (!S) return;
  const hipStream_t s = S->s;
  pool_free(S->X, s);
  pool_free(S->Q, s);
  for (BHWide* t : S->trees) pool_free(t, s);
  pool_free(S->st, s);
  pool_free(S->partial, s);
  pool_free(S->done, s);
  pool_free(S->V, s);
  for (auto& kv : S->groups)
    for (auto& it : kv.second.items) pool_free(it.second.first, s);
  pool_free(S->ident_items, s);
  delete S;
}

// Groups of the template for the group walk, over its Morton order (built on
// the device by device_groups): greedy runs of at most G consecutive
// particles; with f > 0 a run also ends before its bounding-box diagonal
// would exceed f times the median diagonal of aligned G-runs (f = 1.5 and 3
// timed no faster than these on the LiDAR and mesh workloads).
// Tau options fi = 0..3 bound runs of 64 K particles; fi = 4..7 take the
// same bounds on runs of at most 32 (K = 1), which the kernel holds twice
// over the wave's lanes: smaller boxes accept more nodes, and a launch has
// twice as many waves.
static const double kGroupTau[4] = {0.0, 1.0, 2.0, 4.0};
static int group_run(int K, int fi) { return fi >= 4 ? kWave / 2 : kWave * K; }
// leaf sizes the autotuner chooses from (leaf_size 0)
static const int kLeafOpts[] = {1, 2, 4, 8, 16};
constexpr int kNumLeafOpts = 5;

static fga_status upload_items(fga_state* S, const std::vector<int4>& v, int4** out) {
  FGA_TRY(pool_get(out, sizeof(int4) * std::max<size_t>(1, v.size()), S->s));
  FGA_HIP(hipMemcpyAsync(*out, v.data(), sizeof(int4) * v.size(), hipMemcpyHostToDevice, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  return FGA_OK;
}

// Wave items of an iteration that measures the groups' costs: every group
// in `parts` parts by subtrees (a fixed rule, so registrations of identical
// inputs run identical launches), the parts of a group in adjacent waves.
// The parts' list lengths add up to about the group's.
constexpr int kMeasureParts = 2;  // parts per group in the cost-measuring iteration (at most the cap)

static std::vector<int4> measuring_items(const fga_state::Groups& gt, int parts) {
  std::vector<int4> v;
  v.reserve((size_t)gt.n * parts);
  for (int k = 0; k < gt.n; ++k)
    for (int r = 0; r < parts; ++r) v.push_back(make_int4(gt.host[k].x, gt.host[k].y, r | parts << 8, k));
  return v;
}

// Measures the cost of every group: one iteration with `parts` waves per group
// over the whole reference counts the list entries of each group; the state
// is restored afterwards.
static fga_status measure_groups(fga_state* S, int K, int li, fga_state::Groups& gt, int parts) {
  RigidState saved;
  FGA_HIP(hipMemcpyAsync(&saved, S->st, sizeof saved, hipMemcpyDeviceToHost, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  const std::vector<int4> ident = measuring_items(gt, parts);
  int4* wi = nullptr;
  FGA_TRY(upload_items(S, ident, &wi));
  unsigned* cost = nullptr;
  if (pool_get(&cost, sizeof(unsigned) * gt.n, S->s) != FGA_OK) {
    pool_free(wi, S->s);
    return FGA_E_NOMEM;
  }
  PairDev pd = S->pd;
  pd.nodes = S->trees[li];
  pd.n_nodes = S->tree_nodes[li];
  pd.group = K;
  pd.slots = 1;
  pd.tile = kBlock * K;
  pd.witems = wi;
  pd.n_groups = gt.n;
  pd.n_witems = (int)ident.size();
  pd.gcost = cost;
  pd.jr = parts;
  pd.n_items = (pd.n_witems + kBlock / kWave - 1) / (kBlock / kWave);
  gt.cost.assign(gt.n, 0u);
  fga_status st = FGA_OK;
  if (hipMemsetAsync(cost, 0, sizeof(unsigned) * gt.n, S->s) != hipSuccess) st = FGA_E_DEVICE;
  if (st == FGA_OK) st = launch_iteration<float>(pd, S->c, S->s);
  if (st == FGA_OK &&
      (hipMemcpyAsync(gt.cost.data(), cost, sizeof(unsigned) * gt.n, hipMemcpyDeviceToHost, S->s) != hipSuccess ||
       hipMemcpyAsync(S->st, &saved, sizeof saved, hipMemcpyHostToDevice, S->s) != hipSuccess ||
       hipStreamSynchronize(S->s) != hipSuccess))
    st = FGA_E_DEVICE;
  pool_free(cost, S->s);
  pool_free(wi, S->s);
  if (st != FGA_OK) {
    gt.cost.clear();
    if (st == FGA_E_DEVICE) set_error("group cost measurement failed");
  }
  return st;
}

// Device groups of a state for (K, tau option) on tree li, built on first use
// (the group tables do not depend on the tree; their costs do).
static fga_status ensure_groups(fga_state* S, int K, int fi, int li, fga_state::Groups** out) {
  const int key = 64 * li + K * 8 + fi;
  auto it = S->groups.find(key);
  if (it == S->groups.end()) {
    for (auto& kv : S->groups)
      if (kv.first % 64 == key % 64) {  // the same tables for another tree
        fga_state::Groups gt;
        gt.host = kv.second.host;
        gt.n = kv.second.n;
        it = S->groups.emplace(key, std::move(gt)).first;
        *out = &it->second;
        return FGA_OK;
      }
    fga_state::Groups gt;
    std::vector<std::vector<int2>> tabs;
    const int64_t zero = 0, mm = S->m;
    FGA_TRY(device_groups((const float4*)S->Q, 1, &zero, &mm, group_run(K, fi), kGroupTau[fi & 3], tabs,
                          S->s));
    gt.host = std::move(tabs[0]);
    gt.n = (int)gt.host.size();
    it = S->groups.emplace(key, std::move(gt)).first;
  }
  *out = &it->second;
  return FGA_OK;
}

// Wave items of a group table for a cap on the parts per group: a group
// whose measured cost is above the target (the larger of twice the median and
// the total over 8192 waves) is split over nr = 2, 4, ... <= cap waves by
// subtrees. Items are ordered by estimated cost, heaviest first, so that the
// expensive waves start first and the cheap ones fill in behind them.
static fga_status wave_items(fga_state* S, int K, int li, fga_state::Groups& gt, int cap,
                             const int4** dev, int* count) {
  auto it = gt.items.find(cap);
  if (it == gt.items.end()) {
    if (gt.cost.empty()) FGA_TRY(measure_groups(S, K, li, gt, std::min(kMeasureParts, cap)));
    std::vector<double> cs(gt.cost.begin(), gt.cost.end());
    double total = 0.0;
    for (double c : cs) total += c;
    std::nth_element(cs.begin(), cs.begin() + cs.size() / 2, cs.end());
    // heavy groups are split until their parts fall under `target`; with few
    // groups for the chip (under two per resident wave slot) the parts are
    // made finer, so that waves finishing early take over the remaining
    // ones instead of idling while the heaviest finish
    int dev = 0, cus = 256;
    FGA_HIP(hipGetDevice(&dev));
    FGA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const bool few = gt.n < 2 * cus * 4 * kGroupWavesPerSimd;
    const double median = cs[cs.size() / 2];
    const double target = few ? std::max(0.5 * median, total / 32768.0)
                              : std::max(2.0 * median, total / 8192.0);
    std::vector<std::pair<double, int4>> items;
    for (int g = 0; g < gt.n; ++g) {
      const int2 grp = gt.host[g];
      int nr = 1;
      while (2 * nr <= cap && gt.cost[g] > target * nr) nr *= 2;  // a power of two <= cap
      for (int r = 0; r < nr; ++r)
        items.push_back({(double)gt.cost[g] / nr, make_int4(grp.x, grp.y, r | nr << 8, g)});
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) {
                       return x.first > y.first;
                     });
    std::vector<int4> v(items.size());
    for (size_t k = 0; k < items.size(); ++k) v[k] = items[k].second;
    int4* d = nullptr;
    FGA_TRY(upload_items(S, v, &d));
    it = gt.items.emplace(cap, std::make_pair(d, (int)v.size())).first;
  }
  *dev = it->second.first;
  *count = it->second.second;
  return FGA_OK;
}

// Applies a work split (mode << 8 | ranges) to a pair's launch geometry.
// mode: lanes per particle of the per-particle walk (1, 2, 4, 8), with
// `ranges` reference ranges per tile; or 16 + K + 4 fi for the group walk with
// K particles per lane, groups bounded by kGroupTau[fi] and at most `ranges`
// reference ranges per group. With `build` false only the launch size (an
// upper bound for the group walk) is set.
static fga_status apply_split(fga_state* S, PairDev& pd, int code, bool build = true,
                              bool defer = false) {
  const int mode = (code >> 8) & 255;
  const int li = code >> 16;  // tree (leaf size) index
  if (!S->trees.empty()) {
    pd.nodes = S->trees[li];
    pd.n_nodes = S->tree_nodes[li];
  }
  pd.jr = code & 255;
  pd.witems = nullptr;
  pd.gcost = nullptr;
  pd.n_groups = 0;
  pd.n_witems = 0;
  if (mode >= 16) {
    pd.group = (mode - 16) & 3;
    pd.slots = 1;
    pd.tile = kBlock * pd.group;
    fga_state::Groups* gt = nullptr;
    FGA_TRY(ensure_groups(S, pd.group, (mode - 16) >> 2, li, &gt));
    pd.n_groups = gt->n;
    if (build && defer) {
      // a fixed split for now (every group in at most kMeasureParts parts);
      // the first iteration measures the costs (also when tuning measured
      // them already: every registration then runs the same first
      // iteration and the same splits, bit for bit)
      const std::vector<int4> ident = measuring_items(*gt, std::min(kMeasureParts, pd.jr));
      pool_free(S->ident_items, S->s);
      S->ident_items = nullptr;
      FGA_TRY(upload_items(S, ident, &S->ident_items));
      pd.witems = S->ident_items;
      pd.n_witems = (int)ident.size();
      S->pend_K = pd.group;
      S->pend_fi = (mode - 16) >> 2;
      S->pend_cap = pd.jr;
      S->pend_li = li;
    } else if (build) {
      FGA_TRY(wave_items(S, pd.group, li, *gt, pd.jr, &pd.witems, &pd.n_witems));
    } else {
      pd.n_witems = gt->n * pd.jr;  // at most `jr` parts per group
    }
    pd.n_items = (pd.n_witems + kBlock / kWave - 1) / (kBlock / kWave);
  } else {
    pd.group = 0;
    pd.slots = mode;
    pd.tile = kBlock / mode;
    pd.n_items = (int)((S->m + pd.tile - 1) / pd.tile) * pd.jr;
  }
  return FGA_OK;
}

// Times each candidate work split on the state's own kernels, restoring the
// FP64 state after every trial; `times` receives (ms, candidate), fastest
// first.
static fga_status tune_ranges(fga_state* S, const std::vector<int>& cands,
                              std::vector<std::pair<float, int>>* times) {
  RigidState saved;
  FGA_HIP(hipMemcpyAsync(&saved, S->st, sizeof saved, hipMemcpyDeviceToHost, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  hipEvent_t e0, e1;
  FGA_HIP(hipEventCreate(&e0));
  FGA_HIP(hipEventCreate(&e1));
  fga_status st = FGA_OK;
  times->clear();
  for (int c : cands) {
    PairDev pd = S->pd;
    st = apply_split(S, pd, c);
    if (st != FGA_OK) break;
    auto launch = [&]() {
      return S->f64 ? launch_iteration<double>(pd, S->c, S->s) : launch_iteration<float>(pd, S->c, S->s);
    };
    st = launch();
    if (st != FGA_OK) break;
    // the fastest of three separately timed launches: robust to a launch
    // slowed by something else on the device
    float ms = 1e30f;
    for (int r = 0; r < 3 && st == FGA_OK; ++r) {
      float one = 0.f;
      if (hipEventRecord(e0, S->s) != hipSuccess) { st = FGA_E_DEVICE; break; }
      st = launch();
      if (st != FGA_OK) break;
      if (hipEventRecord(e1, S->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&one, e0, e1) != hipSuccess) {
        st = FGA_E_DEVICE;
        break;
      }
      ms = std::min(ms, one);
    }
    if (st != FGA_OK) break;
    times->push_back({ms, c});
    if (hipMemcpyAsync(S->st, &saved, sizeof saved, hipMemcpyHostToDevice, S->s) != hipSuccess ||
        hipStreamSynchronize(S->s) != hipSuccess) {
      st = FGA_E_DEVICE;
      break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FGA_OK) set_error("autotuning the reference ranges failed");
  std::stable_sort(times->begin(), times->end(),
                   [](const std::pair<float, int>& x, const std::pair<float, int>& y) {
                     return x.first < y.first;
                   });
  return st;
}

// Autotuning of a state's work split. The cost of a split changes with the
// template's pose as the registration proceeds (the first, misaligned pose
// can rank the splits differently from the poses where most iterations are
// spent), so every candidate is timed at the initial pose, the state is then
// advanced by kTuneAdvance iterations with the fastest split, the leading
// candidates of up to kTuneFinal walks are timed again there, and the
// initial state is restored. The stop rule is off while tuning.
constexpr int kTuneAdvance = 16;
constexpr int kTuneFinal = 8;

// FGA_TUNE_LOG=1: the autotuner prints every timing round to stderr.
static void tune_log(const char* what, const std::vector<std::pair<float, int>>& times) {
  const char* v = getenv("FGA_TUNE_LOG");
  if (!v || v[0] != '1') return;
  std::fprintf(stderr, "[fga tune] %s:", what);
  for (const auto& t : times) {
    const int mode = (t.second >> 8) & 255;
    std::fprintf(stderr, " L%d/%s%d/c%d=%.3fms", t.second >> 16, mode >= 16 ? "g" : "p",
                 mode >= 16 ? mode - 16 : mode, t.second & 255, t.first);
  }
  std::fprintf(stderr, "\n");
}
constexpr int kTuneLeafLead = 3;  // splits of the first tree retimed on every other tree
static fga_status autotune(fga_state* S, const std::vector<int>& cands, int* best) {
  RigidState init;
  FGA_HIP(hipMemcpyAsync(&init, S->st, sizeof init, hipMemcpyDeviceToHost, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  RigidState open = init;
  open.tol = 0.0;
  FGA_HIP(hipMemcpyAsync(S->st, &open, sizeof open, hipMemcpyHostToDevice, S->s));
  std::vector<std::pair<float, int>> times;
  fga_status st = tune_ranges(S, cands, &times);
  if (st == FGA_OK) tune_log("initial pose", times);
  if (st == FGA_OK && S->trees.size() > 1) {
    // leaf sizes: the leading splits of the first tree (Alg. 1's singleton
    // leaves) timed again on every other tree
    std::vector<int> more;
    for (size_t li = 1; li < S->trees.size(); ++li)
      for (size_t k = 0; k < times.size() && k < (size_t)kTuneLeafLead; ++k)
        more.push_back((int)li << 16 | (times[k].second & 0xffff));
    std::vector<std::pair<float, int>> t2;
    st = tune_ranges(S, more, &t2);
    if (st == FGA_OK) tune_log("leaf sizes", t2);
    times.insert(times.end(), t2.begin(), t2.end());
    std::stable_sort(times.begin(), times.end(),
                     [](const std::pair<float, int>& x, const std::pair<float, int>& y) {
                       return x.first < y.first;
                     });
  }
  if (st == FGA_OK) {
    *best = times[0].second;
    if (times.size() > 1) {
      PairDev adv = S->pd;
      st = apply_split(S, adv, *best);
      for (int k = 0; k < kTuneAdvance && st == FGA_OK; ++k)
        st = S->f64 ? launch_iteration<double>(adv, S->c, S->s) : launch_iteration<float>(adv, S->c, S->s);
      // retimed: the fastest split of each of the kTuneFinal fastest walks
      // (traversal, tau option and tree; the part caps of one walk time
      // alike), and the three fastest splits overall. The initial pose can
      // rank the walks differently from the poses most iterations see.
      std::vector<int> lead;
      for (size_t k = 0; k < times.size() && lead.size() < (size_t)kTuneFinal; ++k) {
        const int walk = times[k].second & ~0xff;
        bool seen = false;
        for (int c : lead) seen = seen || (c & ~0xff) == walk;
        if (!seen) lead.push_back(times[k].second);
      }
      for (size_t k = 0; k < times.size() && k < 3; ++k)
        if (std::find(lead.begin(), lead.end(), times[k].second) == lead.end())
          lead.push_back(times[k].second);
      if (st == FGA_OK) st = tune_ranges(S, lead, &times);
      if (st == FGA_OK) tune_log("after the advance", times);
      if (st == FGA_OK) *best = times[0].second;
    }
  }
  if (hipMemcpyAsync(S->st, &init, sizeof init, hipMemcpyHostToDevice, S->s) != hipSuccess ||
      hipStreamSynchronize(S->s) != hipSuccess)
    st = FGA_E_DEVICE;
  return st;
}

extern "C" {

fga_status fga_default_params(fga_params* p) {
  if (!p) {
    set_error("params is NULL");
    return FGA_E_INVALID_ARG;
  }
  std::memset(p, 0, sizeof *p);
  p->G = 66.7;
  p->eps = 0.2;
  p->eta = 0.2;
  p->dt = 0.1;
  p->theta = 0.6;
  p->a = -5.0;
  p->b = 5.0;
  p->rho = 16;
  p->max_depth = 20;
  p->max_iter = 200;
  p->tol = 1e-8;
  p->damping = FGA_DAMP_FRACTION;
  p->velocity = FGA_VEL_RIGID;
  p->mass_mode = FGA_MASS_NIV;
  p->precision = FGA_PREC_FP32_KAHAN;
  p->leaf_size = 1;
  p->tile = 0;
  p->check_every = 16;
  p->group_width = 0;
  p->rbf_sigma = 0.03;
  p->rbf_weight = 100.0;
  return FGA_OK;
}

const char* fga_last_error(void) { return g_err.c_str(); }

const char* fga_version(void) { return "fga-mi355x 0.1 (gfx950)"; }

fga_status fga_group_runs(const void* Y, int64_t m, int G, double f, int32_t* runs_out, int64_t cap,
                          int64_t* n_runs, void* stream) {
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(runs_out, "runs_out"));
  FGA_TRY(check_ptr(n_runs, "n_runs"));
  FGA_TRY(check_count(m, "m"));
  if (G != 32 && G != 64 && G != 128) {
    set_error("G must be 32, 64 or 128 (got %d)", G);
    return FGA_E_INVALID_ARG;
  }
  if (!(f >= 0.0) || !std::isfinite(f)) {
    set_error("f must be finite and >= 0");
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_device_ptr(Y, "Y"));
  std::vector<int2> runs;
  FGA_TRY(device_groups_xyz((const float*)Y, m, G, f, runs, (hipStream_t)stream));
  *n_runs = (int64_t)runs.size();
  if ((int64_t)runs.size() > cap) {
    set_error("%lld runs, more than cap %lld", (long long)runs.size(), (long long)cap);
    return FGA_E_INVALID_ARG;
  }
  for (size_t k = 0; k < runs.size(); ++k) {
    runs_out[2 * k] = runs[k].x;
    runs_out[2 * k + 1] = runs[k].y;
  }
  return FGA_OK;
}

fga_status fga_kabsch(const double C[9], double R[9]) {
  FGA_TRY(check_ptr(C, "C"));
  FGA_TRY(check_ptr(R, "R"));
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(C[k])) {
      set_error("C has a non-finite entry");
      return FGA_E_NONFINITE;
    }
  if (kabsch3(C, R)) {
    set_error("rank(C) < 2: the rotation is not determined");
    return FGA_E_DEGENERATE;
  }
  return FGA_OK;
}

fga_status fga_masses(const void* pts, fga_dtype dt, int64_t n, const fga_params* p, int norm,
                      void* masses_out, void* stream) {
  FGA_TRY(check_ptr(pts, "pts"));
  FGA_TRY(check_ptr(masses_out, "masses_out"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  if (norm != 0 && norm != 1) {
    set_error("norm must be 0 (sum 1) or 1 (mean 1)");
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_device_ptr(pts, "pts"));
  FGA_TRY(check_device_ptr(masses_out, "masses_out"));
  return masses_only(pts, dt, n, nullptr, 0, *p, norm, masses_out, (hipStream_t)stream);
}

fga_status fga_masses_landmarks(const void* pts, fga_dtype dt, int64_t n, const int64_t* landmarks,
                                int n_landmarks, const fga_params* p, int norm, void* masses_out,
                                void* stream) {
  FGA_TRY(check_ptr(pts, "pts"));
  FGA_TRY(check_ptr(masses_out, "masses_out"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  FGA_TRY(check_landmarks(landmarks, n_landmarks, n, "landmarks"));
  if (norm != 0 && norm != 1) {
    set_error("norm must be 0 (sum 1) or 1 (mean 1)");
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_device_ptr(pts, "pts"));
  FGA_TRY(check_device_ptr(masses_out, "masses_out"));
  return masses_only(pts, dt, n, landmarks, n_landmarks, *p, norm, masses_out, (hipStream_t)stream);
}

fga_status fga_tree_create(const void* X, const void* mX, int64_t n, fga_dtype dt,
                           const fga_params* p, void* stream, fga_tree** out) {
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(mX, "mX"));
  FGA_TRY(check_ptr(out, "out"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(mX, "mX"));
  hipStream_t s = (hipStream_t)stream;
  fga_tree* t = new fga_tree;
  t->n = n;
  t->s = s;
  const size_t v4 = dt == FGA_F64 ? sizeof(double4) : sizeof(float4);
  if (pool_get(&t->Xs, v4 * n, s) != FGA_OK) {
    delete t;
    return FGA_E_NOMEM;
  }
  fga_status st = dt == FGA_F64 ? pack_points<double>(X, mX, n, t->Xs, s)
                                : pack_points<float>(X, mX, n, t->Xs, s);
  TreeSeg seg{0, n};
  int off[2] = {0, 0};
  if (st == FGA_OK)
    st = dt == FGA_F64
             ? build_trees<double>(1, &seg, t->Xs, n, p->leaf_size, &t->nodes, off, &t->order, t->stats, s)
             : build_trees<float>(1, &seg, t->Xs, n, p->leaf_size, &t->nodes, off, &t->order, t->stats, s);
  if (st != FGA_OK) {
    pool_free(t->Xs, s);
    delete t;
    return st;
  }
  t->n_nodes = off[1] - off[0];
  st = relayout_wide(t->nodes, t->n_nodes, 1, off, &t->wide, s);
  if (st != FGA_OK) {
    fga_tree_destroy(t);
    return st;
  }
  *out = t;
  return FGA_OK;
}

fga_status fga_tree_info(const fga_tree* t, int64_t info[4]) {
  FGA_TRY(check_ptr(t, "tree"));
  FGA_TRY(check_ptr(info, "info"));
  info[0] = t->n_nodes;
  info[1] = t->stats[1];
  info[2] = t->stats[2];
  info[3] = t->stats[0];
  return FGA_OK;
}

fga_status fga_tree_export(const fga_tree* t, float* com_mass, int32_t* ints, int32_t* order) {
  FGA_TRY(check_ptr(t, "tree"));
  std::vector<BHNode> h(t->n_nodes);
  FGA_HIP(hipMemcpy(h.data(), t->nodes, sizeof(BHNode) * t->n_nodes, hipMemcpyDeviceToHost));
  // node depth from the stored squared diagonal relative to the root's
  const double l2root = h.empty() ? 0.0 : std::fabs((double)h[0].l2);
  for (int k = 0; k < t->n_nodes; ++k) {
    if (com_mass) {
      com_mass[4 * k] = h[k].cm.x;
      com_mass[4 * k + 1] = h[k].cm.y;
      com_mass[4 * k + 2] = h[k].cm.z;
      com_mass[4 * k + 3] = h[k].cm.w;
    }
    if (ints) {
      ints[4 * k] = h[k].skip;
      ints[4 * k + 1] = h[k].first;
      ints[4 * k + 2] = h[k].last;
      int d = 0;
      const double l2k = std::fabs((double)h[k].l2);
      if (l2root > 0.0 && l2k > 0.0) d = (int)std::lround(0.5 * std::log2(l2root / l2k));
      ints[4 * k + 3] = d;
    }
  }
  if (order) FGA_HIP(hipMemcpy(order, t->order, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost));
  return FGA_OK;
}

void fga_tree_destroy(fga_tree* t) {
  if (!t) return;
  pool_free(t->nodes, t->s);
  pool_free(t->wide, t->s);
  pool_free(t->order, t->s);
  pool_free(t->Xs, t->s);
  delete t;
}

fga_status fga_forces(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                      const void* mY, fga_dtype dt, double theta, const fga_params* p,
                      void* F_out, long long* interactions, void* stream) {
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(mX, "mX"));
  FGA_TRY(check_ptr(F_out, "F_out"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(m, "m"));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  if (!(std::isfinite(theta) && theta >= 0)) {
    set_error("theta must be finite and >= 0 (got %g)", theta);
    return FGA_E_INVALID_ARG;
  }
  if (dt == FGA_F32 && p->precision == FGA_PREC_FP64) {
    set_error("FP64 precision needs FP64 data");
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_device_ptr(Y, "Y"));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(mX, "mX"));
  FGA_TRY(check_device_ptr(F_out, "F_out"));
  if (mY) FGA_TRY(check_device_ptr(mY, "mY"));
  hipStream_t s = (hipStream_t)stream;
  if (theta == 0.0) {
    fga_status st = dt == FGA_F64 ? forces_direct<double>(Y, m, X, n, mX, mY, *p, F_out, s)
                                  : forces_direct<float>(Y, m, X, n, mX, mY, *p, F_out, s);
    if (st == FGA_OK && interactions) *interactions = (long long)m * (long long)n;
    return st;
  }
  // Barnes-Hut: tree on X, template visited in Morton order
  fga_tree* tr = nullptr;
  FGA_TRY(fga_tree_create(X, mX, n, dt, p, stream, &tr));
  void* Y4 = nullptr;
  int* yorder = nullptr;
  const size_t v4 = dt == FGA_F64 ? sizeof(double4) : sizeof(float4);
  fga_status st = FGA_OK;
  if (pool_get(&Y4, v4 * m, s) != FGA_OK || pool_get(&yorder, sizeof(int) * m, s) != FGA_OK)
    st = FGA_E_NOMEM;
  if (st == FGA_OK)  // the masses slot is unused by the sort; any finite array of m values works
    st = dt == FGA_F64 ? pack_points<double>(Y, Y, m, Y4, s) : pack_points<float>(Y, Y, m, Y4, s);
  TreeSeg seg{0, m};
  if (st == FGA_OK)
    st = dt == FGA_F64 ? sort_points_morton<double>(1, &seg, Y4, m, yorder, s)
                       : sort_points_morton<float>(1, &seg, Y4, m, yorder, s);
  if (st == FGA_OK)
    st = dt == FGA_F64
             ? forces_bh_tree<double>(Y, m, yorder, tr->wide, tr->n_nodes, tr->Xs, n, theta, *p, mY, F_out, interactions, s)
             : forces_bh_tree<float>(Y, m, yorder, tr->wide, tr->n_nodes, tr->Xs, n, theta, *p, mY, F_out, interactions, s);
  pool_free(Y4, s);
  pool_free(yorder, s);
  fga_tree_destroy(tr);
  return st;
}

}  // extern "C"

// Device scratch of fga_forces_direct_noalloc: a fixed array in the library's
// code object, one copy per GPU, reached through the address that
// hipGetSymbolAddress gives on each device (the array's name is only a host
// stand-in). Every call on a GPU reuses that GPU's copy.
static __device__ __align__(256) unsigned char scratch[FGA_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per device.
fga_status scratch_for_current_device(void** out) {
  int dev = 0;
  FGA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d is beyond the %d devices this library tracks", dev, kMaxDevices);
    return FGA_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                hipGetErrorString(e));
      return FGA_E_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FGA_OK;
}
}  // namespace

extern "C" {

fga_status fga_forces_direct_noalloc(const void* Y, int64_t m, const void* X, int64_t n,
                                     const void* mX, const void* mY, fga_dtype dt,
                                     const fga_params* p, void* F_out, void* stream) {
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(mX, "mX"));
  FGA_TRY(check_ptr(F_out, "F_out"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(m, "m"));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  if (dt == FGA_F32 && p->precision == FGA_PREC_FP64) {
    set_error("FP64 precision needs FP64 data");
    return FGA_E_INVALID_ARG;
  }
  const size_t need = forces_direct_scratch(m, n, dt == FGA_F64);
  if (need > (size_t)FGA_NOALLOC_SCRATCH_BYTES) {
    set_error("m = %lld, n = %lld need %zu bytes of scratch; the static scratch holds %zu",
              (long long)m, (long long)n, need, (size_t)FGA_NOALLOC_SCRATCH_BYTES);
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_device_ptr(Y, "Y"));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(mX, "mX"));
  FGA_TRY(check_device_ptr(F_out, "F_out"));
  if (mY) FGA_TRY(check_device_ptr(mY, "mY"));
  void* buf = nullptr;
  FGA_TRY(scratch_for_current_device(&buf));
  hipStream_t s = (hipStream_t)stream;
  return dt == FGA_F64 ? forces_direct_into<double>(Y, m, X, n, mX, mY, *p, F_out, buf, s)
                       : forces_direct_into<float>(Y, m, X, n, mX, mY, *p, F_out, buf, s);
}

}  // extern "C"

extern "C" {

// Registration state of Alg. 2 (defined below); lm_X / lm_Y: landmark
// correspondences; dims = 2: planar clouds embedded at z = 0.
// A second stream of the current device, at the default priority, created on
// first use and kept until the process ends: a registration sorts its template
// on it while the reference tree is built on the caller's stream (the two
// chains are independent and launch-bound). Null if it cannot be created.
static hipStream_t side_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t s2 = nullptr;
  if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[dev] = s2;
  return s2;
}

// Work of one registration set-up split over the caller's stream and the side
// stream: constructing a Fork makes the side stream wait for what the
// caller's stream has queued, join() makes the caller's stream wait for what
// the side stream has queued since. Without a side stream (or if an event
// call fails) side() is the caller's stream and everything runs there.
struct Fork {
  hipStream_t s, s2 = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  explicit Fork(hipStream_t st) : s(st) {
    hipStream_t side = side_stream();
    if (!side || hipEventCreateWithFlags(&e0, hipEventDisableTiming) != hipSuccess) return;
    if (hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(e0, s) != hipSuccess || hipStreamWaitEvent(side, e0, 0) != hipSuccess)
      return;
    s2 = side;
  }
  hipStream_t side() const { return s2 ? s2 : s; }
  void join() {
    if (s2) {
      // if the record fails, wait for the whole side stream instead
      if (hipEventRecord(e1, s2) != hipSuccess || hipStreamWaitEvent(s, e1, 0) != hipSuccess)
        (void)hipStreamSynchronize(s2);
      s2 = nullptr;
    }
  }
  ~Fork() {
    join();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

static fga_status state_create(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                               const fga_params* p, void* stream, bool defer, fga_state** out,
                               const int64_t* lm_X = nullptr, const int64_t* lm_Y = nullptr,
                               int n_lm = 0, int dims = 3);

fga_status fga_energy(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                      const void* mY, fga_dtype dt, double theta, const fga_params* p, double* E,
                      long long* interactions, void* stream) {
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(mX, "mX"));
  FGA_TRY(check_ptr(E, "E"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(m, "m"));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  if (!(std::isfinite(theta) && theta >= 0)) {
    set_error("theta must be finite and >= 0 (got %g)", theta);
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_device_ptr(Y, "Y"));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(mX, "mX"));
  if (mY) FGA_TRY(check_device_ptr(mY, "mY"));
  hipStream_t s = (hipStream_t)stream;
  const bool f64 = dt == FGA_F64;
  if (theta == 0.0) {
    fga_status st = f64 ? energy_direct<double>(Y, m, X, n, mX, mY, *p, E, s)
                        : energy_direct<float>(Y, m, X, n, mX, mY, *p, E, s);
    if (st == FGA_OK && interactions) *interactions = (long long)m * (long long)n;
    return st;
  }
  fga_tree* tr = nullptr;
  FGA_TRY(fga_tree_create(X, mX, n, dt, p, stream, &tr));
  void* Y4 = nullptr;
  int* yorder = nullptr;
  const size_t v4 = f64 ? sizeof(double4) : sizeof(float4);
  fga_status st = FGA_OK;
  if (pool_get(&Y4, v4 * m, s) != FGA_OK || pool_get(&yorder, sizeof(int) * m, s) != FGA_OK)
    st = FGA_E_NOMEM;
  if (st == FGA_OK)
    st = f64 ? pack_points<double>(Y, Y, m, Y4, s) : pack_points<float>(Y, Y, m, Y4, s);
  TreeSeg seg{0, m};
  if (st == FGA_OK)
    st = f64 ? sort_points_morton<double>(1, &seg, Y4, m, yorder, s)
             : sort_points_morton<float>(1, &seg, Y4, m, yorder, s);
  if (st == FGA_OK)
    st = f64 ? energy_bh_tree<double>(Y, m, yorder, tr->wide, tr->Xs, theta, *p, mY, E, interactions, s)
             : energy_bh_tree<float>(Y, m, yorder, tr->wide, tr->Xs, theta, *p, mY, E, interactions, s);
  pool_free(Y4, s);
  pool_free(yorder, s);
  fga_tree_destroy(tr);
  return st;
}

// Planar input: n x 2 points copied to n x 3 with z = 0 in pool memory.
static fga_status planar_copy(const void* P, int64_t n, fga_dtype dt, hipStream_t s, void** out) {
  const size_t es = dt == FGA_F64 ? 8 : 4;
  FGA_TRY(pool_get(out, es * 3 * (size_t)n, s));
  fga_status st = embed_planar(P, n, dt == FGA_F64, *out, s);
  if (st != FGA_OK) {
    pool_free(*out, s);
    *out = nullptr;
  }
  return st;
}

fga_status fga_forces_2d(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                         const void* mY, fga_dtype dt, double theta, const fga_params* p,
                         void* F_out, long long* interactions, void* stream) {
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(F_out, "F_out"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(m, "m"));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_params(p));
  FGA_TRY(check_device_ptr(Y, "Y"));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(F_out, "F_out"));
  hipStream_t s = (hipStream_t)stream;
  void *Y3 = nullptr, *X3 = nullptr, *F3 = nullptr;
  fga_status st = planar_copy(Y, m, dt, s, &Y3);
  if (st == FGA_OK) st = planar_copy(X, n, dt, s, &X3);
  if (st == FGA_OK && pool_get(&F3, (dt == FGA_F64 ? 8 : 4) * 3 * (size_t)m, s) != FGA_OK) st = FGA_E_NOMEM;
  if (st == FGA_OK) st = fga_forces(Y3, m, X3, n, mX, mY, dt, theta, p, F3, interactions, stream);
  if (st == FGA_OK) st = take_planar(F3, m, dt == FGA_F64, F_out, s);
  if (st == FGA_OK && hipStreamSynchronize(s) != hipSuccess) st = FGA_E_DEVICE;
  pool_free(Y3, s);
  pool_free(X3, s);
  pool_free(F3, s);
  return st;
}

fga_status fga_register_2d(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                           const fga_params* p, double R[4], double t[2], fga_report* rep,
                           void* stream) {
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(R, "R"));
  FGA_TRY(check_ptr(t, "t"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_count(m, "m"));
  FGA_TRY(check_params(p));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(Y, "Y"));
  const double t0 = now_ms();
  hipStream_t s = (hipStream_t)stream;
  void *X3 = nullptr, *Y3 = nullptr;
  fga_status st = planar_copy(X, n, dt, s, &X3);
  if (st == FGA_OK) st = planar_copy(Y, m, dt, s, &Y3);
  fga_state* S = nullptr;
  if (st == FGA_OK) st = state_create(X3, n, Y3, m, dt, p, stream, true, &S, nullptr, nullptr, 0, 2);
  pool_free(X3, s);
  pool_free(Y3, s);
  double R3[9], t3[3];
  if (st == FGA_OK) st = fga_step(S, p->max_iter);
  if (st == FGA_OK) st = fga_state_get(S, R3, t3, rep);
  if (S) fga_state_destroy(S);
  if (st == FGA_OK) {
    R[0] = R3[0];
    R[1] = R3[1];
    R[2] = R3[3];
    R[3] = R3[4];
    t[0] = t3[0];
    t[1] = t3[1];
  }
  if (rep) rep->ms_total = now_ms() - t0;
  return st;
}

static fga_status validate_pair(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                                const fga_params* p) {
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_dtype(dt));
  FGA_TRY(check_count(n, "n"));
  FGA_TRY(check_count(m, "m"));
  FGA_TRY(check_params(p));
  return FGA_OK;
}

static fga_status state_create(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                               const fga_params* p, void* stream, bool defer, fga_state** out,
                               const int64_t* lm_X, const int64_t* lm_Y, int n_lm, int dims) {
  FGA_TRY(validate_pair(X, n, Y, m, dt, p));
  FGA_TRY(check_ptr(out, "out"));
  FGA_TRY(check_landmarks(lm_X, n_lm, n, "lm_X"));
  FGA_TRY(check_landmarks(lm_Y, n_lm, m, "lm_Y"));
  FGA_TRY(check_device_ptr(X, "X"));
  FGA_TRY(check_device_ptr(Y, "Y"));
  hipStream_t s = (hipStream_t)stream;
  fga_state* S = new fga_state;
  S->p = *p;
  S->dt = dt;
  S->s = s;
  S->f64 = p->precision == FGA_PREC_FP64;
  S->n = n;
  S->m = m;
  const size_t v4 = S->f64 ? sizeof(double4) : sizeof(float4);
  auto fail = [&](fga_status st) {
    state_free(S);
    return st;
  };
  if (pool_get(&S->X, v4 * n, s) != FGA_OK || pool_get(&S->Q, v4 * m, s) != FGA_OK ||
      pool_get(&S->st, sizeof(RigidState), s) != FGA_OK) {
    return fail(FGA_E_NOMEM);
  }
  CloudIn cx{X, n, lm_X, n_lm}, cy{Y, m, lm_Y, n_lm};
  PrepOut po{S->X, S->Q, S->st};
  fga_params pp = *p;
  fga_status st = prep_pairs(1, &cx, &cy, dt, pp, &po, &S->norm, s, dims);
  if (st != FGA_OK) return fail(st);
  // the template's Morton sort on the side stream, beside the tree builds
  // below; joined before anything reads the sorted template
  Fork fork(s);
  TreeSeg sy{0, m};
  st = S->f64 ? sort_points_morton<double>(1, &sy, S->Q, m, nullptr, fork.side())
              : sort_points_morton<float>(1, &sy, S->Q, m, nullptr, fork.side());
  if (st != FGA_OK) {
    fork.join();
    return fail(st);
  }
  const bool bh = p->theta > 0;
  // leaf sizes: the given one, or (leaf_size 0, FP32) every option for the
  // autotuner; FP64 keeps Alg. 1's singleton leaves
  const bool leaf_auto = bh && p->leaf_size == 0 && !S->f64;
  if (bh) {
    if (leaf_auto) S->tree_leaf.assign(kLeafOpts, kLeafOpts + kNumLeafOpts);
    else S->tree_leaf.assign(1, p->leaf_size > 0 ? p->leaf_size : 1);
    S->trees.assign(S->tree_leaf.size(), nullptr);
    S->tree_nodes.assign(S->tree_leaf.size(), 0);
  }
  // builds tree li (leaf size tree_leaf[li]) on the Morton-sorted reference
  auto build_tree = [&](size_t li) -> fga_status {
    TreeSeg sx{0, n};
    int off[2] = {0, 0};
    BHNode* pre = nullptr;
    const int L = S->tree_leaf[li];
    fga_status bs = S->f64 ? build_trees<double>(1, &sx, S->X, n, L, &pre, off, nullptr, S->tree_stats, s)
                           : build_trees<float>(1, &sx, S->X, n, L, &pre, off, nullptr, S->tree_stats, s);
    if (bs != FGA_OK) return bs;
    S->tree_nodes[li] = off[1] - off[0];
    bs = relayout_wide(pre, S->tree_nodes[li], 1, off, &S->trees[li], s);
    pool_free(pre, s);
    return bs;
  };
  // candidate work splits, encoded mode << 8 | reference ranges; mode is the
  // number of lanes per particle (1, 2, 4, 8) of the per-particle walk, or
  // 16 + K for the group walk with K particles per lane
  std::vector<int> modes;
  if (!bh || S->f64) {
    modes.push_back(1);
  } else {
    const int gw = p->group_width;
    if (gw == 0 || gw == 1)
      for (int sl = 1; sl <= (p->precision == FGA_PREC_FP32_KAHAN ? 8 : 1); sl *= 2)
        modes.push_back(sl);
    for (int fi = 0; fi < 4; ++fi) {
      if (gw == 0 || gw == 64) modes.push_back(16 + 1 + 4 * fi);
      if (gw == 0 || gw == 128) modes.push_back(16 + 2 + 4 * fi);
      // runs of 32: on request, and for planar sets, where a run's box is
      // wider for its particle count and the 32-runs timed fastest (13% on
      // the planar mixture); on the LiDAR and mesh workloads every one of
      // them timed slower than the runs of 64 (the walks double)
      if (gw == 32 || (gw == 0 && dims == 2)) modes.push_back(16 + 1 + 4 * (fi + 4));
    }
  }
  std::vector<int> cands;
  for (int md : modes) {
    const int64_t tp = md < 16 ? kBlock / md
                       : ((md - 16) >> 2) >= 4 ? kBlock / 2  // runs of 32 particles
                                               : (int64_t)kBlock * ((md - 16) & 3);
    const int64_t tl = (m + tp - 1) / tp;
    if (p->velocity == FGA_VEL_PARTICLE) {
      cands.push_back(md << 8 | 1);
    } else if (p->tile > 0) {
      cands.push_back(md << 8 | p->tile);
    } else {
      for (int c = 1; c <= (bh ? 16 : 64); c *= 2) {
        const int64_t per = n / c;
        if ((c == 1 || (per >= (bh ? 256 : 64) && tl * c <= 65536)) && tl * c <= 262144)
          cands.push_back(md << 8 | c);
      }
    }
  }
  if (!bh && p->tile == 0 && p->velocity != FGA_VEL_PARTICLE) {
    // the direct sum starts from its occupancy rule; the tuner may improve on it
    const int jd = direct_ranges(m, n);
    if (std::find(cands.begin(), cands.end(), 1 << 8 | jd) == cands.end()) cands.push_back(1 << 8 | jd);
  }
  // a cached tuning result needs only its own split; otherwise every
  // candidate is timed
  const std::string key = tune_key(bh, S->f64, m, n, p->precision, p->group_width) +
                          (bh ? "_t" + std::to_string(std::lround(p->theta * 1000)) + "_L" +
                                    std::to_string(leaf_auto ? 0 : S->tree_leaf[0])
                              : "") +
                          (dims == 2 ? "_D2" : "");
  int best = cands[0];
  bool tuned = cands.size() == 1;
  if (!tuned) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    // the cached split names its tree (leaf size) in the bits above 16; the
    // candidates are listed for the first tree
    if (it != g_tune.end() && (it->second >> 16) < (int)std::max<size_t>(1, S->trees.size()) &&
        std::find(cands.begin(), cands.end(), it->second & 0xffff) != cands.end()) {
      best = it->second;
      tuned = true;
    }
  }
  // the trees: all of them when they are to be tuned, else only the chosen one
  for (size_t li = 0; li < S->trees.size(); ++li)
    if (!tuned || (int)li == (best >> 16))
      if (fga_status bs = build_tree(li); bs != FGA_OK) {
        fork.join();
        return fail(bs);
      }
  fork.join();
  const std::vector<int> used = tuned ? std::vector<int>{best} : cands;
  size_t max_items = 0;
  for (int c : used) {
    PairDev tmp{};
    const fga_status gs = apply_split(S, tmp, c, false);
    if (gs != FGA_OK) return fail(gs);
    max_items = std::max(max_items, (size_t)tmp.n_items);
  }
  const size_t max_chunks = (size_t)completion_chunks((int)max_items);
  if (pool_get(&S->partial, sizeof(double) * kPartialRow * (max_items + max_chunks), s) != FGA_OK ||
      pool_get(&S->done, sizeof(unsigned) * (1 + max_chunks), s) != FGA_OK) {
    return fail(FGA_E_NOMEM);
  }
  if (hipMemsetAsync(S->done, 0, sizeof(unsigned) * (1 + max_chunks), s) != hipSuccess)
    return fail(FGA_E_DEVICE);
  if (p->velocity == FGA_VEL_PARTICLE) {
    const size_t vb = (S->f64 ? 8 : 4) * 3 * (size_t)m;
    if (pool_get(&S->V, vb, s) != FGA_OK) {
      return fail(FGA_E_NOMEM);
    }
    if (hipMemsetAsync(S->V, 0, vb, s) != hipSuccess) return fail(FGA_E_DEVICE);
  }
  PairDev& pd = S->pd;
  pd.X = S->X;
  pd.Q = S->Q;
  pd.nodes = S->nodes;
  pd.V = S->V;
  pd.st = S->st;
  pd.partial = S->partial;
  pd.done = S->done;
  pd.n = (int)n;
  pd.m = (int)m;
  pd.n_nodes = S->n_nodes;
  pd.planar = dims == 2 ? 1 : 0;
  S->c = make_iter_consts(*p);
  // manual stepping has no iteration cap; fga_register applies max_iter itself
  const int big = 0x7fffffff;
  if (hipMemcpyAsync(&S->st->max_iter, &big, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("state initialisation failed");
    return fail(FGA_E_DEVICE);
  }
  if (!tuned) {
    if (fga_status gs = apply_split(S, pd, cands[0]); gs != FGA_OK) return fail(gs);
    fga_status tst = autotune(S, cands, &best);
    if (tst != FGA_OK) return fail(tst);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    tune_save_locked();
  }
  if (bh) {  // the chosen tree stays; the others are released
    const size_t lb = (size_t)(best >> 16);
    for (size_t li = 0; li < S->trees.size(); ++li)
      if (li != lb && S->trees[li]) {
        pool_free(S->trees[li], s);
        S->trees[li] = nullptr;
      }
    S->nodes = S->trees[lb];
    S->n_nodes = S->tree_nodes[lb];
    S->leaf_used = S->tree_leaf[lb];
    pd.nodes = S->nodes;
    pd.n_nodes = S->n_nodes;
  }
  if (fga_status gs = apply_split(S, pd, best, true, defer); gs != FGA_OK) return fail(gs);
  S->run = pd.group ? group_run(pd.group, ((best >> 8) & 255) >= 16 ? (((best >> 8) & 255) - 16) >> 2 : 0) : 0;
  if (S->V) {  // trial iterations wrote per-particle velocities; the state starts at rest
    const size_t vb = (S->f64 ? 8 : 4) * 3 * (size_t)m;
    if (hipMemsetAsync(S->V, 0, vb, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return fail(FGA_E_DEVICE);
  }
  *out = S;
  return FGA_OK;
}

fga_status fga_state_create(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                            const fga_params* p, void* stream, fga_state** out) {
  return state_create(X, n, Y, m, dt, p, stream, false, out);
}

fga_status fga_state_create_landmarks(const void* X, int64_t n, const void* Y, int64_t m,
                                      fga_dtype dt, const int64_t* lm_X, const int64_t* lm_Y,
                                      int n_landmarks, const fga_params* p, void* stream,
                                      fga_state** out) {
  return state_create(X, n, Y, m, dt, p, stream, false, out, lm_X, lm_Y, n_landmarks);
}

// The first iteration of a deferred group split: the fixed measuring split
// counts every group's list entries while it iterates; the balanced wave
// items are then built from those costs.
static fga_status first_step_measured(fga_state* S) {
  fga_state::Groups* gt = nullptr;
  FGA_TRY(ensure_groups(S, S->pend_K, S->pend_fi, S->pend_li, &gt));
  unsigned* cost = nullptr;
  FGA_TRY(pool_get(&cost, sizeof(unsigned) * gt->n, S->s));
  PairDev pd = S->pd;
  pd.gcost = cost;
  gt->cost.assign(gt->n, 0u);
  fga_status st = FGA_OK;
  if (hipMemsetAsync(cost, 0, sizeof(unsigned) * gt->n, S->s) != hipSuccess) st = FGA_E_DEVICE;
  if (st == FGA_OK) st = launch_iteration<float>(pd, S->c, S->s);
  if (st == FGA_OK &&
      (hipMemcpyAsync(gt->cost.data(), cost, sizeof(unsigned) * gt->n, hipMemcpyDeviceToHost, S->s) != hipSuccess ||
       hipStreamSynchronize(S->s) != hipSuccess))
    st = FGA_E_DEVICE;
  pool_free(cost, S->s);
  if (st != FGA_OK) {
    gt->cost.clear();
    if (st == FGA_E_DEVICE) set_error("first iteration with cost measurement failed");
    return st;
  }
  for (auto& kv : gt->items) pool_free(kv.second.first, S->s);  // built from older costs
  gt->items.clear();
  FGA_TRY(wave_items(S, S->pend_K, S->pend_li, *gt, S->pend_cap, &S->pd.witems, &S->pd.n_witems));
  S->pd.n_items = (S->pd.n_witems + kBlock / kWave - 1) / (kBlock / kWave);
  S->pend_K = 0;
  return FGA_OK;
}

static fga_status read_state(const fga_state* S, RigidState* h) {
  FGA_HIP(hipMemcpyAsync(h, S->st, sizeof(RigidState), hipMemcpyDeviceToHost, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  return FGA_OK;
}

fga_status fga_step(fga_state* S, int n_iters) {
  FGA_TRY(check_ptr(S, "state"));
  if (n_iters < 0) {
    set_error("n_iters must be >= 0");
    return FGA_E_INVALID_ARG;
  }
  const int every = S->p.check_every > 0 ? S->p.check_every : 16;
  int k0 = 0;
  if (S->pend_K && n_iters > 0) {
    FGA_TRY(first_step_measured(S));
    k0 = 1;
  }
  for (int k = k0; k < n_iters; ++k) {
    fga_status st = S->f64 ? launch_iteration<double>(S->pd, S->c, S->s)
                           : launch_iteration<float>(S->pd, S->c, S->s);
    if (st != FGA_OK) return st;
    if (S->p.tol > 0 && ((k + 1) % every == 0) && k + 1 < n_iters) {
      int conv = 0;
      FGA_HIP(hipMemcpyAsync(&conv, &S->st->converged, sizeof(int), hipMemcpyDeviceToHost, S->s));
      FGA_HIP(hipStreamSynchronize(S->s));
      if (conv) break;
    }
  }
  FGA_HIP(hipStreamSynchronize(S->s));
  return FGA_OK;
}

fga_status fga_step_profile(fga_state* S, int n_iters, double ms[2]) {
  FGA_TRY(check_ptr(S, "state"));
  FGA_TRY(check_ptr(ms, "ms"));
  if (n_iters < 1) {
    set_error("n_iters must be >= 1");
    return FGA_E_INVALID_ARG;
  }
  if (S->pend_K) FGA_TRY(first_step_measured(S));  // the measuring launch is not timed
  // three events per iteration: before the force launch, between the two
  // launches, after the reduction launch; all queued before one wait, so the
  // host never idles the stream between iterations
  std::vector<hipEvent_t> ev((size_t)3 * n_iters, nullptr);
  fga_status st = FGA_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      st = FGA_E_DEVICE;
      break;
    }
  for (int k = 0; k < n_iters && st == FGA_OK; ++k) {
    if (hipEventRecord(ev[3 * k], S->s) != hipSuccess) st = FGA_E_DEVICE;
    if (st == FGA_OK)
      st = S->f64 ? launch_iteration<double>(S->pd, S->c, S->s, ev[3 * k + 1])
                  : launch_iteration<float>(S->pd, S->c, S->s, ev[3 * k + 1]);
    if (st == FGA_OK && hipEventRecord(ev[3 * k + 2], S->s) != hipSuccess) st = FGA_E_DEVICE;
  }
  if (st == FGA_OK && hipStreamSynchronize(S->s) != hipSuccess) st = FGA_E_DEVICE;
  ms[0] = ms[1] = 0.0;
  for (int k = 0; k < n_iters && st == FGA_OK; ++k) {
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]) != hipSuccess ||
        hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]) != hipSuccess)
      st = FGA_E_DEVICE;
    ms[0] += a;
    ms[1] += b;
  }
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st == FGA_E_DEVICE) set_error("profiled iterations failed");
  return st;
}

fga_status fga_state_get_normalised(const fga_state* S, double R[9], double t[3]) {
  FGA_TRY(check_ptr(S, "state"));
  FGA_TRY(check_ptr(R, "R"));
  FGA_TRY(check_ptr(t, "t"));
  RigidState h;
  FGA_TRY(read_state(S, &h));
  std::memcpy(R, h.R, sizeof(double) * 9);
  std::memcpy(t, h.t, sizeof(double) * 3);
  return FGA_OK;
}

fga_status fga_state_get(const fga_state* S, double R[9], double t[3], fga_report* rep) {
  FGA_TRY(check_ptr(S, "state"));
  FGA_TRY(check_ptr(R, "R"));
  FGA_TRY(check_ptr(t, "t"));
  RigidState h;
  FGA_TRY(read_state(S, &h));
  std::memcpy(R, h.R, sizeof(double) * 9);
  denormalise(S->norm, h.R, h.t, t);
  if (rep) {
    rep->iters = h.iter;
    rep->converged = h.converged == 1;
    rep->last_dT2 = h.dT2;
    rep->interactions = h.interactions;
    rep->ms_total = 0.0;
    rep->traversal = !S->nodes ? 0 : S->pd.group ? S->run : 1;
    rep->leaf_size = S->leaf_used;
  }
  if (h.flags & 2) {
    set_error("Barnes-Hut group walk: traversal stack overflow (forces incomplete)");
    return FGA_E_DEVICE;
  }
  if (h.flags & 1) {
    set_error("the template is collinear: the Kabsch rotation is undetermined");
    return FGA_E_DEGENERATE;
  }
  return FGA_OK;
}

fga_status fga_state_save(const fga_state* S, void* buf, size_t* len) {
  FGA_TRY(check_ptr(S, "state"));
  FGA_TRY(check_ptr(len, "len"));
  const size_t vb = S->V ? (S->f64 ? 8 : 4) * 3 * (size_t)S->m : 0;
  const size_t need = sizeof(RigidState) + vb;
  if (!buf) {
    *len = need;
    return FGA_OK;
  }
  if (*len < need) {
    set_error("buffer too small: %zu < %zu bytes", *len, need);
    return FGA_E_INVALID_ARG;
  }
  FGA_HIP(hipMemcpyAsync(buf, S->st, sizeof(RigidState), hipMemcpyDeviceToHost, S->s));
  if (vb) FGA_HIP(hipMemcpyAsync((char*)buf + sizeof(RigidState), S->V, vb, hipMemcpyDeviceToHost, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  *len = need;
  return FGA_OK;
}

fga_status fga_state_load(fga_state* S, const void* buf, size_t len) {
  FGA_TRY(check_ptr(S, "state"));
  FGA_TRY(check_ptr(buf, "buf"));
  const size_t vb = S->V ? (S->f64 ? 8 : 4) * 3 * (size_t)S->m : 0;
  if (len != sizeof(RigidState) + vb) {
    set_error("saved state has %zu bytes, this state needs %zu", len, sizeof(RigidState) + vb);
    return FGA_E_INVALID_ARG;
  }
  RigidState h;
  std::memcpy(&h, buf, sizeof h);
  if (h.m != (int)S->m) {
    set_error("saved state is for %d template points, this state has %lld", h.m, (long long)S->m);
    return FGA_E_INVALID_ARG;
  }
  FGA_HIP(hipMemcpyAsync(S->st, buf, sizeof(RigidState), hipMemcpyHostToDevice, S->s));
  if (vb) FGA_HIP(hipMemcpyAsync(S->V, (const char*)buf + sizeof(RigidState), vb, hipMemcpyHostToDevice, S->s));
  FGA_HIP(hipStreamSynchronize(S->s));
  return FGA_OK;
}

void fga_state_destroy(fga_state* S) { state_free(S); }

fga_status fga_register(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                        const fga_params* p, double R[9], double t[3], fga_report* rep,
                        void* stream) {
  FGA_TRY(validate_pair(X, n, Y, m, dt, p));
  FGA_TRY(check_ptr(R, "R"));
  FGA_TRY(check_ptr(t, "t"));
  const double t0 = now_ms();
  fga_state* S = nullptr;
  FGA_TRY(state_create(X, n, Y, m, dt, p, stream, true, &S));
  fga_status st = fga_step(S, p->max_iter);
  if (st == FGA_OK) st = fga_state_get(S, R, t, rep);
  fga_state_destroy(S);
  if (rep) rep->ms_total = now_ms() - t0;
  return st;
}

fga_status fga_register_landmarks(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                                  const int64_t* lm_X, const int64_t* lm_Y, int n_landmarks,
                                  const fga_params* p, double R[9], double t[3], fga_report* rep,
                                  void* stream) {
  FGA_TRY(validate_pair(X, n, Y, m, dt, p));
  FGA_TRY(check_ptr(R, "R"));
  FGA_TRY(check_ptr(t, "t"));
  const double t0 = now_ms();
  fga_state* S = nullptr;
  FGA_TRY(state_create(X, n, Y, m, dt, p, stream, true, &S, lm_X, lm_Y, n_landmarks));
  fga_status st = fga_step(S, p->max_iter);
  if (st == FGA_OK) st = fga_state_get(S, R, t, rep);
  fga_state_destroy(S);
  if (rep) rep->ms_total = now_ms() - t0;
  return st;
}

}  // extern "C"

namespace {

struct BatchBufs {
  std::vector<void*> ptrs;
  hipStream_t own = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipEvent_t ev = nullptr;
  int tuned_fi = 0, tuned_cap = 0;  // the group walk's tau option and part cap in use
  int tuned_leaf = 0;               // leaf size of the trees in use
  ~BatchBufs() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own) (void)hipStreamSynchronize(own);
    for (void* q : ptrs) pool_free(q, own);  // the stream has drained: reusable at once
    if (own) (void)hipStreamDestroy(own);
    if (ev) (void)hipEventDestroy(ev);
  }
  template <typename P>
  fga_status get(P** out, size_t bytes) {
    void* q = pool_alloc(bytes < 16 ? 16 : bytes, own);
    if (!q) return FGA_E_NOMEM;
    ptrs.push_back(q);
    *out = (P*)q;
    return FGA_OK;
  }
};

template <typename T>
fga_status batch_impl(int npairs, const void* const* X, const int64_t* n, const void* const* Y,
                      const int64_t* m, fga_dtype dt, const fga_params& p, double* R, double* t,
                      fga_report* reps, hipStream_t caller) {
  const double t0 = now_ms();
  BatchBufs B;
  // private non-default stream: graph capture needs one; ordered after the caller's work
  FGA_HIP(hipStreamCreateWithFlags(&B.own, hipStreamNonBlocking));
  FGA_HIP(hipEventCreateWithFlags(&B.ev, hipEventDisableTiming));
  FGA_HIP(hipEventRecord(B.ev, caller));
  FGA_HIP(hipStreamWaitEvent(B.own, B.ev, 0));
  hipStream_t s = B.own;
  std::vector<int64_t> xoff(npairs + 1, 0), yoff(npairs + 1, 0);
  for (int k = 0; k < npairs; ++k) {
    xoff[k + 1] = xoff[k] + n[k];
    yoff[k + 1] = yoff[k] + m[k];
  }
  const int64_t NX = xoff[npairs], NY = yoff[npairs];
  if (NX > kMaxPoints || NY > kMaxPoints) {
    set_error("batch too large: %lld reference and %lld template points", (long long)NX, (long long)NY);
    return FGA_E_INVALID_ARG;
  }
  vec4_t<T>*Xp, *Qp;
  RigidState* st;
  FGA_TRY(B.get(&Xp, sizeof(vec4_t<T>) * NX));
  FGA_TRY(B.get(&Qp, sizeof(vec4_t<T>) * NY));
  FGA_TRY(B.get(&st, sizeof(RigidState) * npairs));
  std::vector<CloudIn> cx(npairs), cy(npairs);
  for (int k = 0; k < npairs; ++k) {
    cx[k] = {X[k], n[k]};
    cy[k] = {Y[k], m[k]};
  }
  std::vector<NormInfo> norm(npairs);
  PrepOut po{Xp, Qp, st};
  FGA_TRY(prep_pairs(npairs, cx.data(), cy.data(), dt, p, &po, norm.data(), s));
  std::vector<TreeSeg> ys(npairs), xs(npairs);
  for (int k = 0; k < npairs; ++k) {
    ys[k] = {yoff[k], m[k]};
    xs[k] = {xoff[k], n[k]};
  }
  FGA_TRY(sort_points_morton<T>(npairs, ys.data(), Qp, NY, nullptr, s));
  const bool grouped = sizeof(T) == 4 && p.theta > 0 && p.group_width != 1;
  // the trees of all pairs for one leaf size (one set of launches)
  struct TreeSet {
    int leaf;
    BHWide* nodes;
    std::vector<int> off;
  };
  std::vector<TreeSet> tsets;
  auto build_set = [&](int L) -> fga_status {
    TreeSet ts{L, nullptr, std::vector<int>(npairs + 1, 0)};
    BHNode* pre = nullptr;
    int tstats[3];
    FGA_TRY(build_trees<T>(npairs, xs.data(), Xp, NX, L, &pre, ts.off.data(), nullptr, tstats, s));
    B.ptrs.push_back(pre);
    FGA_TRY(relayout_wide(pre, ts.off[npairs], npairs, ts.off.data(), &ts.nodes, s));
    B.ptrs.push_back(ts.nodes);
    tsets.push_back(std::move(ts));
    return FGA_OK;
  };
  if (p.theta > 0) FGA_TRY(build_set(p.leaf_size > 0 ? p.leaf_size : 1));
  BHWide* nodes = p.theta > 0 ? tsets[0].nodes : nullptr;
  std::vector<int> noff = p.theta > 0 ? tsets[0].off : std::vector<int>(npairs + 1, 0);
  int dev = 0, cus = 256;
  FGA_HIP(hipGetDevice(&dev));
  FGA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const IterConsts c = make_iter_consts(p);
  // the group walk (FP32 Barnes-Hut unless group_width = 1) with one particle
  // per lane: groups of consecutive template particles bounded by
  // kGroupTau[fi] times the median box of fixed 64-runs, heavy groups split
  // into at most `cap` parts by their measured cost. (fi, cap) are tuned on
  // the batch itself (tile = 0) and cached for batches of the same shape
  // class, or fixed by the caller (tile > 0: cap = the largest power of two
  // <= tile, fi = 2).
  std::vector<PairDev> pds(npairs);
  const int kCap = 16;  // most parts per group (capacity of the wave-item arrays)
  std::vector<int> fis{2}, caps{16};
  std::vector<int> leaves{p.leaf_size > 0 ? p.leaf_size : 1};
  std::string bkey;
  bool btuned = true;
  if (grouped) {
    if (p.tile > 0) {
      int cap = 1;
      while (2 * cap <= std::min(p.tile, kCap)) cap *= 2;
      caps = {cap};
    } else {
      auto lg = [](int64_t v) {
        int q = 0;
        while ((int64_t(1) << (q + 1)) <= v) ++q;
        return q;
      };
      char buf[96];
      snprintf(buf, sizeof buf, "batch_p%d_k%d_m%d_n%d_t%d_L%d", p.precision, lg(npairs), lg(NY),
               lg(NX), (int)std::lround(p.theta * 1000), p.leaf_size);
      bkey = buf;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_load_locked();
      auto it = g_tune.find(bkey);
      if (it != g_tune.end()) {
        fis = {(it->second >> 8) & 255};
        caps = {it->second & 255};
        leaves = {it->second >> 16};
      } else {
        fis = {1, 2, 3};
        caps = {4, 16};
        if (p.leaf_size == 0) leaves = {1, 4, 8};
        btuned = false;
      }
    }
  }
  // group tables of every candidate tau option (built on the device), and
  // their offsets
  std::map<int, std::vector<std::vector<int2>>> gtab;
  std::map<int, std::vector<int>> gofs;
  int max_groups = 0;
  for (int fi : fis) {
    if (!grouped) break;
    auto& g = gtab[fi];
    auto& go = gofs[fi];
    go.assign(npairs + 1, 0);
    FGA_TRY(device_groups((const float4*)Qp, npairs, yoff.data(), m, kWave, kGroupTau[fi], g, s));
    for (int k = 0; k < npairs; ++k) go[k + 1] = go[k] + (int)g[k].size();
    max_groups = std::max(max_groups, go[npairs]);
  }
  std::vector<int> item_off(npairs + 1, 0);
  for (int k = 0; k < npairs; ++k) {
    if (grouped) {
      // capacity for up to kCap wave items per group (the most groups of any candidate)
      int ng = 0;
      for (int fi : fis) ng = std::max(ng, (int)gtab[fi][k].size());
      const int nwi = ng * kCap;
      pds[k].n_items = (nwi + kBlock / kWave - 1) / (kBlock / kWave);
      pds[k].jr = 1;
      pds[k].tile = kBlock;
      pds[k].slots = 1;
      pds[k].group = 1;
    } else {
      const bool big = NY >= 262144;
      int jr = big ? 1 : (p.theta > 0 ? bh_ranges(m[k], n[k]) : direct_ranges(m[k], n[k]));
      const int tiles = (int)((m[k] + kBlock - 1) / kBlock);
      pds[k].jr = jr;
      pds[k].n_items = tiles * jr;
      pds[k].tile = kBlock;
      pds[k].slots = 1;
      pds[k].group = 0;
    }
    item_off[k + 1] = item_off[k] + pds[k].n_items;
  }
  // per pair: items + chunks partial rows, 1 + chunks completion counters
  // (sized for the largest item count the pair can have)
  std::vector<size_t> poff(npairs + 1, 0), doff(npairs + 1, 0);
  for (int k = 0; k < npairs; ++k) {
    const int ch = completion_chunks(pds[k].n_items);
    poff[k + 1] = poff[k] + (size_t)kPartialRow * (pds[k].n_items + ch);
    doff[k + 1] = doff[k] + 1 + ch;
  }
  const int max_queue = item_off[npairs];
  double* partial;
  unsigned *done, *queue, *gcost = nullptr;
  PairDev* dpairs;
  int2* ditems;
  int4* dwitems = nullptr;
  FGA_TRY(B.get(&partial, sizeof(double) * poff[npairs]));
  FGA_TRY(B.get(&done, sizeof(unsigned) * doff[npairs]));
  FGA_TRY(B.get(&queue, sizeof(unsigned) * 2));
  FGA_TRY(B.get(&dpairs, sizeof(PairDev) * npairs));
  FGA_TRY(B.get(&ditems, sizeof(int2) * max_queue));
  if (grouped) {
    FGA_TRY(B.get(&dwitems, sizeof(int4) * (size_t)max_groups * kCap));
    FGA_TRY(B.get(&gcost, sizeof(unsigned) * max_groups));
  }
  for (int k = 0; k < npairs; ++k) {
    PairDev& pd = pds[k];
    pd.X = Xp + xoff[k];
    pd.Q = Qp + yoff[k];
    pd.nodes = nodes ? nodes + noff[k] : nullptr;
    pd.V = nullptr;
    pd.st = st + k;
    pd.partial = partial + poff[k];
    pd.done = done + doff[k];
    pd.n = (int)n[k];
    pd.m = (int)m[k];
    pd.n_nodes = nodes ? noff[k + 1] - noff[k] : 0;
    pd.witems = nullptr;
    pd.gcost = nullptr;
    pd.n_groups = 0;
    pd.n_witems = 0;
  }
  FGA_HIP(hipMemsetAsync(done, 0, sizeof(unsigned) * doff[npairs], s));
  FGA_HIP(hipMemsetAsync(queue, 0, sizeof(unsigned) * 2, s));
  std::vector<int2> items;
  if (grouped) {
    std::vector<RigidState> saved(npairs);
    FGA_HIP(hipMemcpyAsync(saved.data(), st, sizeof(RigidState) * npairs, hipMemcpyDeviceToHost, s));
    FGA_HIP(hipStreamSynchronize(s));
    auto restore = [&]() -> fga_status {
      FGA_HIP(hipMemcpyAsync(st, saved.data(), sizeof(RigidState) * npairs, hipMemcpyHostToDevice, s));
      FGA_HIP(hipStreamSynchronize(s));
      return FGA_OK;
    };
    auto upload = [&]() -> fga_status {
      FGA_HIP(hipMemcpyAsync(dpairs, pds.data(), sizeof(PairDev) * npairs, hipMemcpyHostToDevice, s));
      FGA_HIP(hipMemcpyAsync(ditems, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, s));
      return FGA_OK;
    };
    auto launch = [&]() -> fga_status {
      int rb = 1;
      for (int k = 0; k < npairs; ++k) rb = std::max(rb, reduce_blocks(pds[k].n_items));
      return launch_batch_iteration<T>(dpairs, npairs, rb, ditems, (int)items.size(), queue,
                                       std::min((int)items.size(), cus * 8), c, s, true, true);
    };
    // one iteration with one wave per group measures every group's cost for
    // the tau option fi; the rigid states are restored afterwards
    std::map<int, std::vector<unsigned>> costs;  // key 16 * tree set + fi
    int cur_set = 0;
    auto use_set = [&](int ti) {
      cur_set = ti;
      for (int k = 0; k < npairs; ++k) {
        pds[k].nodes = tsets[ti].nodes + tsets[ti].off[k];
        pds[k].n_nodes = tsets[ti].off[k + 1] - tsets[ti].off[k];
      }
    };
    auto measure = [&](int fi) -> fga_status {
      const auto& g = gtab[fi];
      const auto& go = gofs[fi];
      std::vector<int4> wi((size_t)go[npairs]);
      items.clear();
      for (int k = 0; k < npairs; ++k) {
        for (int q = 0; q < (int)g[k].size(); ++q)
          wi[(size_t)go[k] + q] = make_int4(g[k][q].x, g[k][q].y, 1 << 8, go[k] + q);
        pds[k].witems = dwitems + go[k];
        pds[k].n_groups = (int)g[k].size();
        pds[k].n_witems = (int)g[k].size();
        pds[k].gcost = gcost;
        const int nb = (pds[k].n_witems + kBlock / kWave - 1) / (kBlock / kWave);
        pds[k].n_items = nb;
        for (int b = 0; b < nb; ++b) items.push_back(make_int2(k, b));
      }
      FGA_HIP(hipMemcpyAsync(dwitems, wi.data(), sizeof(int4) * wi.size(), hipMemcpyHostToDevice, s));
      FGA_TRY(upload());
      FGA_HIP(hipMemsetAsync(gcost, 0, sizeof(unsigned) * go[npairs], s));
      FGA_TRY(launch());
      auto& cv = costs[16 * cur_set + fi];
      cv.assign(go[npairs], 0u);
      FGA_HIP(hipMemcpyAsync(cv.data(), gcost, sizeof(unsigned) * cv.size(), hipMemcpyDeviceToHost, s));
      return restore();
    };
    // wave items for (fi, cap): heavy groups split over parts; blocks of four
    // items of one pair, queued heaviest first
    auto build = [&](int fi, int cap) -> fga_status {
      const auto& g = gtab[fi];
      const auto& go = gofs[fi];
      const auto& cost = costs[16 * cur_set + fi];
      std::vector<double> cs(cost.begin(), cost.end());
      double total = 0.0;
      for (double v : cs) total += v;
      std::nth_element(cs.begin(), cs.begin() + cs.size() / 2, cs.end());
      const double target = std::max(2.0 * cs[cs.size() / 2], total / 8192.0);
      std::vector<int4> wi((size_t)go[npairs] * kCap);
      std::vector<std::pair<double, int2>> blocks;
      items.clear();
      size_t base = 0;
      for (int k = 0; k < npairs; ++k) {
        std::vector<std::pair<double, int4>> w;
        for (int q = 0; q < (int)g[k].size(); ++q) {
          const unsigned cg = cost[go[k] + q];
          int nr = 1;
          while (2 * nr <= cap && cg > target * nr) nr *= 2;
          for (int r = 0; r < nr; ++r)
            w.push_back({(double)cg / nr, make_int4(g[k][q].x, g[k][q].y, r | nr << 8, go[k] + q)});
        }
        std::stable_sort(w.begin(), w.end(), [](const std::pair<double, int4>& x, const std::pair<double, int4>& y) {
          return x.first > y.first;
        });
        for (size_t e = 0; e < w.size(); ++e) wi[base + e] = w[e].second;
        pds[k].witems = dwitems + base;
        base += w.size();
        pds[k].n_groups = (int)g[k].size();
        pds[k].n_witems = (int)w.size();
        pds[k].gcost = nullptr;
        const int nb = (pds[k].n_witems + kBlock / kWave - 1) / (kBlock / kWave);
        pds[k].n_items = nb;
        for (int b = 0; b < nb; ++b) {
          double bc = 0.0;
          for (int e = 4 * b; e < std::min((int)w.size(), 4 * b + 4); ++e) bc += w[e].first;
          blocks.push_back({bc, make_int2(k, b)});
        }
      }
      std::stable_sort(blocks.begin(), blocks.end(), [](const std::pair<double, int2>& x, const std::pair<double, int2>& y) {
        return x.first > y.first;
      });
      for (auto& b : blocks) items.push_back(b.second);
      FGA_HIP(hipMemcpyAsync(dwitems, wi.data(), sizeof(int4) * base, hipMemcpyHostToDevice, s));
      return upload();
    };
    int best_fi = fis[0], best_cap = caps[0], best_set = 0;
    if (btuned && leaves[0] != tsets[0].leaf) {  // cached leaf size differs from the one built
      FGA_TRY(build_set(leaves[0]));
      best_set = 1;
    }
    use_set(best_set);
    if (!btuned) {
      // every (fi, cap) timed as the faster of two iterations on the batch itself
      hipEvent_t e0, e1;
      FGA_HIP(hipEventCreate(&e0));
      FGA_HIP(hipEventCreate(&e1));
      float best_ms = 1e30f;
      fga_status ts = FGA_OK;
      for (int fi : fis) {
        if ((ts = measure(fi)) != FGA_OK) break;
        for (int cap : caps) {
          if ((ts = build(fi, cap)) != FGA_OK) break;
          float ms = 1e30f;
          for (int r = 0; r < 2 && ts == FGA_OK; ++r) {
            float one = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) ts = FGA_E_DEVICE;
            if (ts == FGA_OK) ts = launch();
            if (ts == FGA_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&one, e0, e1) != hipSuccess))
              ts = FGA_E_DEVICE;
            ms = std::min(ms, one);
          }
          if (ts == FGA_OK) ts = restore();
          if (ts != FGA_OK) break;
          if (ms < best_ms) {
            best_ms = ms;
            best_fi = fi;
            best_cap = cap;
          }
        }
        if (ts != FGA_OK) break;
      }
      // then the other leaf sizes with the best (fi, cap): trees of every pair
      // built again, costs measured on them, and the same timing
      for (size_t li = 1; li < leaves.size() && ts == FGA_OK; ++li) {
        if ((ts = build_set(leaves[li])) != FGA_OK) break;
        use_set((int)tsets.size() - 1);
        if ((ts = measure(best_fi)) != FGA_OK || (ts = build(best_fi, best_cap)) != FGA_OK) break;
        float ms = 1e30f;
        for (int r = 0; r < 2 && ts == FGA_OK; ++r) {
          float one = 0.f;
          if (hipEventRecord(e0, s) != hipSuccess) ts = FGA_E_DEVICE;
          if (ts == FGA_OK) ts = launch();
          if (ts == FGA_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&one, e0, e1) != hipSuccess))
            ts = FGA_E_DEVICE;
          ms = std::min(ms, one);
        }
        if (ts == FGA_OK) ts = restore();
        if (ts == FGA_OK && ms < best_ms) {
          best_ms = ms;
          best_set = (int)tsets.size() - 1;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (ts != FGA_OK) {
        set_error("tuning the batched group walk failed");
        return ts;
      }
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[bkey] = tsets[best_set].leaf << 16 | best_fi << 8 | best_cap;
      tune_save_locked();
    }
    use_set(best_set);
    nodes = tsets[best_set].nodes;
    noff = tsets[best_set].off;
    if (!costs.count(16 * best_set + best_fi)) FGA_TRY(measure(best_fi));
    FGA_TRY(build(best_fi, best_cap));
    B.tuned_leaf = tsets[best_set].leaf;
    B.tuned_fi = best_fi;
    B.tuned_cap = best_cap;
  } else {
    std::vector<int> order(npairs);
    for (int k = 0; k < npairs; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return n[x] > n[y]; });
    for (int k : order)
      for (int e = 0; e < pds[k].n_items; ++e) items.push_back(make_int2(k, e));
  }
  const int n_items = (int)items.size();
  FGA_HIP(hipMemcpyAsync(dpairs, pds.data(), sizeof(PairDev) * npairs, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(ditems, items.data(), sizeof(int2) * n_items, hipMemcpyHostToDevice, s));
  const int n_blocks = std::min(n_items, cus * 8);
  int n_reduce = 1;
  for (int k = 0; k < npairs; ++k) n_reduce = std::max(n_reduce, reduce_blocks(pds[k].n_items));
  // one graph holds `every` iterations; replay until all pairs stopped
  const int every = std::max(1, std::min(p.check_every > 0 ? p.check_every : 16, std::max(1, p.max_iter)));
  FGA_HIP(hipStreamSynchronize(s));
  FGA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  fga_status cst = FGA_OK;
  for (int k = 0; k < every && cst == FGA_OK; ++k)
    cst = launch_batch_iteration<T>(dpairs, npairs, n_reduce, ditems, n_items, queue, n_blocks,
                                    c, s, nodes != nullptr, grouped);
  hipError_t ce = hipStreamEndCapture(s, &B.graph);
  if (cst != FGA_OK) return cst;
  FGA_HIP(ce);
  FGA_HIP(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
  std::vector<RigidState> hs(npairs);
  const int replays = (p.max_iter + every - 1) / every;
  for (int r = 0; r < replays; ++r) {
    FGA_HIP(hipGraphLaunch(B.exec, s));
    FGA_HIP(hipMemcpyAsync(hs.data(), st, sizeof(RigidState) * npairs, hipMemcpyDeviceToHost, s));
    FGA_HIP(hipStreamSynchronize(s));
    bool all = true;
    for (int k = 0; k < npairs && all; ++k) all = hs[k].converged != 0;
    if (all) break;
  }
  if (p.max_iter == 0) {
    FGA_HIP(hipMemcpyAsync(hs.data(), st, sizeof(RigidState) * npairs, hipMemcpyDeviceToHost, s));
    FGA_HIP(hipStreamSynchronize(s));
  }
  const double ms = now_ms() - t0;
  fga_status result = FGA_OK;
  for (int k = 0; k < npairs; ++k) {
    std::memcpy(R + 9 * k, hs[k].R, sizeof(double) * 9);
    denormalise(norm[k], hs[k].R, hs[k].t, t + 3 * k);
    if (reps) {
      reps[k].iters = hs[k].iter;
      reps[k].converged = hs[k].converged == 1;
      reps[k].last_dT2 = hs[k].dT2;
      reps[k].interactions = hs[k].interactions;
      reps[k].ms_total = ms;
      reps[k].traversal = grouped ? kWave : nodes ? 1 : 0;
      reps[k].leaf_size = !nodes ? 0 : grouped ? B.tuned_leaf : std::max(1, p.leaf_size);
    }
    if ((hs[k].flags & 2) && result == FGA_OK) {
      set_error("pair %d: Barnes-Hut group walk: traversal stack overflow (forces incomplete)", k);
      result = FGA_E_DEVICE;
    }
    if ((hs[k].flags & 1) && result == FGA_OK) {
      set_error("pair %d: the template is collinear; the Kabsch rotation is undetermined", k);
      result = FGA_E_DEGENERATE;
    }
  }
  return result;
}

}  // namespace

extern "C" fga_status fga_register_batch(int npairs, const void* const* X, const int64_t* n,
                                         const void* const* Y, const int64_t* m, fga_dtype dt,
                                         const fga_params* p, double* R, double* t,
                                         fga_report* reps, void* stream) {
  if (npairs < 1) {
    set_error("npairs must be >= 1 (got %d)", npairs);
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_ptr(X, "X"));
  FGA_TRY(check_ptr(Y, "Y"));
  FGA_TRY(check_ptr(n, "n"));
  FGA_TRY(check_ptr(m, "m"));
  FGA_TRY(check_ptr(R, "R"));
  FGA_TRY(check_ptr(t, "t"));
  for (int k = 0; k < npairs; ++k) FGA_TRY(validate_pair(X[k], n[k], Y[k], m[k], dt, p));
  if (p->velocity == FGA_VEL_PARTICLE) {
    set_error("particle velocities are not supported in batched registration");
    return FGA_E_UNSUPPORTED;
  }
  if (p->group_width == 128 || p->group_width == 32) {
    set_error("the batched group walk holds groups of 64 particles (group_width 0, 1 or 64)");
    return FGA_E_UNSUPPORTED;
  }
  for (int k = 0; k < npairs; ++k) {
    FGA_TRY(check_device_ptr(X[k], "X[k]"));
    FGA_TRY(check_device_ptr(Y[k], "Y[k]"));
  }
  hipStream_t s = (hipStream_t)stream;
  return p->precision == FGA_PREC_FP64
             ? batch_impl<double>(npairs, X, n, Y, m, dt, *p, R, t, reps, s)
             : batch_impl<float>(npairs, X, n, Y, m, dt, *p, R, t, reps, s);
}

extern "C" fga_status fga_register_sequence(int nframes, const void* const* frames,
                                            const int64_t* sizes, fga_dtype dt, const fga_params* p,
                                            double* R_rel, double* t_rel, double* R_abs,
                                            double* t_abs, fga_report* reps, void* stream) {
  if (nframes < 2) {
    set_error("a sequence needs at least 2 frames (got %d)", nframes);
    return FGA_E_INVALID_ARG;
  }
  FGA_TRY(check_ptr(frames, "frames"));
  FGA_TRY(check_ptr(sizes, "sizes"));
  FGA_TRY(check_ptr(R_rel, "R_rel"));
  FGA_TRY(check_ptr(t_rel, "t_rel"));
  // pair k registers frame k + 1 (template) to frame k (reference); every
  // frame but the last is a reference once, so its tree is built once
  const int np = nframes - 1;
  FGA_TRY(fga_register_batch(np, frames, sizes, frames + 1, sizes + 1, dt, p, R_rel, t_rel, reps,
                             stream));
  if (R_abs && t_abs) {
    // T_0 = [I | 0]; T_{k+1} = T_k o T_rel(k): frame k+1's points in frame 0
    for (int e = 0; e < 9; ++e) R_abs[e] = (e % 4 == 0) ? 1.0 : 0.0;
    for (int a = 0; a < 3; ++a) t_abs[a] = 0.0;
    for (int k = 0; k < np; ++k) {
      const double* Rk = R_abs + 9 * k;
      const double* tk = t_abs + 3 * k;
      const double* Rr = R_rel + 9 * k;
      const double* tr = t_rel + 3 * k;
      double* Rn = R_abs + 9 * (k + 1);
      double* tn = t_abs + 3 * (k + 1);
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int l = 0; l < 3; ++l) v += Rk[3 * i + l] * Rr[3 * l + j];
          Rn[3 * i + j] = v;
        }
        double v = tk[i];
        for (int l = 0; l < 3; ++l) v += Rk[3 * i + l] * tr[l];
        tn[i] = v;
      }
    }
  }
  return FGA_OK;
}
