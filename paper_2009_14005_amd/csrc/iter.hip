// Steps a2-a7 of the hot path, two launches per iteration (a2-a6 in the force
// launch, the end of a6 and a7 in the reduction launch):
//   a2  template pose y_i = R q_i + mu                  (FP64 state -> FP32 lanes)
//   a3/a4 acceleration g_i by direct sum or Barnes-Hut  (Eq. GAForce; Alg. 2)
//   a5  damped velocity and displacement               (Eqs. GAForceDissipative,
//       v' = (1 - c_i) v_i + dt g_i,  d_i = dt v'       TotalGAForce, PreviousVelocity)
//   a6  FP64 moments sum d_i and sum d_i q_i^T, reduced per block into one row
//       per item; a second, small launch sums the rows in a fixed order
//   a7  Kabsch step and state update by the last block of that launch (Eqs.
//       R_Kabsch, transEst; template update and composition of Alg. 2)
//
// Work is split into items (template tile of kBlock particles) x (reference
// range). The moments are linear in g_i, so every item adds its own share and
// no per-particle force has to be combined across items: the velocity term
// enters only through the item of reference range 0.
#include "common.h"
#include "force.h"
#include "reduce.h"
#include "rigid.h"

namespace fga {
namespace {

constexpr int kMom = 12;                // moments: sum d_i, sum d_i q_i^T
constexpr int kRow = kPartialRow;       // + the interaction count (exact in FP64)
static_assert(kRow == kMom + 1, "partial row layout");

template <typename T>
struct Coef {
  T R[9], mu[3], A[9], b[3];
};

template <typename T>
__device__ inline Coef<T> load_coef(const RigidState* st);
template <>
__device__ inline Coef<float> load_coef<float>(const RigidState* st) {
  Coef<float> c;
  for (int k = 0; k < 9; ++k) {
    c.R[k] = st->fR[k];
    c.A[k] = st->fA[k];
  }
  for (int k = 0; k < 3; ++k) {
    c.mu[k] = st->fmu[k];
    c.b[k] = st->fb[k];
  }
  return c;
}
template <>
__device__ inline Coef<double> load_coef<double>(const RigidState* st) {
  Coef<double> c;
  for (int k = 0; k < 9; ++k) {
    c.R[k] = st->R[k];
    c.A[k] = st->A[k];
  }
  for (int k = 0; k < 3; ++k) {
    c.mu[k] = st->mu[k];
    c.b[k] = st->b[k];
  }
  return c;
}

template <typename T> __device__ inline T cG(const IterConsts& c);
template <> __device__ inline float cG<float>(const IterConsts& c) { return c.fG; }
template <> __device__ inline double cG<double>(const IterConsts& c) { return c.G; }
template <typename T> __device__ inline T cEps2(const IterConsts& c);
template <> __device__ inline float cEps2<float>(const IterConsts& c) { return c.feps2; }
template <> __device__ inline double cEps2<double>(const IterConsts& c) { return c.eps2; }
template <typename T> __device__ inline T cDt(const IterConsts& c);
template <> __device__ inline float cDt<float>(const IterConsts& c) { return c.fdt; }
template <> __device__ inline double cDt<double>(const IterConsts& c) { return c.dt; }

// Reference range jr of jrn: [j0, j1), boundaries on multiples of 64.
__device__ inline void jrange(int n, int jrn, int jr, int& j0, int& j1) {
  const int per = ((n + jrn - 1) / jrn + 63) & ~63;
  j0 = min(n, jr * per);
  j1 = min(n, j0 + per);
}

// Steps a5-a6 for the K template particles this thread holds (those with
// owner[k] set): damped velocity and displacement, FP64 moments and the
// block's row of partial sums.
// The velocity coefficients and the template coordinates are read again here
// rather than kept in registers through the force sum.
template <typename T, bool BH, int PREC, int K>
__device__ void finish_item(const PairDev& pd, const IterConsts& c, int item, int jr,
                            const int (&idx)[K], const bool (&owner)[K], const T (&acc)[K][3],
                            unsigned cnt, double* lds) {
  const T G = cG<T>(c), dt = cDt<T>(c);
  const Coef<T> cf = load_coef<T>(pd.st);
  const vec4_t<T>* Q = (const vec4_t<T>*)pd.Q;
  vec4_t<T> q[K];
#pragma unroll
  for (int k = 0; k < K; ++k) q[k] = Q[owner[k] ? idx[k] : 0];
  double mom[kRow];
#pragma unroll
  for (int k = 0; k < kRow; ++k) mom[k] = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // a5: damped velocity and displacement
    T v0 = 0, v1 = 0, v2 = 0;
    if (jr == 0 && owner[k]) {
      if (c.velocity == FGA_VEL_RIGID) {
        v0 = cf.A[0] * q[k].x + cf.A[1] * q[k].y + cf.A[2] * q[k].z + cf.b[0];
        v1 = cf.A[3] * q[k].x + cf.A[4] * q[k].y + cf.A[5] * q[k].z + cf.b[1];
        v2 = cf.A[6] * q[k].x + cf.A[7] * q[k].y + cf.A[8] * q[k].z + cf.b[2];
      } else {
        const T* V = (const T*)pd.V;
        v0 = V[3 * idx[k]];
        v1 = V[3 * idx[k] + 1];
        v2 = V[3 * idx[k] + 2];
      }
    }
    const T keep = (T)1 - q[k].w;  // 1 - c_i
    const T w0 = keep * v0 + dt * (G * acc[k][0]);
    const T w1 = keep * v1 + dt * (G * acc[k][1]);
    const T w2 = keep * v2 + dt * (G * acc[k][2]);
    if (c.velocity == FGA_VEL_PARTICLE && owner[k]) {  // only with a single reference range
      T* V = (T*)pd.V;
      V[3 * idx[k]] = w0;
      V[3 * idx[k] + 1] = w1;
      V[3 * idx[k] + 2] = w2;
    }
    // a6: moments of the displacement d = dt v'
    if (!owner[k]) continue;
    if (PREC == FGA_PREC_FP32_ALL) {
      const float d[3] = {(float)(dt * w0), (float)(dt * w1), (float)(dt * w2)};
      const float qq[3] = {(float)q[k].x, (float)q[k].y, (float)q[k].z};
      for (int a = 0; a < 3; ++a) mom[a] = (double)((float)mom[a] + d[a]);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          mom[3 + 3 * a + b] = (double)((float)mom[3 + 3 * a + b] + d[a] * qq[b]);
    } else {
      const double d[3] = {(double)(dt * w0), (double)(dt * w1), (double)(dt * w2)};
      const double qq[3] = {(double)q[k].x, (double)q[k].y, (double)q[k].z};
      for (int a = 0; a < 3; ++a) mom[a] += d[a];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) mom[3 + 3 * a + b] += d[a] * qq[b];
    }
  }
  // the block's interaction count travels in the row (no atomics here: the
  // count is summed by the reduction launch)
  mom[kMom] = BH ? (double)cnt : 0.0;
  block_sum<kRow>(mom, lds);
  // the block's row of partial moments; the reduction launch sums the rows
  if (threadIdx.x == 0)
    for (int k = 0; k < kRow; ++k)
      pd.partial[(size_t)item * kRow + k] =
          PREC == FGA_PREC_FP32_ALL && k < kMom ? (double)(float)mom[k] : mom[k];
}

// Threads of a reduction block: kRow waves, so that a stride of the block
// over the flat array of rows keeps every thread on one column of the row and
// every load of the block is contiguous.
constexpr int kReduceThreads = kRow * kWave;

// Ordered sum of partial-moment rows [r0, r1). Thread t adds column t mod kRow
// of the flat elements t, t + kReduceThreads, ... (rows t / kRow + 64 j),
// then thread k < kRow adds the kWave per-thread sums of column k in thread
// order: a fixed order, so the result is deterministic. FP32_ALL adds the
// moments in FP32. The result is valid in every thread.
template <int PREC>
__device__ inline void sum_rows(const double* base, int r0, int r1, double (&tot)[kRow],
                                double* lds /* kReduceThreads + kRow */) {
  const int t = (int)threadIdx.x;
  const bool f32 = PREC == FGA_PREC_FP32_ALL && t % kRow < kMom;
  const double* p = base + (size_t)r0 * kRow;
  const int ne = (r1 - r0) * kRow;
  double s = 0.0;
  float sf = 0.f;
#pragma unroll 8
  for (int e = t; e < ne; e += kReduceThreads) {
    const double v = p[e];
    if (f32) sf += (float)v;
    else s += v;
  }
  lds[t] = f32 ? (double)sf : s;
  __syncthreads();
  if (t < kRow) {
    double a = 0.0;
    float af = 0.f;
    for (int i = 0; i < kWave; ++i) {
      const double v = lds[t + kRow * i];
      if (f32) af += (float)v;
      else a += v;
    }
    lds[kReduceThreads + t] = f32 ? (double)af : a;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRow; ++k) tot[k] = lds[kReduceThreads + k];
}

// a6/a7 completion of one pair's iteration, block b of the reduction launch:
// the block sums kReduceRows rows of the iteration kernel's partial moments;
// with several blocks the last one to finish sums their results (both levels
// in a fixed order, so the result is deterministic) and applies the rigid
// step. Running this in a launch of its own keeps device-scope fences, which
// write back and invalidate the L2 of the issuing XCD, out of the force
// kernel, whose tree and points live in that L2.
template <int PREC>
__device__ void reduce_step(const PairDev& pd, const IterConsts& c, int b, double* lds) {
  __shared__ int s_last;
  const int nb = reduce_blocks(pd.n_items);
  double tot[kRow];
  if (nb == 1)
    sum_rows<PREC>(pd.partial, 0, pd.n_items, tot, lds);
  else
    sum_rows<PREC>(pd.partial, b * kReduceRows, min(pd.n_items, (b + 1) * kReduceRows), tot, lds);
  if (nb > 1) {
    double* bpart = pd.partial + (size_t)pd.n_items * kRow;  // one row per reduction block
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < kRow; ++k) bpart[(size_t)b * kRow + k] = tot[k];
      __threadfence();
      const unsigned prev = atomicAdd(pd.done, 1u);
      s_last = prev == (unsigned)(nb - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    sum_rows<PREC>(bpart, 0, nb, tot, lds);
  }
  if (threadIdx.x == 0) {
    pd.st->interactions += pd.nodes ? (long long)tot[kMom] : (long long)pd.n * (long long)pd.m;
    rigid_update(*pd.st, tot, c.dt);
    *pd.done = 0u;
  }
}

// One item of the force launch with one particle per S lanes (the direct
// sum with S = 1, or the per-particle Barnes-Hut traversal).
template <typename T, bool BH, int PREC, int S>
__device__ void iteration_item(const PairDev& pd, const IterConsts& c, int item,
                               double* lds, StackEntry* stk) {
  const RigidState* st = pd.st;
  const int it = item / pd.jr, jr = item - (item / pd.jr) * pd.jr;
  const int i = it * (kBlock / S) + (int)threadIdx.x / S;
  const bool valid = i < pd.m;
  const Coef<T> cf = load_coef<T>(st);
  const vec4_t<T>* Q = (const vec4_t<T>*)pd.Q;
  const vec4_t<T> q = Q[valid ? i : pd.m - 1];
  const T y0 = cf.R[0] * q.x + cf.R[1] * q.y + cf.R[2] * q.z + cf.mu[0];
  const T y1 = cf.R[3] * q.x + cf.R[4] * q.y + cf.R[5] * q.z + cf.mu[1];
  const T y2 = cf.R[6] * q.x + cf.R[7] * q.y + cf.R[8] * q.z + cf.mu[2];
  int j0, j1;
  jrange(pd.n, pd.jr, jr, j0, j1);
  T ax = 0, ay = 0, az = 0;
  unsigned cnt = 0;
  if (BH) {
    bh_accum<T, S>(pd.nodes, (const vec4_t<T>*)pd.X, j0, j1, c.ftheta2, cEps2<T>(c), valid, y0,
                   y1, y2, ax, ay, az, cnt, stk + (threadIdx.x / kWave) * kStack);
  } else if constexpr (sizeof(T) == 8) {
    direct_f64((const double4*)pd.X, j0, j1, y0, y1, y2, c.eps2, ax, ay, az);
  } else {
    if (PREC == FGA_PREC_FP32_KAHAN)
      direct_f32<true, 64>((const float4*)pd.X, j0, j1, y0, y1, y2, c.feps2, ax, ay, az);
    else
      direct_f32<false, 64>((const float4*)pd.X, j0, j1, y0, y1, y2, c.feps2, ax, ay, az);
  }
  const int idx[1] = {i};
  const bool owner[1] = {valid && (threadIdx.x & (S - 1)) == 0};
  const T acc[1][3] = {{ax, ay, az}};
  finish_item<T, BH, PREC, 1>(pd, c, item, jr, idx, owner, acc, cnt, lds);
}

// One block of the group traversal: every wave takes one wave item, a run of
// at most 64 K consecutive template particles (lane l, slot k: particle
// first + K l + k) sharing one walk of the tree, restricted to
// part r of nr of the walk (heavy groups are split over several waves by
// subtrees).
// FP32 only.
template <int PREC, int K, bool PL = false>
__device__ void iteration_item_group(const PairDev& pd, const IterConsts& c, int item,
                                     double* lds, GroupLds* g) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x & (kWave - 1);
  const float4* Q = (const float4*)pd.Q;
  const int wi = item * (kBlock / kWave) + wave;
  int gi = -1, r = 0, nr = 1;
  int2 grp = make_int2(0, 0);
  if (wi < pd.n_witems) {
    const int4 w = pd.witems[wi];
    grp = make_int2(w.x, w.y);
    r = w.z & 255;
    nr = w.z >> 8;
    gi = w.w;
  }
  // a small group is held R times over the lanes (K = 1): R copies of at
  // most 64 / R particles, each copy summing every R-th list entry
  int R = 1;
  if (K == 1)
    while (R < kGRepMax && grp.y <= kWave / (2 * R)) R *= 2;
  const int pl = lane & (kWave / R - 1);
  int idx[K];
  bool valid[K];
  float y[K][3], acc[K][3];
  {
    const RigidState* st = pd.st;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      valid[k] = K * pl + k < grp.y;
      idx[k] = grp.x + K * pl + k;
      const float4 q = Q[valid[k] ? idx[k] : pd.m - 1];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        y[k][a] = st->fR[3 * a] * q.x + st->fR[3 * a + 1] * q.y + st->fR[3 * a + 2] * q.z + st->fmu[a];
      acc[k][0] = acc[k][1] = acc[k][2] = 0.f;
    }
  }
  unsigned cnt = 0, entries = 0;
  const bool ok = bh_group<K, PREC == FGA_PREC_FP32_KAHAN, PL>(
      pd.nodes, pd.n_nodes, (const float4*)pd.X, pd.n, r, nr, R, c.ftheta2, c.feps2,
      valid, y, acc, cnt, entries, g[wave]);
  if (!ok && lane == 0) atomicOr(&pd.st->flags, 2);
  if (pd.gcost && lane == 0 && gi >= 0) atomicAdd(&pd.gcost[gi], entries);
  bool owner[K];
#pragma unroll
  for (int k = 0; k < K; ++k) owner[k] = valid[k] && lane < kWave / R;
  finish_item<float, true, PREC, K>(pd, c, item, r, idx, owner, acc, cnt, lds);
}

template <typename T, bool BH, int PREC, int S>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_iteration(PairDev pd, IterConsts c) {
  __shared__ double lds[kRow * (kBlock / kWave)];
  __shared__ StackEntry stk[BH ? (kBlock / kWave) * kStack : 1];
  if (pd.st->converged) return;  // uniform: the state was written by the previous launch
  iteration_item<T, BH, PREC, S>(pd, c, (int)blockIdx.x, lds, stk);
}

template <int PREC, int K, bool PL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kGroupWavesPerSimd))) void k_iteration_group(PairDev pd, IterConsts c) {
  __shared__ double lds[kRow * (kBlock / kWave)];
  __shared__ GroupLds g[kBlock / kWave];
  if (pd.st->converged) return;  // uniform: the state was written by the previous launch
  iteration_item_group<PREC, K, PL>(pd, c, (int)blockIdx.x, lds, g);
}

// Persistent batched iteration: blocks pull (pair, item) entries from a work
// queue ordered by decreasing cost until it is empty. The block that drains
// the last entry resets the queue for the next launch.
template <typename T, bool BH, int PREC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_iteration(const PairDev* pairs,
                                                            const int2* items, int n_items,
                                                            unsigned* queue, IterConsts c) {
  __shared__ double lds[kRow * (kBlock / kWave)];
  __shared__ StackEntry stk[BH ? (kBlock / kWave) * kStack : 1];
  __shared__ int s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&queue[0], 1u);
    __syncthreads();
    // uniform across the block: in a scalar register, so the pair's fields
    // below are scalar loads rather than per-lane copies
    const int e = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (e >= n_items) break;
    const int2 w = items[e];
    const PairDev& pd = pairs[w.x];  // read in place (uniform address: scalar loads)
    if (pd.st->converged) continue;
    iteration_item<T, BH, PREC, 1>(pd, c, w.y, lds, stk);
    __syncthreads();
  }
}

// Persistent batched iteration with the group walk (K = 1): queue entries are
// (pair, block of four wave items of that pair), ordered heaviest first.
template <int PREC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kGroupWavesPerSimd))) void k_batch_iteration_group(
    const PairDev* pairs, const int2* items, int n_items, unsigned* queue, IterConsts c) {
  __shared__ double lds[kRow * (kBlock / kWave)];
  __shared__ GroupLds g[kBlock / kWave];
  __shared__ int s_item;
  while (true) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&queue[0], 1u);
    __syncthreads();
    // uniform across the block: in a scalar register, so the pair's fields
    // below are scalar loads rather than per-lane copies
    const int e = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (e >= n_items) break;
    const int2 w = items[e];
    const PairDev& pd = pairs[w.x];  // read in place (uniform address: scalar loads)
    if (pd.st->converged) continue;
    iteration_item_group<PREC, 1>(pd, c, w.y, lds, g);
    __syncthreads();
  }
}

template <int PREC>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_step(PairDev pd, IterConsts c) {
  __shared__ double lds[kReduceThreads + kRow];
  if (pd.st->converged) return;  // uniform: the state was written by an earlier launch
  reduce_step<PREC>(pd, c, (int)blockIdx.x, lds);
}

// Reduction launch of the batched iteration: blockIdx.y is the pair. Block
// (0, 0) also rewinds the work queue for the next iteration.
template <int PREC>
__global__ __launch_bounds__(kReduceThreads) void k_batch_reduce_step(const PairDev* pairs,
                                                                      unsigned* queue,
                                                                      IterConsts c) {
  __shared__ double lds[kReduceThreads + kRow];
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) queue[0] = 0u;
  const PairDev pd = pairs[blockIdx.y];
  if ((int)blockIdx.x >= reduce_blocks(pd.n_items) || pd.st->converged) return;
  reduce_step<PREC>(pd, c, (int)blockIdx.x, lds);
}

template <int PREC>
inline void reduce_launch(const PairDev& pd, const IterConsts& c, hipStream_t s) {
  k_reduce_step<PREC><<<reduce_blocks(pd.n_items), kReduceThreads, 0, s>>>(pd, c);
}

}  // namespace

template <typename T>
fga_status launch_iteration(const PairDev& pd, const IterConsts& c, hipStream_t s, hipEvent_t between) {
  const bool bh = pd.nodes != nullptr;
  const dim3 grid((unsigned)pd.n_items);
  if (sizeof(T) == 4 && bh && pd.group > 0 && pd.planar) {  // planar sets: no z terms
    switch (c.prec * 4 + pd.group) {
      case FGA_PREC_FP32 * 4 + 1: k_iteration_group<FGA_PREC_FP32, 1, true><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32 * 4 + 2: k_iteration_group<FGA_PREC_FP32, 2, true><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32_ALL * 4 + 1: k_iteration_group<FGA_PREC_FP32_ALL, 1, true><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32_ALL * 4 + 2: k_iteration_group<FGA_PREC_FP32_ALL, 2, true><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32_KAHAN * 4 + 2: k_iteration_group<FGA_PREC_FP32_KAHAN, 2, true><<<grid, kBlock, 0, s>>>(pd, c); break;
      default: k_iteration_group<FGA_PREC_FP32_KAHAN, 1, true><<<grid, kBlock, 0, s>>>(pd, c);
    }
  } else if (sizeof(T) == 4 && bh && pd.group > 0) {  // group traversal, K particles per lane
    switch (c.prec * 4 + pd.group) {
      case FGA_PREC_FP32 * 4 + 1: k_iteration_group<FGA_PREC_FP32, 1, false><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32 * 4 + 2: k_iteration_group<FGA_PREC_FP32, 2, false><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32_ALL * 4 + 1: k_iteration_group<FGA_PREC_FP32_ALL, 1, false><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32_ALL * 4 + 2: k_iteration_group<FGA_PREC_FP32_ALL, 2, false><<<grid, kBlock, 0, s>>>(pd, c); break;
      case FGA_PREC_FP32_KAHAN * 4 + 2: k_iteration_group<FGA_PREC_FP32_KAHAN, 2, false><<<grid, kBlock, 0, s>>>(pd, c); break;
      default: k_iteration_group<FGA_PREC_FP32_KAHAN, 1, false><<<grid, kBlock, 0, s>>>(pd, c);
    }
  } else if (sizeof(T) == 8) {
    if (bh) k_iteration<T, true, FGA_PREC_FP64, 1><<<grid, kBlock, 0, s>>>(pd, c);
    else k_iteration<T, false, FGA_PREC_FP64, 1><<<grid, kBlock, 0, s>>>(pd, c);
  } else {
    switch (c.prec) {
      case FGA_PREC_FP32:
        if (bh) k_iteration<T, true, FGA_PREC_FP32, 1><<<grid, kBlock, 0, s>>>(pd, c);
        else k_iteration<T, false, FGA_PREC_FP32, 1><<<grid, kBlock, 0, s>>>(pd, c);
        break;
      case FGA_PREC_FP32_ALL:
        if (bh) k_iteration<T, true, FGA_PREC_FP32_ALL, 1><<<grid, kBlock, 0, s>>>(pd, c);
        else k_iteration<T, false, FGA_PREC_FP32_ALL, 1><<<grid, kBlock, 0, s>>>(pd, c);
        break;
      default:
        if (!bh) {
          k_iteration<T, false, FGA_PREC_FP32_KAHAN, 1><<<grid, kBlock, 0, s>>>(pd, c);
        } else {
          switch (pd.slots) {  // traversal width chosen by the autotuner
            case 2: k_iteration<T, true, FGA_PREC_FP32_KAHAN, 2><<<grid, kBlock, 0, s>>>(pd, c); break;
            case 4: k_iteration<T, true, FGA_PREC_FP32_KAHAN, 4><<<grid, kBlock, 0, s>>>(pd, c); break;
            case 8: k_iteration<T, true, FGA_PREC_FP32_KAHAN, 8><<<grid, kBlock, 0, s>>>(pd, c); break;
            default: k_iteration<T, true, FGA_PREC_FP32_KAHAN, 1><<<grid, kBlock, 0, s>>>(pd, c);
          }
        }
    }
  }
  if (between) FGA_HIP(hipEventRecord(between, s));  // splits the force and reduction launches
  if (sizeof(T) == 8) reduce_launch<FGA_PREC_FP64>(pd, c, s);
  else if (c.prec == FGA_PREC_FP32_ALL) reduce_launch<FGA_PREC_FP32_ALL>(pd, c, s);
  else reduce_launch<FGA_PREC_FP32_KAHAN>(pd, c, s);
  FGA_HIP(hipGetLastError());
  return FGA_OK;
}

template <typename T>
fga_status launch_batch_iteration(const PairDev* pairs_dev, int npairs, int reduce_blocks,
                                  const int2* items, int n_items, unsigned* queue, int n_blocks,
                                  const IterConsts& c, hipStream_t s, bool bh, bool group) {
  if (sizeof(T) == 4 && bh && group) {
    switch (c.prec) {
      case FGA_PREC_FP32: k_batch_iteration_group<FGA_PREC_FP32><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      case FGA_PREC_FP32_ALL: k_batch_iteration_group<FGA_PREC_FP32_ALL><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      default: k_batch_iteration_group<FGA_PREC_FP32_KAHAN><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c);
    }
  } else if (sizeof(T) == 8) {
    if (bh) k_batch_iteration<T, true, FGA_PREC_FP64><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c);
    else k_batch_iteration<T, false, FGA_PREC_FP64><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c);
  } else {
    switch (c.prec * 2 + (bh ? 1 : 0)) {
      case FGA_PREC_FP32 * 2 + 1: k_batch_iteration<T, true, FGA_PREC_FP32><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      case FGA_PREC_FP32 * 2: k_batch_iteration<T, false, FGA_PREC_FP32><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      case FGA_PREC_FP32_ALL * 2 + 1: k_batch_iteration<T, true, FGA_PREC_FP32_ALL><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      case FGA_PREC_FP32_ALL * 2: k_batch_iteration<T, false, FGA_PREC_FP32_ALL><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      case FGA_PREC_FP32_KAHAN * 2 + 1: k_batch_iteration<T, true, FGA_PREC_FP32_KAHAN><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c); break;
      default: k_batch_iteration<T, false, FGA_PREC_FP32_KAHAN><<<n_blocks, kBlock, 0, s>>>(pairs_dev, items, n_items, queue, c);
    }
  }
  const dim3 rgrid((unsigned)std::max(1, reduce_blocks), (unsigned)npairs);
  if (sizeof(T) == 8) k_batch_reduce_step<FGA_PREC_FP64><<<rgrid, kReduceThreads, 0, s>>>(pairs_dev, queue, c);
  else if (c.prec == FGA_PREC_FP32_ALL) k_batch_reduce_step<FGA_PREC_FP32_ALL><<<rgrid, kReduceThreads, 0, s>>>(pairs_dev, queue, c);
  else k_batch_reduce_step<FGA_PREC_FP32_KAHAN><<<rgrid, kReduceThreads, 0, s>>>(pairs_dev, queue, c);
  FGA_HIP(hipGetLastError());
  return FGA_OK;
}

template fga_status launch_iteration<float>(const PairDev&, const IterConsts&, hipStream_t, hipEvent_t);
template fga_status launch_iteration<double>(const PairDev&, const IterConsts&, hipStream_t, hipEvent_t);
template fga_status launch_batch_iteration<float>(const PairDev*, int, int, const int2*, int,
                                                  unsigned*, int, const IterConsts&, hipStream_t,
                                                  bool, bool);
template fga_status launch_batch_iteration<double>(const PairDev*, int, int, const int2*, int,
                                                   unsigned*, int, const IterConsts&, hipStream_t,
                                                   bool, bool);

// ------------------------------------------------------------------ forces
namespace {

// Packs X (n x 3) and its masses into vec4 (x, y, z, m).
template <typename T>
__global__ void k_pack4(const T* X, const T* m, int64_t n, vec4_t<T>* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make4<T>(X[3 * i], X[3 * i + 1], X[3 * i + 2], m[i]);
}

// Direct forces of one reference range: acc of Eq. (GAForce) per particle,
// written to part[jr][i][3].
template <typename T, int PREC>
__global__ __launch_bounds__(kBlock) void k_forces_direct(const T* Y, int m, const vec4_t<T>* X,
                                                          int n, int jrn, T eps2, T* part) {
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  const int jr = blockIdx.y;
  const bool valid = i < m;
  const int ii = valid ? i : m - 1;
  const T yx = Y[3 * ii], yy = Y[3 * ii + 1], yz = Y[3 * ii + 2];
  int j0, j1;
  jrange(n, jrn, jr, j0, j1);
  T ax = 0, ay = 0, az = 0;
  if constexpr (sizeof(T) == 8) {
    direct_f64((const double4*)X, j0, j1, yx, yy, yz, eps2, ax, ay, az);
  } else {
    if (PREC == FGA_PREC_FP32)
      direct_f32<false, 64>((const float4*)X, j0, j1, yx, yy, yz, eps2, ax, ay, az);
    else
      direct_f32<true, 64>((const float4*)X, j0, j1, yx, yy, yz, eps2, ax, ay, az);
  }
  if (valid) {
    T* o = part + ((size_t)jr * m + i) * 3;
    o[0] = ax;
    o[1] = ay;
    o[2] = az;
  }
}

// F_i = G m_Y,i sum_jr part[jr][i] (ranges combined in order, in FP64).
template <typename T>
__global__ void k_forces_combine(const T* part, int m, int jrn, const T* mY, double G, T* F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int r = 0; r < jrn; ++r)
    for (int a = 0; a < 3; ++a) s[a] += (double)part[((size_t)r * m + i) * 3 + a];
  const double w = G * (mY ? (double)mY[i] : 1.0);
  for (int a = 0; a < 3; ++a) F[3 * i + a] = (T)(w * s[a]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_forces_bh(const T* Y, const int* yorder, int m,
                                                      const BHWide* nodes, int n_nodes,
                                                      const vec4_t<T>* Xs, float theta2, T eps2,
                                                      const T* mY, double G, T* F,
                                                      unsigned long long* count) {
  __shared__ StackEntry stk[(kBlock / kWave) * kStack];
  constexpr int S = 1;
  const int k = blockIdx.x * (kBlock / S) + (int)threadIdx.x / S;
  const bool valid = k < m;
  const bool owner = valid && (threadIdx.x & (S - 1)) == 0;
  const int i = valid ? yorder[k] : 0;
  const T yx = Y[3 * i], yy = Y[3 * i + 1], yz = Y[3 * i + 2];
  T ax = 0, ay = 0, az = 0;
  unsigned cnt = 0;
  (void)n_nodes;
  bh_accum<T, S>(nodes, Xs, 0, 0x7fffffff, theta2, eps2, valid, yx, yy, yz, ax, ay, az, cnt,
                 stk + (threadIdx.x / kWave) * kStack);
  if (owner) {
    const double w = G * (mY ? (double)mY[i] : 1.0);
    F[3 * i] = (T)(w * (double)ax);
    F[3 * i + 1] = (T)(w * (double)ay);
    F[3 * i + 2] = (T)(w * (double)az);
  }
  unsigned long long c = cnt;
  for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(count, c);
}

// ------------------------------------------------------ Plummer energy
// E = -G sum_i m_Y,i sum_j m_X,j / sqrt(|y_i - x_j|^2 + eps^2), the energy
// whose negative gradient is Eq. (GAForce) (a convergence diagnostic).
// Direct: per (template tile, reference range) the partial potentials, summed
// per particle in FP64 in range order (tiles of 64 terms in the data's
// precision); BH: the per-particle walk of Alg. 2 with the potential terms.
// Both end in one FP64 partial per block and an ordered final sum.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy_direct(const T* Y, int m, const vec4_t<T>* X,
                                                          int n, int jrn, T eps2, double* part) {
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  const int jr = blockIdx.y;
  const bool valid = i < m;
  const int ii = valid ? i : m - 1;
  const T yx = Y[3 * ii], yy = Y[3 * ii + 1], yz = Y[3 * ii + 2];
  int j0, j1;
  jrange(n, jrn, jr, j0, j1);
  double acc = 0.0;
  for (int j = j0; j < j1; j += 64) {
    const int je = min(j + 64, j1);
    T t = 0;
    for (int q = j; q < je; ++q) {
      const vec4_t<T> x = X[q];
      const T dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
      t += rsqrt1_mass<T>(x.w, dx * dx + dy * dy + dz * dz + eps2);
    }
    acc += (double)t;
  }
  if (valid) part[(size_t)jr * m + i] = acc;
}

// One FP64 partial per block: sum over its particles of m_Y,i * potential_i.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy_rows(const double* part, int m, int jrn,
                                                        const T* mY, double* rows) {
  __shared__ double lds[kBlock / kWave];
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  double v[1] = {0.0};
  if (i < m) {
    for (int r = 0; r < jrn; ++r) v[0] += part[(size_t)r * m + i];
    v[0] *= mY ? (double)mY[i] : 1.0;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) rows[blockIdx.x] = v[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_energy_bh(const T* Y, const int* yorder, int m,
                                                      const BHWide* nodes, const vec4_t<T>* Xs,
                                                      float theta2, T eps2, const T* mY,
                                                      double* rows, unsigned long long* count) {
  __shared__ StackEntry stk[(kBlock / kWave) * kStack];
  __shared__ double lds[kBlock / kWave];
  const int k = blockIdx.x * kBlock + (int)threadIdx.x;
  const bool valid = k < m;
  const int i = valid ? yorder[k] : 0;
  const T yx = Y[3 * i], yy = Y[3 * i + 1], yz = Y[3 * i + 2];
  T pot = 0, unused_y = 0, unused_z = 0;
  unsigned cnt = 0;
  bh_accum<T, 1, true>(nodes, Xs, 0, 0x7fffffff, theta2, eps2, valid, yx, yy, yz, pot, unused_y,
                       unused_z, cnt, stk + (threadIdx.x / kWave) * kStack);
  double v[1] = {valid ? (double)pot * (mY ? (double)mY[i] : 1.0) : 0.0};
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) rows[blockIdx.x] = v[0];
  unsigned long long c = cnt;
  for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(count, c);
}

// E = -G sum of the block partials, in block order (one block).
__global__ __launch_bounds__(kBlock) void k_energy_final(const double* rows, int nrows, double G,
                                                         double* E) {
  __shared__ double lds[kBlock / kWave];
  double v[1] = {0.0};
  // each thread sums a contiguous run of rows, then the block adds the runs
  const int per = (nrows + kBlock - 1) / kBlock;
  for (int r = (int)threadIdx.x * per; r < min(nrows, ((int)threadIdx.x + 1) * per); ++r) v[0] += rows[r];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) *E = -G * v[0];
}

// Group traversal for fga_forces: every wave takes 64 K / R consecutive
// template particles of the Morton order yorder (R = 2: a group of 32 held
// twice over the lanes, K = 1) and writes F_i = G m_Y,i acc_i.
template <int K, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_forces_group(const float* Y, const int* yorder, int m,
                                                         const BHWide* nodes, int n_nodes,
                                                         const float4* Xs, int n_points,
                                                         float theta2, float eps2, const float* mY,
                                                         double G, float* F,
                                                         unsigned long long* count, int R) {
  __shared__ GroupLds g[kBlock / kWave];
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x & (kWave - 1);
  const int per_wave = kWave * K / R, pl = lane & (kWave / R - 1);
  int idx[K];
  bool valid[K];
  float y[K][3], acc[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int pos = blockIdx.x * (kBlock / kWave) * per_wave + wave * per_wave + K * pl + k;
    valid[k] = pos < m;
    idx[k] = valid[k] ? yorder[pos] : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      y[k][a] = Y[3 * idx[k] + a];
      acc[k][a] = 0.f;
    }
  }
  unsigned cnt = 0, entries = 0;
  const bool ok = bh_group<K, KAHAN>(nodes, n_nodes, Xs, n_points, 0, 1, R, theta2, eps2, valid,
                                    y, acc, cnt, entries, g[wave]);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (valid[k] && lane < kWave / R) {
      const double w = G * (mY ? (double)mY[idx[k]] : 1.0);
#pragma unroll
      for (int a = 0; a < 3; ++a) F[3 * idx[k] + a] = ok ? (float)(w * (double)acc[k][a]) : __builtin_nanf("");
    }
  unsigned long long c = cnt;
  for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if (lane == 0) atomicAdd(count, c);
}

}  // namespace

// Number of reference ranges so that the launch has about 8 waves per SIMD.
int direct_ranges(int64_t m, int64_t n) {
  const int64_t tiles = (m + kBlock - 1) / kBlock;
  const int64_t want = 4096;  // blocks of 4 waves: 16 waves per SIMD on 256 CUs
  int64_t jr = (want + tiles - 1) / tiles;
  const int64_t maxjr = (n + 1023) / 1024;  // at least 1024 reference points per range
  if (jr > maxjr) jr = maxjr;
  if (jr < 1) jr = 1;
  return (int)jr;
}

// Scratch of the direct sum: the packed reference (n vec4) at offset 0, the
// partial forces of the jrn reference ranges (jrn x m x 3) after it, each part
// starting on a 256-byte boundary.
static size_t direct_part_offset(int64_t n, bool f64) {
  const size_t x4 = (f64 ? sizeof(double4) : sizeof(float4)) * (size_t)n;
  return (x4 + 255) / 256 * 256;
}

size_t forces_direct_scratch(int64_t m, int64_t n, bool f64) {
  return direct_part_offset(n, f64) + (f64 ? 8 : 4) * 3 * (size_t)m * direct_ranges(m, n);
}

template <typename T>
fga_status forces_direct_into(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                              const void* mY, const fga_params& p, void* F, void* scratch,
                              hipStream_t s) {
  const int jrn = direct_ranges(m, n);
  vec4_t<T>* X4 = (vec4_t<T>*)scratch;
  T* part = (T*)((char*)scratch + direct_part_offset(n, sizeof(T) == 8));
  k_pack4<T><<<(int)((n + 255) / 256), 256, 0, s>>>((const T*)X, (const T*)mX, n, X4);
  const dim3 grid((unsigned)((m + kBlock - 1) / kBlock), (unsigned)jrn);
  const T eps2 = (T)(p.eps * p.eps);
  if (sizeof(T) == 8 || p.precision == FGA_PREC_FP32_KAHAN)
    k_forces_direct<T, FGA_PREC_FP32_KAHAN><<<grid, kBlock, 0, s>>>((const T*)Y, (int)m, X4, (int)n, jrn, eps2, part);
  else
    k_forces_direct<T, FGA_PREC_FP32><<<grid, kBlock, 0, s>>>((const T*)Y, (int)m, X4, (int)n, jrn, eps2, part);
  k_forces_combine<T><<<(int)((m + 255) / 256), 256, 0, s>>>(part, (int)m, jrn, (const T*)mY, p.G, (T*)F);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("direct force kernels failed to launch: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  return FGA_OK;
}

template <typename T>
fga_status forces_direct(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                         const void* mY, const fga_params& p, void* F, hipStream_t s) {
  void* scratch = nullptr;
  FGA_TRY(pool_get(&scratch, forces_direct_scratch(m, n, sizeof(T) == 8), s));
  fga_status st = forces_direct_into<T>(Y, m, X, n, mX, mY, p, F, scratch, s);
  const hipError_t e = hipStreamSynchronize(s);
  pool_free(scratch, s);
  if (st == FGA_OK && e != hipSuccess) {
    set_error("direct force kernels failed: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  return st;
}

template <typename T>
fga_status pack_points(const void* X, const void* mX, int64_t n, void* out, hipStream_t s) {
  k_pack4<T><<<(int)((n + 255) / 256), 256, 0, s>>>((const T*)X, (const T*)mX, n, (vec4_t<T>*)out);
  FGA_HIP(hipGetLastError());
  return FGA_OK;
}
template fga_status pack_points<float>(const void*, const void*, int64_t, void*, hipStream_t);
template fga_status pack_points<double>(const void*, const void*, int64_t, void*, hipStream_t);

template <typename T>
fga_status forces_bh_tree(const void* Y, int64_t m, const int* yorder, const BHWide* nodes,
                          int n_nodes, const void* Xs, int64_t n, double theta,
                          const fga_params& p, const void* mY, void* F, long long* interactions,
                          hipStream_t s) {
  unsigned long long* cnt = nullptr;
  FGA_TRY(pool_get(&cnt, sizeof(unsigned long long), s));
  (void)hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s);
  // 32 -> K = 1 held twice (R = 2), 64 -> K = 1, 128 -> K = 2
  const int K = sizeof(T) == 4 ? (p.group_width == 32 ? 1 : p.group_width / kWave) : 0;
  const int R = p.group_width == 32 ? 2 : 1;
  if constexpr (sizeof(T) == 4) {
    if (K == 1 || K == 2) {
      const int tp = kBlock * K / R;
      const dim3 grid((unsigned)((m + tp - 1) / tp));
      const float t2 = (float)(theta * theta), e2 = (float)(p.eps * p.eps);
      const float* Yf = (const float*)Y;
      const float4* X4 = (const float4*)Xs;
      const bool kahan = p.precision == FGA_PREC_FP32_KAHAN;
      if (K == 1 && kahan)
        k_forces_group<1, true><<<grid, kBlock, 0, s>>>(Yf, yorder, (int)m, nodes, n_nodes, X4, (int)n, t2, e2, (const float*)mY, p.G, (float*)F, cnt, R);
      else if (K == 1)
        k_forces_group<1, false><<<grid, kBlock, 0, s>>>(Yf, yorder, (int)m, nodes, n_nodes, X4, (int)n, t2, e2, (const float*)mY, p.G, (float*)F, cnt, R);
      else if (kahan)
        k_forces_group<2, true><<<grid, kBlock, 0, s>>>(Yf, yorder, (int)m, nodes, n_nodes, X4, (int)n, t2, e2, (const float*)mY, p.G, (float*)F, cnt, R);
      else
        k_forces_group<2, false><<<grid, kBlock, 0, s>>>(Yf, yorder, (int)m, nodes, n_nodes, X4, (int)n, t2, e2, (const float*)mY, p.G, (float*)F, cnt, R);
    }
  }
  if (K != 1 && K != 2) {
    constexpr int tp = kBlock;
    k_forces_bh<T><<<(int)((m + tp - 1) / tp), kBlock, 0, s>>>(
        (const T*)Y, yorder, (int)m, nodes, n_nodes, (const vec4_t<T>*)Xs, (float)(theta * theta),
        (T)(p.eps * p.eps), (const T*)mY, p.G, (T*)F, cnt);
  }
  unsigned long long h = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  pool_free(cnt, s);
  if (e != hipSuccess) {
    set_error("BH force kernel failed: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  if (interactions) *interactions = (long long)h;
  return FGA_OK;
}

template <typename T>
fga_status energy_direct(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                         const void* mY, const fga_params& p, double* E_host, hipStream_t s) {
  const int jrn = direct_ranges(m, n);
  const int nb = (int)((m + kBlock - 1) / kBlock);
  const size_t x4 = ((sizeof(vec4_t<T>) * (size_t)n + 255) / 256) * 256;
  const size_t pb = ((sizeof(double) * (size_t)m * jrn + 255) / 256) * 256;
  char* buf = nullptr;
  FGA_TRY(pool_get(&buf, x4 + pb + sizeof(double) * (nb + 1), s));
  vec4_t<T>* X4 = (vec4_t<T>*)buf;
  double* part = (double*)(buf + x4);
  double* rows = (double*)(buf + x4 + pb);
  k_pack4<T><<<(int)((n + 255) / 256), 256, 0, s>>>((const T*)X, (const T*)mX, n, X4);
  k_energy_direct<T><<<dim3((unsigned)nb, (unsigned)jrn), kBlock, 0, s>>>((const T*)Y, (int)m, X4, (int)n, jrn,
                                                                          (T)(p.eps * p.eps), part);
  k_energy_rows<T><<<nb, kBlock, 0, s>>>(part, (int)m, jrn, (const T*)mY, rows);
  k_energy_final<<<1, kBlock, 0, s>>>(rows, nb, p.G, rows + nb);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(E_host, rows + nb, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  pool_free(buf, s);
  if (e != hipSuccess) {
    set_error("energy kernels failed: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  return FGA_OK;
}

template <typename T>
fga_status energy_bh_tree(const void* Y, int64_t m, const int* yorder, const BHWide* nodes,
                          const void* Xs, double theta, const fga_params& p, const void* mY,
                          double* E_host, long long* interactions, hipStream_t s) {
  const int nb = (int)((m + kBlock - 1) / kBlock);
  char* buf = nullptr;
  FGA_TRY(pool_get(&buf, sizeof(double) * (nb + 1) + sizeof(unsigned long long), s));
  double* rows = (double*)buf;
  unsigned long long* cnt = (unsigned long long*)(buf + sizeof(double) * (nb + 1));
  hipError_t e = hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s);
  k_energy_bh<T><<<nb, kBlock, 0, s>>>((const T*)Y, yorder, (int)m, nodes, (const vec4_t<T>*)Xs,
                                       (float)(theta * theta), (T)(p.eps * p.eps), (const T*)mY,
                                       rows, cnt);
  k_energy_final<<<1, kBlock, 0, s>>>(rows, nb, p.G, rows + nb);
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(E_host, rows + nb, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  pool_free(buf, s);
  if (e != hipSuccess) {
    set_error("BH energy kernel failed: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  if (interactions) *interactions = (long long)h;
  return FGA_OK;
}

// Planar point sets (n x 2) embedded at z = 0 (n x 3), and back.
template <typename T>
__global__ void k_embed_planar(const T* in, int64_t n, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    out[3 * i] = in[2 * i];
    out[3 * i + 1] = in[2 * i + 1];
    out[3 * i + 2] = (T)0;
  }
}
template <typename T>
__global__ void k_take_planar(const T* in, int64_t n, T* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    out[2 * i] = in[3 * i];
    out[2 * i + 1] = in[3 * i + 1];
  }
}
fga_status embed_planar(const void* in, int64_t n, bool f64, void* out, hipStream_t s) {
  if (f64) k_embed_planar<double><<<(int)((n + 255) / 256), 256, 0, s>>>((const double*)in, n, (double*)out);
  else k_embed_planar<float><<<(int)((n + 255) / 256), 256, 0, s>>>((const float*)in, n, (float*)out);
  FGA_HIP(hipGetLastError());
  return FGA_OK;
}
fga_status take_planar(const void* in, int64_t n, bool f64, void* out, hipStream_t s) {
  if (f64) k_take_planar<double><<<(int)((n + 255) / 256), 256, 0, s>>>((const double*)in, n, (double*)out);
  else k_take_planar<float><<<(int)((n + 255) / 256), 256, 0, s>>>((const float*)in, n, (float*)out);
  FGA_HIP(hipGetLastError());
  return FGA_OK;
}

template fga_status energy_direct<float>(const void*, int64_t, const void*, int64_t, const void*,
                                         const void*, const fga_params&, double*, hipStream_t);
template fga_status energy_direct<double>(const void*, int64_t, const void*, int64_t, const void*,
                                          const void*, const fga_params&, double*, hipStream_t);
template fga_status energy_bh_tree<float>(const void*, int64_t, const int*, const BHWide*, const void*,
                                          double, const fga_params&, const void*, double*, long long*,
                                          hipStream_t);
template fga_status energy_bh_tree<double>(const void*, int64_t, const int*, const BHWide*, const void*,
                                           double, const fga_params&, const void*, double*, long long*,
                                           hipStream_t);
template fga_status forces_direct<float>(const void*, int64_t, const void*, int64_t, const void*,
                                         const void*, const fga_params&, void*, hipStream_t);
template fga_status forces_direct<double>(const void*, int64_t, const void*, int64_t, const void*,
                                          const void*, const fga_params&, void*, hipStream_t);
template fga_status forces_direct_into<float>(const void*, int64_t, const void*, int64_t, const void*,
                                              const void*, const fga_params&, void*, void*, hipStream_t);
template fga_status forces_direct_into<double>(const void*, int64_t, const void*, int64_t, const void*,
                                               const void*, const fga_params&, void*, void*, hipStream_t);
template fga_status forces_bh_tree<float>(const void*, int64_t, const int*, const BHWide*, int,
                                          const void*, int64_t, double, const fga_params&,
                                          const void*, void*, long long*, hipStream_t);
template fga_status forces_bh_tree<double>(const void*, int64_t, const int*, const BHWide*, int,
                                           const void*, int64_t, double, const fga_params&,
                                           const void*, void*, long long*, hipStream_t);

}  // namespace fga
