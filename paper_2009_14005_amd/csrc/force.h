// Per-lane force accumulation: the direct sum of Eq. (GAForce) over a range
// of reference points, and the Barnes-Hut traversal of Alg. 2 (BHForce) with
// the acceptance test of Eq. (MAC). Both accumulate
//   acc = sum_j m_j (x_j - y) / (|y - x_j|^2 + eps^2)^(3/2)
// so that the acceleration is g = G * acc and the force F = m_Y * g.
#pragma once
#include "common.h"
#include "reduce.h"

namespace fga {

// ------------------------------------------------------------- direct sum
// FP32 lanes: each lane owns one template particle and reads the reference
// points wave-uniformly (scalar loads), TILE points per partial sum. With
// KAHAN the tile sums are added to the running total with Kahan
// compensation; otherwise the lane accumulates directly.
template <bool KAHAN, int TILE>
__device__ inline void direct_f32(const float4* __restrict__ X, int j0, int j1, float yx,
                                  float yy, float yz, float eps2, float& ax, float& ay,
                                  float& az) {
  float cx = 0.f, cy = 0.f, cz = 0.f;
  for (int jt = j0; jt < j1; jt += TILE) {
    const int je = min(jt + TILE, j1);
    float tx = 0.f, ty = 0.f, tz = 0.f;
    if (!KAHAN) {
      tx = ax;
      ty = ay;
      tz = az;
    }
#pragma unroll 8
    for (int j = jt; j < je; ++j) {
      const float4 x = X[j];
      const float dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
      const float r = __builtin_amdgcn_rsqf(r2);
      const float s = x.w * r * (r * r);
      tx = fmaf(dx, s, tx);
      ty = fmaf(dy, s, ty);
      tz = fmaf(dz, s, tz);
    }
    if (KAHAN) {  // total += tile sum, compensated
      float u = tx - cx, t = ax + u;
      cx = (t - ax) - u;
      ax = t;
      u = ty - cy;
      t = ay + u;
      cy = (t - ay) - u;
      ay = t;
      u = tz - cz;
      t = az + u;
      cz = (t - az) - u;
      az = t;
    } else {
      ax = tx;
      ay = ty;
      az = tz;
    }
  }
}

// FP64 lanes: the same sum in double precision (IEEE sqrt and division).
// 1/sqrt(x) in FP64 for x > 0: the hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - x y^2) / 2, each of which squares the
// relative error, so the result is within a few ulps of the rounded value.
// About a third of the instructions of a square root followed by a division.
__device__ inline double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__device__ inline void direct_f64(const double4* __restrict__ X, int j0, int j1, double yx,
                                  double yy, double yz, double eps2, double& ax, double& ay,
                                  double& az) {
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    const double4 x = X[j];
    const double dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    const double r = rsqrt_f64(r2);
    const double s = x.w * r * (r * r);
    ax += dx * s;
    ay += dy * s;
    az += dz * s;
  }
}

template <typename T>
__device__ inline T rsqrt3_mass(T m, T r2);
template <>
__device__ inline float rsqrt3_mass<float>(float m, float r2) {
  const float r = __builtin_amdgcn_rsqf(r2);
  return m * r * (r * r);
}
template <>
__device__ inline double rsqrt3_mass<double>(double m, double r2) {
  const double r = rsqrt_f64(r2);
  return m * r * (r * r);
}

// m / sqrt(r2): one term of the Plummer potential (the energy diagnostic).
template <typename T>
__device__ inline T rsqrt1_mass(T m, T r2);
template <>
__device__ inline float rsqrt1_mass<float>(float m, float r2) {
  return m * __builtin_amdgcn_rsqf(r2);
}
template <>
__device__ inline double rsqrt1_mass<double>(double m, double r2) {
  return m * rsqrt_f64(r2);
}


// ------------------------------------------------------------- Barnes-Hut
// Wavefront-cooperative traversal with per-lane decisions. Lanes are template
// particles; the wave walks the union of the nodes its lanes need, and every
// lane makes exactly the accept/open decisions of Alg. 2 for its own particle,
// whatever its neighbours do. The walk is a depth-first stack of child blocks
// kept in LDS: an entry is (first child, number of children, mask of the lanes
// that opened the parent). Popping an entry fetches the whole block (the
// children are contiguous), so one round trip to memory serves up to eight
// nodes. For every node of the block each active lane
//   - accepts it when l^2 < theta^2 r^2 (Eq. MAC with l / r < theta; r = 0
//     never accepts) and adds the node's Eq. (GAForce) term;
//   - otherwise evaluates a leaf, or a twig (an internal node whose children
//     are all singleton leaves, whose opening evaluates every child exactly),
//     point by point;
//   - otherwise opens it: the lanes that open a node push its child block.
// Singleton leaves are always evaluated directly in FP32 lanes: the node holds
// the point and its mass, so acceptance and opening give the same term.
//
// A traversal may be restricted to reference points [j0, j1): subtrees outside
// the range are skipped, an accepted node is counted only by the range that
// holds its first point, and a leaf contributes only its points inside the
// range. The ranges of one particle together give exactly its Alg. 2 sum.
constexpr int kStack = 192;  // entries per wave; a walk needs at most 8 per tree level
struct StackEntry {
  int start;
  int count;
  unsigned long long mask;
};

// One exact term of Eq. (GAForce) (per unit G and template mass); with POT
// the Plummer potential term m / sqrt(r^2 + eps^2), added to ax alone.
template <typename T, bool POT = false>
__device__ inline void accum_point(const vec4_t<T>& x, T yx, T yy, T yz, T eps2, T& ax, T& ay,
                                   T& az) {
  const T ex = x.x - yx, ey = x.y - yy, ez = x.z - yz;
  if constexpr (POT) {
    ax += rsqrt1_mass<T>(x.w, ex * ex + ey * ey + ez * ez + eps2);
  } else {
    const T s = rsqrt3_mass<T>(x.w, ex * ex + ey * ey + ez * ez + eps2);
    ax += ex * s;
    ay += ey * s;
    az += ez * s;
  }
}

// Lanes per particle in the traversal. Each particle is held by S lanes
// ("slots"); the S lanes of a particle evaluate S nodes of a child block at
// once, so a wave walks the union of only 64 / S particles' trees and every
// instruction of the walk serves S nodes. The slots' partial sums are added
// at the end.
template <int S>
struct SlotMask;  // bits of the slot-0 lanes, one per particle of the wave
template <> struct SlotMask<1> { static constexpr unsigned long long v = ~0ull; };
template <> struct SlotMask<2> { static constexpr unsigned long long v = 0x5555555555555555ull; };
template <> struct SlotMask<4> { static constexpr unsigned long long v = 0x1111111111111111ull; };
template <> struct SlotMask<8> { static constexpr unsigned long long v = 0x0101010101010101ull; };

// With POT the traversal makes the same decisions and sums the Plummer
// potential instead (node term M / sqrt(r^2 + eps^2), into ax).
template <typename T, int S, bool POT = false>
__device__ inline void bh_accum(const BHWide* __restrict__ nodes,
                                const vec4_t<T>* __restrict__ X, int j0, int j1, float theta2,
                                T eps2, bool active, T yx, T yy, T yz, T& ax, T& ay, T& az,
                                unsigned& count, StackEntry* stk) {
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane & (S - 1);
  const int pbit = lane & ~(S - 1);  // bit of this lane's particle in the lane masks
  constexpr unsigned long long kRep = SlotMask<S>::v;
  const unsigned long long amask = __ballot(active) & kRep;
  T bx = 0, by = 0, bz = 0;  // this slot's share of the particle's sum
  if (amask != 0ull) {
    if (lane == 0) stk[0] = StackEntry{0, 1, amask};
    int sp = 1;
    while (sp > 0) {
      --sp;
      const int start = __builtin_amdgcn_readfirstlane(stk[sp].start);
      const int cnt = __builtin_amdgcn_readfirstlane(stk[sp].count);
      const unsigned long long emask =
          ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(stk[sp].mask >> 32)) << 32) |
          (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)stk[sp].mask);
      const bool mine = (emask >> pbit) & 1ull;
      BHWide nd = nodes[start + (slot < cnt ? slot : 0)];
      for (int base = 0; base < cnt; base += S) {
        const int k = base + slot;
        const bool has = k < cnt;
        // the next round's node is fetched before this one is processed
        const int kn = k + S < cnt ? k + S : (has ? k : 0);
        const BHWide nxt = nodes[start + kn];
        // some point of the range lies below this node
        const bool on = has && mine && nd.first < j1 && nd.last >= j0;
        const bool leaf = nd.child == -1;
        const bool twig = __float_as_uint(nd.l2) >> 31;
        const float l2 = fabsf(nd.l2);
        const T dx = (T)nd.cm.x - yx, dy = (T)nd.cm.y - yy, dz = (T)nd.cm.z - yz;
        const T r2 = dx * dx + dy * dy + dz * dz;
        const bool take =
            (sizeof(T) == 4 && leaf && nd.first == nd.last) || l2 < theta2 * (float)r2;
        {  // the node's term, kept only where this lane takes it and this range owns it
          const bool own = on && take && nd.first >= j0;
          if constexpr (POT) {
            const T s = rsqrt1_mass<T>((T)nd.cm.w, r2 + eps2);
            bx += own ? s : (T)0;
          } else {
            const T s = rsqrt3_mass<T>((T)nd.cm.w, r2 + eps2);
            const T sk = own ? s : (T)0;
            bx += dx * sk;
            by += dy * sk;
            bz += dz * sk;
          }
          count += own ? 1u : 0u;
        }
        const bool exact = leaf || twig;
        const bool open_pts = on && !take && exact;
        if (__ballot(open_pts) != 0ull) {
          const int p0 = max(nd.first, j0);
          const int np = open_pts ? min(nd.last, j1 - 1) - p0 + 1 : 0;
          for (int t = 0;; ++t) {  // every slot walks its own leaf
            const bool go = t < np;
            if (__ballot(go) == 0ull) break;
            if (go) {
              accum_point<T, POT>(X[p0 + t], yx, yy, yz, eps2, bx, by, bz);
              ++count;
            }
          }
        }
        const unsigned long long ob = __ballot(on && !take && !exact);
        if (ob != 0ull) {
          for (int s = 0; s < S; ++s) {  // the particles that opened slot s's node
            const unsigned long long om = (ob >> s) & kRep;
            if (om != 0ull && sp < kStack) {
              const int ch = __builtin_amdgcn_readlane(nd.child, s);
              if (lane == 0)
                stk[sp] = StackEntry{ch & ((1 << kChildShift) - 1),
                                     (int)((unsigned)ch >> kChildShift) + 1, om};
              ++sp;
            }
          }
        }
        nd = nxt;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < S; o <<= 1) {  // add the slots of each particle
    bx += __shfl_xor(bx, o, kWave);
    by += __shfl_xor(by, o, kWave);
    bz += __shfl_xor(bz, o, kWave);
  }
  ax += bx;
  ay += by;
  az += bz;
}


// ------------------------------------------------ Barnes-Hut, group traversal
// The particles of a wave (64 K, consecutive in the template's body-frame
// Morton order, hence spatially close) share one walk of the tree. A node is
// accepted for the whole group when l^2 < theta^2 d^2, with d the distance
// from its centre of mass to the group's bounding box: then l / r < theta
// holds for every particle of the group, so each accepted node is one that
// Alg. 2 would also accept (or reach only through an accepted ancestor), and
// the sum differs from the per-particle one only in nodes opened further,
// i.e. it is at least as close to the direct sum. The walk and the sum are
// separated:
//   - walk: lanes take up to 64 nodes at once from an LDS stack of child
//     blocks, test them, append accepted nodes (centre of mass + mass) and
//     the points of opened leaves and twigs to an LDS interaction list, and
//     push the child blocks of the other opened nodes;
//   - sum: whenever the list is nearly full, every lane evaluates its K
//     particles against the whole list (one broadcast LDS read per entry and
//     K Eq. (GAForce) terms), as in the direct sum.
// A heavy group's walk can be split over several waves by subtrees.
constexpr int kGList = 128;   // interaction-list entries per wave
constexpr int kGStack = 512;  // child-block entries per wave
// Stack entries kept free for a depth-first descent: every level of the tree
// (at most kQBits + 1 below the root) adds at most 7 entries to the stack.
constexpr int kGReserve = 8 * (kQBits + 2);

constexpr int kGRepMax = 8;   // replicas of a small group's particles over the lanes
struct GroupLds {
  float4 list[kGList + kGRepMax];  // slack for zero-mass padding to a multiple of the replicas
  int stk[kGStack];
  unsigned mark[kWave];            // nonzero where an entry starts: 1 (pops), 1 + its lane (point appends)
};

__device__ inline float wave_min_f(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ inline float wave_max_f(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Adds the list entries [0, cnt) to the K particles of this lane if `sel`.
// With KAHAN the list's sum is one tile, added to the total with Kahan
// compensation.
template <int K, bool KAHAN, bool PL = false>
__device__ inline void group_sum(const float4* list, int cnt, const float (&y)[K][3], float eps2,
                                 bool sel, float (&acc)[K][3], float (&cmp)[K][3]) {
  float t[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) t[k][a] = KAHAN ? 0.f : acc[k][a];
#pragma unroll 4
  for (int e = 0; e < cnt; ++e) {
    const float4 x = list[e];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float dx = x.x - y[k][0], dy = x.y - y[k][1], dz = PL ? 0.f : x.z - y[k][2];
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, PL ? eps2 : fmaf(dz, dz, eps2)));
      const float r = __builtin_amdgcn_rsqf(r2);
      const float s = x.w * r * (r * r);
      t[k][0] = fmaf(dx, s, t[k][0]);
      t[k][1] = fmaf(dy, s, t[k][1]);
      if (!PL) t[k][2] = fmaf(dz, s, t[k][2]);
    }
  }
  if (!sel) return;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (KAHAN) {
        const float u = t[k][a] - cmp[k][a], v = acc[k][a] + u;
        cmp[k][a] = (v - acc[k][a]) - u;
        acc[k][a] = v;
      } else {
        acc[k][a] = t[k][a];
      }
    }
}

// The same sum for a group held R > 1 times over the lanes: replica `rep`
// takes entries rep, rep + R, ... of the list (padded with zero-mass entries
// to a multiple of R, cnt).
template <int K, bool KAHAN, bool PL = false>
__device__ inline void group_sum_rep(const float4* list, int cnt, int rep, int R,
                                     const float (&y)[K][3], float eps2, bool sel,
                                     float (&acc)[K][3], float (&cmp)[K][3]) {
  float t[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) t[k][a] = KAHAN ? 0.f : acc[k][a];
  const int n = cnt / R;  // entries per replica, uniform
#pragma unroll 4
  for (int i = 0; i < n; ++i) {
    const float4 x = list[i * R + rep];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float dx = x.x - y[k][0], dy = x.y - y[k][1], dz = PL ? 0.f : x.z - y[k][2];
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, PL ? eps2 : fmaf(dz, dz, eps2)));
      const float r = __builtin_amdgcn_rsqf(r2);
      const float s = x.w * r * (r * r);
      t[k][0] = fmaf(dx, s, t[k][0]);
      t[k][1] = fmaf(dy, s, t[k][1]);
      if (!PL) t[k][2] = fmaf(dz, s, t[k][2]);
    }
  }
  if (!sel) return;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (KAHAN) {
        const float u = t[k][a] - cmp[k][a], v = acc[k][a] + u;
        cmp[k][a] = (v - acc[k][a]) - u;
        acc[k][a] = v;
      } else {
        acc[k][a] = t[k][a];
      }
    }
}

// Squared diagonal of the box of the lanes selected by `sel` (their valid
// particles), and the box itself, uniform over the wave. PL: a planar set,
// whose z is the same for every point (the box is flat).
template <int K, bool PL = false>
__device__ inline float group_box(const bool (&valid)[K], const float (&y)[K][3], bool sel,
                                  float (&lo)[3], float (&hi)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = __builtin_huge_valf();
    hi[a] = -__builtin_huge_valf();
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (sel && valid[k]) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], y[k][a]);
        hi[a] = fmaxf(hi[a], y[k][a]);
      }
    }
  float d2 = 0.f;
#pragma unroll
  for (int a = 0; a < (PL ? 2 : 3); ++a) {
    lo[a] = wave_min_f(lo[a]);
    hi[a] = wave_max_f(hi[a]);
    d2 = fmaf(hi[a] - lo[a], hi[a] - lo[a], d2);
  }
  if (PL) lo[2] = hi[2] = 0.f;  // unused
  return d2;
}

// Squared distance from c to the box [lo, hi] (0 inside); PL: in the plane
// of a planar set (x and y only).
template <bool PL = false>
__device__ inline float box_dist2(const float (&lo)[3], const float (&hi)[3], const float (&c)[3]) {
  float d2 = 0.f;
#pragma unroll
  for (int a = 0; a < (PL ? 2 : 3); ++a) {
    const float u = fmaxf(fmaxf(lo[a] - c[a], c[a] - hi[a]), 0.f);
    d2 = fmaf(u, u, d2);
  }
  return d2;
}

// Work split of one group's walk over nr waves (part r): nodes of more than
// kSplitPts points are walked by every part, and their accepted terms and leaf
// points belong to part 0; a node of at most kSplitPts points whose parent is
// larger (a frontier node) belongs, with its whole subtree, to part
// (index mod nr). The parts' sums add up to the group's sum, and the many
// small subtrees around a dense region spread evenly over the parts. Every
// part walks the shared nodes again, so the bound is set high: 128 points
// (LiDAR pair 106 against 115 us per force launch with 32; 64: 109, 256:
// 111, 512: 107; the mesh within 0.5% for all of them).
constexpr int kSplitPts = 128;
constexpr int kLargeParent = 1 << 28;  // stack entry flag: the block's parent is shared
constexpr int kIndexMask = kLargeParent - 1;

// The walk for a group: the particles of the lanes with `sel`, part r of nr.
template <int K, bool KAHAN, bool PL = false>
__device__ inline bool group_walk(const BHWide* __restrict__ nodes, int n_nodes,
                                  const float4* __restrict__ X, int n_points, int r, int nr,
                                  float theta2, float eps2, bool sel,
                                  int nvalid, int rep, int R, const float (&lo)[3],
                                  const float (&hi)[3],
                                  const float (&y)[K][3], float (&acc)[K][3],
                                  float (&cmp)[K][3], unsigned& count, unsigned& entries,
                                  GroupLds& g) {
  const int lane = threadIdx.x & (kWave - 1);
  bool ok = true;
  int cnt = 0;  // list entries
  int sp = 1;   // stack entries; the root is a block of one node at index 0
  {
    // The top two levels, decided up front: when the root, and then every
    // child of the root, is an internal node that is not a twig, holds more
    // than kSplitPts points (so every part walks it) and fails the MAC
    // against the group's box, the walk starts from their child blocks
    // instead: the same nodes are visited and accepted, two steps sooner.
    auto walked_open = [&](const BHWide& b) {
      const float c3[3] = {b.cm.x, b.cm.y, b.cm.z};
      const float d2 = box_dist2<PL>(lo, hi, c3);
      return b.child != -1 && !(__float_as_uint(b.l2) >> 31) && b.last - b.first + 1 > kSplitPts &&
             !(fabsf(b.l2) < theta2 * d2);
    };
    const BHWide root = nodes[0];
    int top = kLargeParent;
    if (walked_open(root)) {
      top = root.child | kLargeParent;
      const int nc = (int)((unsigned)root.child >> kChildShift) + 1;
      const BHWide ch = nodes[min((root.child & ((1 << kChildShift) - 1)) + lane, n_nodes - 1)];
      if (__ballot(lane < nc && !walked_open(ch)) == 0ull) {
        if (lane < nc) g.stk[lane] = ch.child | kLargeParent;
        sp = nc;
      }
    }
    if (sp == 1 && lane == 0) g.stk[0] = top;
  }
  auto flush = [&]() {
    if (R == 1) {
      group_sum<K, KAHAN, PL>(g.list, cnt, y, eps2, sel, acc, cmp);
    } else {
      const int padded = (cnt + R - 1) / R * R;  // zero-mass entries up to a multiple of R
      if (lane < padded - cnt) g.list[cnt + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
      group_sum_rep<K, KAHAN, PL>(g.list, padded, rep, R, y, eps2, sel, acc, cmp);
    }
    count += (sel && rep == 0) ? (unsigned)(cnt * nvalid) : 0u;
    entries += (unsigned)cnt;
    cnt = 0;
  };
  // pops whole child blocks from the top (at most 64 nodes, and only while the
  // stack stays below kGStack - kGReserve even if every node is opened), one
  // node per lane, and starts the loads of those nodes
  int T = 0, node = 0, pke = 0;
  BHWide nd;
  auto pop = [&]() {
    const int avail = min(sp, kWave);
    int ch = 0, c = 0;
    if (lane < avail) {
      ch = g.stk[sp - 1 - lane];
      c = (int)((unsigned)ch >> kChildShift) + 1;
    }
    const int incl = wave_incl_sum_dpp(c);
    const bool take = lane < avail && incl <= kWave &&
                      (lane == 0 || sp - (lane + 1) + incl <= kGStack - kGReserve);
    const int E = __popcll(__ballot(take));
    T = E > 0 ? __builtin_amdgcn_readlane(incl, E - 1) : 0;
    sp -= E;
    // this lane's node: entry e is the last whose first lane (incl - c) is at
    // or below the lane. The entries' first lanes are distinct and increase
    // with the entry, so e is the number of first lanes at or below this
    // lane, minus one: each entry marks its first lane, a ballot collects the
    // marks (relaxed atomics: the marks pass between lanes, so a lane's own
    // store must not be forwarded to its read)
    __hip_atomic_store(&g.mark[lane], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (lane < E)
      __hip_atomic_store(&g.mark[incl - c], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const bool first =
        __hip_atomic_load(&g.mark[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) != 0u;
    const unsigned long long starts = __ballot(first);
    const int e = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(starts >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((unsigned)starts, 0u)) +
                  (first ? 1 : 0) - 1;
    // entry lane: its first node minus its first lane (+ 64, >= 1) and the
    // shared-parent flag in bit 30, fetched by the node lanes in one move
    const int pk = ((ch & kIndexMask) - (incl - c) + kWave) | ((ch & kLargeParent) ? 1 << 30 : 0);
    pke = __shfl(pk, e < 0 ? 0 : e, kWave);
    node = min((pke & ((1 << 30) - 1)) - kWave + lane, n_nodes - 1);
    nd = nodes[lane < T ? node : 0];
  };
  pop();
  while (T > 0) {
    const bool act = lane < T;
    const bool shared = nd.last - nd.first + 1 > kSplitPts;
    const bool frontier = !shared && (pke & (1 << 30));
    const bool on = act && (!frontier || (node & (nr - 1)) == r);  // nr: a power of two
    const bool mine = !shared || r == 0;  // owns the node's own term or points
    const bool leaf = nd.child == -1;
    const bool twig = __float_as_uint(nd.l2) >> 31;
    const float c3[3] = {nd.cm.x, nd.cm.y, nd.cm.z};
    const float d2 = box_dist2<PL>(lo, hi, c3);
    const bool accept = on && ((leaf && nd.first == nd.last) || fabsf(nd.l2) < theta2 * d2);
    const bool own = accept && mine;
    const bool pts = on && !accept && (leaf || twig) && mine;
    const bool inner = on && !accept && !leaf && !twig;
    // push the child blocks of the opened internal nodes
    const unsigned long long im = __ballot(inner);
    if (inner) {
      const int pos = sp + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(im >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)im, 0u));
      if (pos < kGStack) g.stk[pos] = nd.child | (shared ? kLargeParent : 0);
    }
    sp += __popcll(im);
    if (sp > kGStack) {
      ok = false;
      sp = kGStack;
    }
    // append the accepted nodes (cnt <= kGList - 64 here)
    const unsigned long long om = __ballot(own);
    if (own) {
      const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(om >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned)om, 0u));
      g.list[pos] = nd.cm;
    }
    cnt += __popcll(om);
    // append the points of opened leaves and twigs, 64 at a time
    const int p0 = nd.first;
    const int np = pts ? nd.last - p0 + 1 : 0;
    if (__ballot(np > 0) != 0ull) {
      const int pincl = wave_incl_sum_dpp(np);
      const int P = __builtin_amdgcn_readlane(pincl, kWave - 1);
      const int pex = pincl - np;          // first list slot of this lane's points
      const int off = p0 - pex;            // point index = slot + off for this lane's slots
      const unsigned long long has = __ballot(np > 0);
      for (int base = 0; base < P; base += kWave) {
        if (cnt > kGList - kWave) flush();
        const int k = base + lane;
        // owner of slot k: the last lane with points whose first slot is at or
        // below k; slot `base` may continue a lane that started earlier
        const unsigned long long before = __ballot(np > 0 && pex <= base) & has;
        const int carry = 63 - __builtin_clzll(before);
        __hip_atomic_store(&g.mark[lane], lane == 0 ? (unsigned)carry + 1u : 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (np > 0 && pex > base && pex < base + kWave)
          __hip_atomic_store(&g.mark[pex - base], (unsigned)lane + 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WAVEFRONT);
        const int o = (int)wave_incl_max_u32(__hip_atomic_load(&g.mark[lane], __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_WAVEFRONT)) - 1;
        const int ooff = __shfl(off, o, kWave);
        if (k < P) g.list[cnt + lane] = X[min(max(k + ooff, 0), n_points - 1)];
        cnt += min(kWave, P - base);
      }
    }
    // the next step's nodes are requested before the list is summed, so
    // their load latency overlaps the arithmetic
    if (sp > 0) {
      pop();
    } else {
      T = 0;
    }
    if (cnt > kGList - kWave) flush();
  }
  if (cnt > 0) flush();
  return ok;
}

// Lane l holds particles K p .. K p + K - 1 of the wave's group, p = l mod
// (64 / R): with R > 1 (K = 1, groups of at most 64 / R particles) every
// particle is held by R lanes that split the list between them. The walk is
// part r of nr (see kSplitPts); `entries`
// (uniform) receives the number of list entries evaluated. Returns false if
// the stack overflowed (never for trees of depth at most kQBits + 1;
// the sum is then incomplete).
template <int K, bool KAHAN, bool PL = false>
__device__ inline bool bh_group(const BHWide* __restrict__ nodes, int n_nodes,
                                const float4* __restrict__ X, int n_points, int r, int nr, int R,
                                float theta2, float eps2,
                                const bool (&valid)[K], const float (&y)[K][3],
                                float (&acc)[K][3], unsigned& count, unsigned& entries,
                                GroupLds& g) {
  int nvalid = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) nvalid += valid[k] ? 1 : 0;
  if (__ballot(nvalid > 0) == 0ull) return true;
  float lo[3], hi[3];
  group_box<K, PL>(valid, y, true, lo, hi);
  float cmp[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) cmp[k][a] = 0.f;
  const int rep = (int)(threadIdx.x & (kWave - 1)) / (kWave / R);
  const bool ok = group_walk<K, KAHAN, PL>(nodes, n_nodes, X, n_points, r, nr, theta2, eps2, true,
                                       nvalid, rep, R, lo, hi, y, acc, cmp, count, entries, g);
  if (R > 1) {  // add the replicas' partial sums
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float v = KAHAN ? acc[k][a] - cmp[k][a] : acc[k][a];
        for (int o = kWave / R; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
        acc[k][a] = v;
      }
  }
  return ok;
}

}  // namespace fga
