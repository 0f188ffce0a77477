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
__device__ inline void direct_f64(const double4* __restrict__ X, int j0, int j1, double yx,
                                  double yy, double yz, double eps2, double& ax, double& ay,
                                  double& az) {
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    const double4 x = X[j];
    const double dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
    const double r2 = dx * dx + dy * dy + dz * dz + eps2;
    const double s = x.w / (r2 * sqrt(r2));
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
  return m / (r2 * sqrt(r2));
}

// ------------------------------------------------------------- Barnes-Hut
// Wavefront-cooperative traversal with per-lane decisions. Nodes are in
// depth-first preorder, so every lane's walk is a sequence of increasing node
// indices: after visiting node n a lane continues at n + 1 (node opened) or
// at skip(n) (node accepted, leaf done, or subtree irrelevant). The wave
// visits the smallest index any lane wants next; lanes that do not want that
// node idle. Each lane therefore makes exactly the accept/open decisions of
// Alg. 2 for its own particle, whatever its neighbours do.
//
// A traversal may be restricted to reference points [j0, j1): subtrees outside
// the range are skipped, an accepted node is counted only by the range that
// holds its first point, and an opened leaf contributes only its points inside
// the range. The ranges of one particle together give exactly its Alg. 2 sum.
//
// theta2 = theta^2; a node is accepted when l^2 < theta^2 r^2 (Eq. MAC with
// l / r < theta; r = 0 never accepts). Singleton leaves are always evaluated
// directly: the node holds the point and its mass, so acceptance and opening
// give the same term.
template <typename T>
__device__ inline void bh_accum(const BHNode* __restrict__ nodes,
                                const vec4_t<T>* __restrict__ X, int root, int end, int j0,
                                int j1, float theta2, T eps2, bool active, T yx, T yy, T yz,
                                T& ax, T& ay, T& az, unsigned& count) {
  unsigned next = active ? (unsigned)root : 0xFFFFFFFFu;
  const unsigned uend = (unsigned)end;
  // a correct walk visits every node at most once; the cap only bounds the loop
  for (unsigned visits = 0; visits <= uend; ++visits) {
    const unsigned n = wave_min_u32(next);
    if (n >= uend) break;
    const BHNode nd = nodes[n];
    const bool here = next == n;
    const unsigned after = (unsigned)nd.skip > n ? (unsigned)nd.skip : n + 1;
    if (nd.first >= j1 || nd.last < j0) {  // no point of the range below this node
      if (here) next = after;
      continue;
    }
    const bool leaf = (unsigned)nd.skip == n + 1;
    const bool single = leaf && nd.first == nd.last;
    bool open_leaf = false;
    if (here) {
      const T dx = (T)nd.cm.x - yx, dy = (T)nd.cm.y - yy, dz = (T)nd.cm.z - yz;
      const T r2 = dx * dx + dy * dy + dz * dz;
      const bool direct_single = single && sizeof(T) == 4;
      if (direct_single || nd.l2 < theta2 * (float)r2) {
        if (nd.first >= j0) {  // this range owns the node
          const T s = rsqrt3_mass<T>((T)nd.cm.w, r2 + eps2);
          ax += dx * s;
          ay += dy * s;
          az += dz * s;
          ++count;
        }
        next = after;
      } else if (leaf) {
        open_leaf = true;
        next = after;
      } else {
        next = n + 1;
      }
    }
    if (leaf && __ballot(open_leaf) != 0ull) {
      const int p0 = max(nd.first, j0), p1 = min(nd.last, j1 - 1);
      for (int p = p0; p <= p1; ++p) {
        const vec4_t<T> x = X[p];
        if (open_leaf) {
          const T dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
          const T s = rsqrt3_mass<T>(x.w, dx * dx + dy * dy + dz * dz + eps2);
          ax += dx * s;
          ay += dy * s;
          az += dz * s;
          ++count;
        }
      }
    }
  }
}

}  // namespace fga
