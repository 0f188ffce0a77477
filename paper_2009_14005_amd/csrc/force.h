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

// One exact term of Eq. (GAForce) (per unit G and template mass).
template <typename T>
__device__ inline void accum_point(const vec4_t<T>& x, T yx, T yy, T yz, T eps2, T& ax, T& ay,
                                   T& az) {
  const T ex = x.x - yx, ey = x.y - yy, ez = x.z - yz;
  const T s = rsqrt3_mass<T>(x.w, ex * ex + ey * ey + ez * ez + eps2);
  ax += ex * s;
  ay += ey * s;
  az += ez * s;
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
  unsigned n = wave_min_u32(next);
  if (n >= uend) return;
  BHNode nd = nodes[n];
  // a correct walk visits every node at most once; the cap only bounds the loop
  for (unsigned visits = 0; visits <= uend; ++visits) {
    // the next node in preorder is the most likely successor: fetch it early
    const unsigned nn = n + 1 < uend ? n + 1 : n;
    const BHNode ahead = nodes[nn];
    const bool here = next == n;
    const unsigned after = (unsigned)nd.skip > n ? (unsigned)nd.skip : n + 1;
    if (nd.first < j1 && nd.last >= j0) {  // some point of the range lies below this node
      const bool leaf = (unsigned)nd.skip == n + 1;
      // A twig is an internal node whose children are all singleton leaves
      // (its subtree holds one node per point). Opening it evaluates every
      // child exactly, whatever the children's own MAC outcome, so it is
      // walked like a leaf: the same terms without visiting the children.
      const bool twig = __float_as_uint(nd.l2) >> 31;
      const float l2 = fabsf(nd.l2);
      const T dx = (T)nd.cm.x - yx, dy = (T)nd.cm.y - yy, dz = (T)nd.cm.z - yz;
      const T r2 = dx * dx + dy * dy + dz * dz;
      // singleton leaves are taken directly in FP32 lanes (the node is the point)
      const bool take_node =
          (sizeof(T) == 4 && leaf && nd.first == nd.last) || l2 < theta2 * (float)r2;
      if (here && take_node && nd.first >= j0) {  // this range owns the node
        const T s = rsqrt3_mass<T>((T)nd.cm.w, r2 + eps2);
        ax += dx * s;
        ay += dy * s;
        az += dz * s;
        ++count;
      }
      const bool exact = leaf || twig;
      const bool open_pts = here && !take_node && exact;
      if (here) next = (take_node || exact) ? after : n + 1;
      if (exact && __ballot(open_pts) != 0ull) {
        const int p0 = max(nd.first, j0), p1 = min(nd.last, j1 - 1);
        int p = p0;
        for (; p + 3 <= p1; p += 4) {  // four points per round: loads issued together
          const vec4_t<T> x0 = X[p], x1 = X[p + 1], x2 = X[p + 2], x3 = X[p + 3];
          if (open_pts) {
            accum_point<T>(x0, yx, yy, yz, eps2, ax, ay, az);
            accum_point<T>(x1, yx, yy, yz, eps2, ax, ay, az);
            accum_point<T>(x2, yx, yy, yz, eps2, ax, ay, az);
            accum_point<T>(x3, yx, yy, yz, eps2, ax, ay, az);
            count += 4;
          }
        }
        for (; p <= p1; ++p) {
          const vec4_t<T> x = X[p];
          if (open_pts) {
            accum_point<T>(x, yx, yy, yz, eps2, ax, ay, az);
            ++count;
          }
        }
      }
    } else if (here) {
      next = after;
    }
    // successor: n + 1 whenever some lane opened n, else the smallest wanted index
    if (__ballot(next == n + 1) != 0ull) {
      n = n + 1;
      if (n >= uend) break;
      nd = ahead;
    } else {
      n = wave_min_u32(next);
      if (n >= uend) break;
      nd = nodes[n];
    }
  }
}

}  // namespace fga
