// Internal declarations shared by the HIP translation units of libfga.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fga.h"

namespace fga {

constexpr int kBlock = 256;  // threads per block for every kernel
constexpr int kWave = 64;    // CDNA wavefront width
constexpr int kQBits = 20;   // octree depth limit: 20 octal digits, 60-bit Morton codes

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
#define FGA_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::fga::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      return e_ == hipErrorOutOfMemory ? FGA_E_NOMEM : FGA_E_DEVICE;                   \
    }                                                                                  \
  } while (0)
#define FGA_TRY(call)                \
  do {                               \
    fga_status s_ = (call);          \
    if (s_ != FGA_OK) return s_;     \
  } while (0)

// ------------------------------------------------- caching device allocator
// pool.hip: device blocks cached in size classes and reused once the work
// queued on them before their release has finished. pool_alloc returns nullptr
// (error message set) on failure; pool_free takes the last stream that used
// the block.
void* pool_alloc(size_t bytes, hipStream_t s);
void pool_free(void* p, hipStream_t s);
fga_status pool_trim();
template <typename P>
inline fga_status pool_get(P** out, size_t bytes, hipStream_t s) {
  void* p = pool_alloc(bytes, s);
  if (!p) return FGA_E_NOMEM;
  *out = (P*)p;
  return FGA_OK;
}

// --------------------------------------------------------- vector helpers
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec4_t = typename Vec4<T>::type;

template <typename T> __host__ __device__ inline vec4_t<T> make4(T a, T b, T c, T d);
template <> __host__ __device__ inline float4 make4<float>(float a, float b, float c, float d) {
  return make_float4(a, b, c, d);
}
template <> __host__ __device__ inline double4 make4<double>(double a, double b, double c, double d) {
  return make_double4(a, b, c, d);
}

// --------------------------------------------------------------- the state
// FP64 rigid state of one registration pair, resident in device memory.
// Template particle i sits at y_i = R q_i + mu, with q_i its centred
// body-frame coordinate (normalised template minus its mean mu0), so the
// accumulated transform of Alg. 2 is Y_k = R Yn + t with t = mu - R mu0.
struct RigidState {
  double R[9];    // accumulated rotation (row-major)
  double t[3];    // accumulated translation, normalised frame
  double mu[3];   // current template centroid
  double A[9];    // rigid velocity field v_i = A q_i + b of the last step
  double b[3];
  double S0[9];   // sum_i q_i q_i^T
  double mu0[3];  // mean of the normalised template
  double Vw[9];   // right singular vectors of the last Kabsch matrix (start of the next SVD)
  double dT2;     // ||T_k - T_{k-1}||_F^2 of the last step
  double tol;     // convergence tolerance (<= 0: never converged)
  double rank_tol;  // singular-value ratio below which C counts as rank deficient
  long long interactions;  // running count of force interactions
  int iter;
  int converged;
  int m;          // template particles
  int flags;      // bit 0: degenerate Kabsch (rank(C) < 2) seen; bit 1: traversal stack overflow
  int max_iter;
  int dims;       // 3, or 2 for planar point sets (z = const): the rigid step is then the 2 x 2 Kabsch
  float fR[9], fmu[3], fA[9], fb[3];  // FP32 copies read by the FP32 force kernels
};

// Iteration constants of one registration (identical for all pairs of a batch).
struct IterConsts {
  double G, eps2, dt, theta2;
  float fG, feps2, fdt, ftheta2;
  int damping;   // fga_damping
  int velocity;  // fga_velocity
  int prec;      // fga_precision
  int pad_;
};

// Barnes-Hut node, 32 bytes, depth-first preorder. A node's first child is the
// next node; `skip` is the index right after its subtree; a leaf has
// skip == index + 1. Points [first, last] (inclusive) of the Morton-sorted
// reference lie in the node's cell.
struct alignas(16) BHNode {
  float4 cm;   // centre of mass (x, y, z) and mass
  int skip;
  int first;
  int last;
  float l2;    // squared box diagonal of the cell (Alg. 1: l = ||X_max - X_min||);
               // the sign bit marks a twig (an internal node whose children are
               // all singleton leaves)
};

// The same tree laid out for the traversal kernels: the children of every
// internal node are stored contiguously (a "child block"), blocks of the
// parents in preorder, so opening a node fetches all its children at once.
// 32 bytes. Indices are local to the node's segment.
struct alignas(16) BHWide {
  float4 cm;   // centre of mass (x, y, z) and mass
  int first;   // points [first, last] of the Morton-sorted reference
  int last;
  int child;   // internal: index of the first child | (children - 1) << 29 (as unsigned
               // bits; the index is below 2^28, so the field is never -1); leaf: -1
  float l2;    // squared box diagonal; sign bit: twig (all children singleton leaves)
};
constexpr int kChildShift = 29;

// Completion of an iteration: every item writes one row of kPartialRow
// doubles (12 partial moments and its interaction count); the reduction
// launch sums kReduceRows rows per block, and its last block the block
// results. A pair with n items needs (n + chunks) rows and one counter (zero
// at rest).
constexpr int kPartialRow = 13;

// Waves per SIMD the group-walk kernels are compiled for (their register
// budget); the host sizes the heavy-group split by it.
constexpr int kGroupWavesPerSimd = 6;
constexpr int kReduceRows = 256;
__host__ __device__ inline int completion_chunks(int n_items) {
  return (n_items + kReduceRows - 1) / kReduceRows;
}
// Blocks of the reduction launch: one block sums up to kOneBlockRows rows by
// itself (no second level, no cross-block completion); more rows take one
// block per kReduceRows rows. Never more than completion_chunks(n_items).
constexpr int kOneBlockRows = 4096;
__host__ __device__ inline int reduce_blocks(int n_items) {
  return n_items <= kOneBlockRows ? 1 : completion_chunks(n_items);
}

// Geometry of one registration pair on the device, for the iteration kernels.
struct PairDev {
  const void* X;        // reference (x, y, z, mass) as vec4, normalised; Morton-sorted for BH
  const void* Q;        // template (q_x, q_y, q_z, c) as vec4 in the body frame; c = damping coeff
  const BHWide* nodes;  // BH nodes in child-block layout, or nullptr for the direct sum
  void* V;              // per-particle velocities (particle mode), m x 3 of T, else nullptr
  RigidState* st;
  double* partial;      // (n_items + chunks) x kPartialRow partial moments and counts
  unsigned* done;       // completion counter of the reduction launch
  int n, m;
  int n_nodes;
  int jr;               // reference ranges per template tile
  int n_items;          // template tiles x jr
  int tile;             // template particles per tile (kBlock / slots)
  int slots;            // lanes per template particle in the Barnes-Hut traversal (1, 2, 4, 8)
  int group;            // 0: per-particle traversal; K > 0: group traversal, K particles per lane
  const int4* witems;   // group walk, one per wave: (first particle, count <= 64 K,
                        // part r | parts << 8 (a power of two), group) of the wave's particles
  unsigned* gcost;      // optional: list entries evaluated per group are added here
  int n_groups;
  int n_witems;
  int planar = 0;       // 1: planar sets (z constant): the group walk skips the z terms
};


// ------------------------------------------------------------ declarations
// prep.hip: normalisation, masses and packing (Appendix A; Eq. NIV)
struct CloudIn {
  const void* p;  // n x 3 row-major device array (dtype of the call)
  int64_t n;
  const int64_t* lm = nullptr;  // host: indices of its landmark points (RBF masses)
  int n_lm = 0;
};
struct PrepOut {
  void* X;          // packed reference vec4 (n_x)
  void* Q;          // packed template vec4 (n_y)
  RigidState* st;   // initialised rigid state
};
struct NormInfo {   // host copy of the Appendix A normalisation
  double xbar[3], ybar[3], l, r, a, b;
};
// dims = 2: the clouds are planar point sets embedded at z = 0 (NIV on the
// planar lattice with disc areas; 2 x 2 Kabsch steps)
fga_status prep_pairs(int npairs, const CloudIn* X, const CloudIn* Y, fga_dtype dt,
                      const fga_params& p, PrepOut* out, NormInfo* info, hipStream_t s,
                      int dims = 3);
fga_status masses_only(const void* pts, fga_dtype dt, int64_t n, const int64_t* lm, int n_lm,
                       const fga_params& p, int norm, void* out, hipStream_t s);
constexpr int kMaxLandmarkPairs = 64;  // landmark correspondences per registration

// tree.hip: Morton codes, LDS radix sort, octree build
struct TreeSeg {       // one reference cloud in a concatenated packed array
  int64_t off, n;
};
struct TreeOut {
  BHNode* nodes;       // all segments' nodes, segment-contiguous
  int* node_off;       // host: first node of each segment (nseg + 1 entries)
  int* order;          // device: sorted position -> input position (n total)
  int max_depth;
  int leaves;
};
template <typename T>
fga_status build_trees(int nseg, const TreeSeg* segs, void* Xpacked, int64_t ntotal,
                       int leaf_size, BHNode** nodes_out, int* node_off_host, int** order_out,
                       int* stats_host, hipStream_t s);
// Child-block layout of preorder trees (all segments); node_off_host bounds
// each segment's nodes, which keep their count and offsets.
fga_status relayout_wide(const BHNode* pre, int total, int nseg, const int* node_off_host,
                         BHWide** out, hipStream_t s);
template <typename T>
fga_status sort_points_morton(int nseg, const TreeSeg* segs, void* Q, int64_t ntot, int* perm,
                              hipStream_t s);

// groups.hip: group tables of the group walk over Morton-ordered templates
// Q (nseg segments at off[k], m[k] particles): aligned blocks of G particles
// cut into runs whose bounding-box diagonal stays within f times the median
// block diagonal of the segment (f = 0: one run per block). out[k] receives
// segment k's runs as (first particle, count), first relative to off[k].
fga_status device_groups(const float4* Q, int nseg, const int64_t* off, const int64_t* m, int G,
                         double f, std::vector<std::vector<int2>>& out, hipStream_t s);
// The same for one segment of m x 3 FP32 points (device), in their order.
fga_status device_groups_xyz(const float* Y, int64_t m, int G, double f, std::vector<int2>& out,
                             hipStream_t s);

// iter.hip: force-only evaluation (fga_forces)
int direct_ranges(int64_t m, int64_t n);
template <typename T>
fga_status forces_direct(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                         const void* mY, const fga_params& p, void* F, hipStream_t s);
// Bytes of device scratch the direct sum needs (packed reference, then the
// per-range partial forces), and its launches into caller-provided scratch
// (aligned to 256 bytes); queues the work without waiting for it.
size_t forces_direct_scratch(int64_t m, int64_t n, bool f64);
template <typename T>
fga_status forces_direct_into(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                              const void* mY, const fga_params& p, void* F, void* scratch,
                              hipStream_t s);
template <typename T>
fga_status forces_bh_tree(const void* Y, int64_t m, const int* yorder, const BHWide* nodes,
                          int n_nodes, const void* Xs, int64_t n, double theta,
                          const fga_params& p, const void* mY, void* F, long long* interactions,
                          hipStream_t s);
template <typename T>
fga_status pack_points(const void* X, const void* mX, int64_t n, void* out, hipStream_t s);
// iter.hip: Plummer energy (fga_energy), direct and through the per-particle walk
template <typename T>
fga_status energy_direct(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                         const void* mY, const fga_params& p, double* E_host, hipStream_t s);
template <typename T>
fga_status energy_bh_tree(const void* Y, int64_t m, const int* yorder, const BHWide* nodes,
                          const void* Xs, double theta, const fga_params& p, const void* mY,
                          double* E_host, long long* interactions, hipStream_t s);
// iter.hip: planar point sets (n x 2) to z = 0 embedded n x 3 and back
fga_status embed_planar(const void* in, int64_t n, bool f64, void* out, hipStream_t s);
fga_status take_planar(const void* in, int64_t n, bool f64, void* out, hipStream_t s);

// iter.hip: one iteration as two launches (pose, forces, ODE and per-block
// moments; then the ordered moment sum and the Kabsch step)
template <typename T>
fga_status launch_iteration(const PairDev& pd, const IterConsts& c, hipStream_t s,
                            hipEvent_t between = nullptr);
template <typename T>
fga_status launch_batch_iteration(const PairDev* pairs_dev, int npairs, int reduce_blocks,
                                  const int2* items, int n_items, unsigned* queue, int n_blocks,
                                  const IterConsts& c, hipStream_t s, bool bh, bool group);


}  // namespace fga
