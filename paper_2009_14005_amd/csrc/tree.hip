// Step a1 of the hot path, once per registration: the Barnes-Hut tree of
// Alg. 1 on the static reference, built bottom-up from Morton order.
//
//  1. Bounding box of each reference cloud (tight box, Alg. 1).
//  2. Per-axis quantisation q = min(floor(2^20 (x - lo) / (hi - lo)), 2^20 - 1)
//     in FP64, interleaved into a 60-bit Morton code: octal digit k (k = 0 is
//     the root split) is the cell a point enters at depth k + 1, so sorting by
//     code orders points by their cells at every depth.
//  3. Stable LSD radix sort (8-bit digits) of (code, index) with LDS ranking.
//     Segments (one per registration pair) are sorted together: tiles never
//     straddle a segment and the digit offsets are scanned in
//     (segment, digit, tile) order.
//  4. Octree topology from the sorted codes (a Karras-style construction on
//     octal digits). For adjacent points k, k+1 with d common leading digits
//     (d < 20) the cell at depth d containing both branches. That cell's
//     points form the maximal run around k whose codes share d digits; it is
//     found with two exponential/binary searches. Among the separators of one
//     cell, the leftmost one emits the node. Runs of identical codes are
//     depth-20 leaves (singletons when the run has one point).
//     Chains of single-child cells are represented by their deepest cell:
//     they hold the same points (same mass and centre of mass) and the
//     deepest has the smallest diagonal, so it is accepted by the MAC exactly
//     when some cell of the chain would be, with the same force.
//  5. Depth-first preorder without a tree walk: all nodes whose point range
//     starts at point p form a chain ordered by depth, so the preorder index
//     is (number of nodes starting before p) + (rank of the node's depth in
//     that chain), and the node after a subtree is the first node starting
//     after its last point.
//  6. Mass and centre of mass of every node from FP64 prefix sums of m and
//     m * x over the sorted points (the sum over the node's contiguous range).
#include <math.h>

#include <vector>

#include "common.h"
#include "reduce.h"

namespace fga {
namespace {

constexpr int kSortItems = 16;                    // keys per thread per tile
constexpr int kSortTile = kBlock * kSortItems;    // keys per tile
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

using u64 = unsigned long long;

struct SortTile {
  int seg;
  int tile_in_seg;
  int ntiles_seg;
  int hbase;      // first histogram entry of the tile's segment: 256 * (tiles before it)
  int64_t start;  // first key
  int count;
  int pad_;
};

struct SegBox {   // per segment, device
  double lo[3], hi[3];  // tight box (exact: minima and maxima of the stored values)
  double lroot;         // diagonal of the root box
};

// ------------------------------------------------------------ bounding box
template <typename T>
__global__ __launch_bounds__(kBlock) void k_box_part(const vec4_t<T>* X, const SortTile* tiles,
                                                     double* part) {
  __shared__ double lds[6 * kBlock / kWave];
  const SortTile t = tiles[blockIdx.x];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = threadIdx.x; k < t.count; k += kBlock) {
    const vec4_t<T> p = X[t.start + k];
    mn[0] = fmin(mn[0], (double)p.x);
    mn[1] = fmin(mn[1], (double)p.y);
    mn[2] = fmin(mn[2], (double)p.z);
    mx[0] = fmax(mx[0], (double)p.x);
    mx[1] = fmax(mx[1], (double)p.y);
    mx[2] = fmax(mx[2], (double)p.z);
  }
  block_minmax<3>(mn, mx, lds);
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) {
      part[6 * blockIdx.x + a] = mn[a];
      part[6 * blockIdx.x + 3 + a] = mx[a];
    }
}

// One wave per segment: lane j takes tiles j, j + 64, ... of the segment.
__global__ __launch_bounds__(kWave) void k_box_fin(const double* part, const int* seg_tile0,
                                                   int nseg, SegBox* box) {
  const int s = blockIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int t = seg_tile0[s] + (int)threadIdx.x; t < seg_tile0[s + 1]; t += kWave)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], part[6 * t + a]);
      hi[a] = fmax(hi[a], part[6 * t + 3 + a]);
    }
  for (int o = kWave / 2; o > 0; o >>= 1)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], __shfl_xor(lo[a], o, kWave));
      hi[a] = fmax(hi[a], __shfl_xor(hi[a], o, kWave));
    }
  if (threadIdx.x != 0) return;
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    box[s].lo[a] = lo[a];
    box[s].hi[a] = hi[a];
    d2 += (hi[a] - lo[a]) * (hi[a] - lo[a]);
  }
  box[s].lroot = sqrt(d2);
}

// ------------------------------------------------------------ Morton codes
__device__ inline unsigned quant20(double x, double lo, double hi) {
  const double ext = hi - lo;
  if (!(ext > 0.0)) return 0u;
  const double cells = 1048576.0;  // 2^20
  const double f = floor((x - lo) / ext * cells);
  return f >= cells - 1.0 ? 1048575u : (f <= 0.0 ? 0u : (unsigned)f);
}

__device__ inline u64 spread3(unsigned v) {  // bit b of v -> bit 3b
  u64 x = v & 0xFFFFFu;
  x = (x | (x << 32)) & 0x1F00000000FFFFull;
  x = (x | (x << 16)) & 0x1F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_morton(const vec4_t<T>* X, const SortTile* tiles,
                                                   const SegBox* box, u64* keys, unsigned* vals) {
  const SortTile t = tiles[blockIdx.x];
  const SegBox b = box[t.seg];
  for (int k = threadIdx.x; k < t.count; k += kBlock) {
    const int64_t i = t.start + k;
    const vec4_t<T> p = X[i];
    const unsigned qx = quant20((double)p.x, b.lo[0], b.hi[0]);
    const unsigned qy = quant20((double)p.y, b.lo[1], b.hi[1]);
    const unsigned qz = quant20((double)p.z, b.lo[2], b.hi[2]);
    keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    vals[i] = (unsigned)i;
  }
}

// ------------------------------------------------------------ radix sort
__global__ __launch_bounds__(kBlock) void k_rs_hist(const u64* keys, const SortTile* tiles,
                                                    int shift, unsigned* hist) {
  __shared__ unsigned h[256];
  const SortTile t = tiles[blockIdx.x];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < t.count; k += kBlock)
    atomicAdd(&h[(unsigned)(keys[t.start + k] >> shift) & 255u], 1u);
  __syncthreads();
  hist[t.hbase + threadIdx.x * t.ntiles_seg + t.tile_in_seg] = h[threadIdx.x];
}

// Exclusive scan of n unsigned values in place by one block.
__global__ __launch_bounds__(1024) void k_scan_u32_1block(unsigned* v, int n) {
  __shared__ unsigned lds[1024 / kWave];
  const int per = (n + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(n, b + per);
  unsigned s = 0;
  for (int i = b; i < e; ++i) s += v[i];
  // block exclusive scan of s (1024 threads)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned inc = s;
  for (int o = 1; o < 64; o <<= 1) {
    unsigned y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  unsigned base = 0;
  for (int ww = 0; ww < w; ++ww) base += lds[ww];
  unsigned run = base + inc - s;
  for (int i = b; i < e; ++i) {
    const unsigned x = v[i];
    v[i] = run;
    run += x;
  }
}

// Exclusive scan of n unsigned values in place over many blocks: each block
// scans a tile of kHScanTile values (kHScanItems contiguous ones per thread) and
// writes its total; one block scans the totals (k_scan_u32_1block); a third
// launch adds each tile's offset. Three short launches instead of one block
// walking the whole histogram (the radix sort's histograms have 256 entries
// per tile of keys: 65,536 for a million points).
constexpr int kHScanItems = 16;
constexpr int kHScanTile = kBlock * kHScanItems;
__global__ __launch_bounds__(kBlock) void k_scan_tile(unsigned* v, int n, unsigned* tot) {
  __shared__ unsigned lds[kBlock / kWave];
  const int base = blockIdx.x * kHScanTile + (int)threadIdx.x * kHScanItems;
  unsigned x[kHScanItems];
  unsigned s = 0;
#pragma unroll
  for (int k = 0; k < kHScanItems; ++k) {
    x[k] = base + k < n ? v[base + k] : 0u;
    s += x[k];
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  unsigned inc = s;
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  unsigned run = inc - s;
  for (int ww = 0; ww < w; ++ww) run += lds[ww];
  if (threadIdx.x == kBlock - 1) tot[blockIdx.x] = run + s;
#pragma unroll
  for (int k = 0; k < kHScanItems; ++k) {
    if (base + k < n) v[base + k] = run;
    run += x[k];
  }
}
__global__ __launch_bounds__(kBlock) void k_scan_add(unsigned* v, int n, const unsigned* tot) {
  const unsigned add = tot[blockIdx.x];
  for (int k = 0; k < kHScanItems; ++k) {
    const int i = blockIdx.x * kHScanTile + k * kBlock + (int)threadIdx.x;
    if (i < n) v[i] += add;
  }
}

__global__ __launch_bounds__(kBlock) void k_rs_scatter(const u64* kin, const unsigned* vin,
                                                       const SortTile* tiles, int shift,
                                                       const unsigned* offs, u64* kout,
                                                       unsigned* vout) {
  __shared__ unsigned s_off[256];
  __shared__ unsigned s_base[256];
  __shared__ unsigned s_wc[kBlock / kWave][256];
  const SortTile t = tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  s_off[tid] = offs[t.hbase + tid * t.ntiles_seg + t.tile_in_seg];
  s_base[tid] = 0;
  const u64 lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int r = 0; r < kSortItems; ++r) {
    const int k = r * kBlock + tid;
    const bool valid = k < t.count;
    u64 key = 0;
    unsigned val = 0, dig = 0;
    if (valid) {
      key = kin[t.start + k];
      val = vin[t.start + k];
      dig = (unsigned)(key >> shift) & 255u;
    }
#pragma unroll
    for (int ww = 0; ww < kBlock / kWave; ++ww) s_wc[ww][tid] = 0;
    __syncthreads();
    u64 peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool b = (dig >> bit) & 1u;
      const u64 m = __ballot(b);
      peers &= b ? m : ~m;
    }
    const unsigned rank = (unsigned)__popcll(peers & lt);
    if (valid && rank == 0) s_wc[w][dig] = (unsigned)__popcll(peers);
    __syncthreads();
    if (valid) {
      unsigned pos = s_off[dig] + s_base[dig] + rank;
      for (int ww = 0; ww < w; ++ww) pos += s_wc[ww][dig];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    unsigned add = 0;
#pragma unroll
    for (int ww = 0; ww < kBlock / kWave; ++ww) add += s_wc[ww][tid];
    s_base[tid] += add;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather4(const vec4_t<T>* in, const unsigned* perm,
                                                    int64_t n, vec4_t<T>* out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

// ------------------------------------------------------------ octree topology
__device__ inline int lcp_digits(u64 a, u64 b) {
  const u64 x = a ^ b;
  if (x == 0) return kQBits;
  const int hb = 63 - __clzll((long long)x);
  return (kQBits - 1) - hb / 3;
}

struct SegRange {
  int64_t s0, s1;  // sorted positions [s0, s1) of one segment
};

__device__ inline int find_seg(const SegRange* sr, int nseg, int64_t i) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sr[mid].s0 <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// smallest i in [lo, k] with lcp(c[i], c[k]) >= d (pred(k) holds)
__device__ inline int64_t search_left(const u64* c, int64_t lo, int64_t k, int d) {
  const u64 ck = c[k];
  int64_t good = k, step = 1;
  while (true) {  // exponential phase
    const int64_t i = good - step;
    if (i < lo) break;
    if (lcp_digits(c[i], ck) >= d) {
      good = i;
      step <<= 1;
    } else {
      break;
    }
  }
  int64_t lo2 = good - step + 1 < lo ? lo : good - step + 1, hi2 = good;  // answer in [lo2, hi2]
  while (lo2 < hi2) {
    const int64_t mid = (lo2 + hi2) >> 1;
    if (lcp_digits(c[mid], ck) >= d) hi2 = mid;
    else lo2 = mid + 1;
  }
  return lo2;
}

// largest j in [k, hi] with lcp(c[k], c[j]) >= d (pred(k) holds)
__device__ inline int64_t search_right(const u64* c, int64_t k, int64_t hi, int d) {
  const u64 ck = c[k];
  int64_t good = k, step = 1;
  while (true) {
    const int64_t j = good + step;
    if (j > hi) break;
    if (lcp_digits(ck, c[j]) >= d) {
      good = j;
      step <<= 1;
    } else {
      break;
    }
  }
  int64_t lo2 = good, hi2 = good + step - 1 > hi ? hi : good + step - 1;
  while (lo2 < hi2) {
    const int64_t mid = (lo2 + hi2 + 1) >> 1;
    if (lcp_digits(ck, c[mid]) >= d) lo2 = mid;
    else hi2 = mid - 1;
  }
  return lo2;
}

// One thread per sorted point p: (a) the separator between p and p + 1 emits
// the branching cell it owns; (b) p is marked when a leaf (run of identical
// codes) starts at it.
__global__ __launch_bounds__(kBlock) void k_topo(const u64* codes, const SegRange* sr, int nseg,
                                                 int64_t n, unsigned* mask, int* own_d,
                                                 int* own_a, int* own_b, unsigned char* leaf0) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const SegRange s = sr[find_seg(sr, nseg, k)];
  leaf0[k] = (k == s.s0 || lcp_digits(codes[k - 1], codes[k]) < kQBits) ? 1 : 0;
  own_d[k] = -1;
  if (k + 1 >= s.s1) return;
  const int d = lcp_digits(codes[k], codes[k + 1]);
  if (d >= kQBits) return;
  const int64_t a = search_left(codes, s.s0, k, d);
  if (a != k && lcp_digits(codes[a], codes[k]) == d) return;  // not the leftmost separator
  const int64_t b = search_right(codes, k + 1, s.s1 - 1, d);
  own_d[k] = d;
  own_a[k] = (int)a;
  own_b[k] = (int)b;
  atomicOr(&mask[a], 1u << d);
}

__global__ __launch_bounds__(kBlock) void k_count(const unsigned* mask,
                                                  const unsigned char* leaf0, int64_t n,
                                                  unsigned* cnt) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < n) cnt[p] = (unsigned)__popc(mask[p]) + leaf0[p];
}

// ------------------------------------------------------------ prefix sums
struct D4 {
  double m, x, y, z;
};
__device__ inline D4 operator+(const D4& a, const D4& b) { return {a.m + b.m, a.x + b.x, a.y + b.y, a.z + b.z}; }

template <typename V>
__device__ inline V scan_zero();
template <> __device__ inline unsigned scan_zero<unsigned>() { return 0u; }
template <> __device__ inline D4 scan_zero<D4>() { return {0.0, 0.0, 0.0, 0.0}; }

template <typename V>
__device__ inline V shfl_up_v(V x, int o);
template <> __device__ inline unsigned shfl_up_v<unsigned>(unsigned x, int o) { return __shfl_up(x, o, kWave); }
template <> __device__ inline D4 shfl_up_v<D4>(D4 x, int o) {
  return {__shfl_up(x.m, o, kWave), __shfl_up(x.x, o, kWave), __shfl_up(x.y, o, kWave), __shfl_up(x.z, o, kWave)};
}

// Block-wide exclusive scan in thread order; returns the block total in *tot.
template <typename V>
__device__ inline V block_scan_excl(V x, V* lds, V* tot) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  V inc = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    V y = shfl_up_v(inc, o);
    if (lane >= o) inc = inc + y;
  }
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  V base = scan_zero<V>(), t = scan_zero<V>();
  for (int ww = 0; ww < kBlock / kWave; ++ww) {
    if (ww < w) base = base + lds[ww];
    t = t + lds[ww];
  }
  __syncthreads();
  *tot = t;
  // exclusive = base + inc - x, written without subtraction for exactness
  V prev = shfl_up_v(inc, 1);
  if (lane == 0) prev = scan_zero<V>();
  return base + prev;
}

template <typename V, typename Load>
__global__ __launch_bounds__(kBlock) void k_scan_up(Load ld, int64_t n, V* bsum) {
  __shared__ V lds[kBlock / kWave];
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  V s = scan_zero<V>();
  for (int k = 0; k < kScanItems; ++k)
    if (b0 + k < n) s = s + ld(b0 + k);
  V tot;
  (void)block_scan_excl(s, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_scan_mid(V* bsum, int nb) {
  __shared__ V lds[kBlock / kWave];
  V carry = scan_zero<V>();
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + threadIdx.x;
    const V x = i < nb ? bsum[i] : scan_zero<V>();
    V tot;
    const V ex = block_scan_excl(x, lds, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry = carry + tot;
  }
}

// out[i] = sum of ld(0..i-1) for i in [0, n]; out has n + 1 entries.
template <typename V, typename Load>
__global__ __launch_bounds__(kBlock) void k_scan_down(Load ld, int64_t n, const V* bsum, V* out) {
  __shared__ V lds[kBlock / kWave];
  const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  V v[kScanItems];
  V s = scan_zero<V>();
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (b0 + k < n) ? ld(b0 + k) : scan_zero<V>();
    s = s + v[k];
  }
  V tot;
  V run = bsum[blockIdx.x] + block_scan_excl(s, lds, &tot);
  for (int k = 0; k < kScanItems; ++k) {
    if (b0 + k <= n) out[b0 + k] = run;
    run = run + v[k];
  }
}

struct LoadCnt {
  const unsigned* c;
  __device__ unsigned operator()(int64_t i) const { return c[i]; }
};
template <typename T>
struct LoadMass {
  const vec4_t<T>* X;
  __device__ D4 operator()(int64_t i) const {
    const vec4_t<T> p = X[i];
    const double m = (double)p.w;
    return {m, m * (double)p.x, m * (double)p.y, m * (double)p.z};
  }
};

template <typename V, typename Load>
fga_status exclusive_scan(Load ld, int64_t n, V* out, V* bsum_scratch, hipStream_t s) {
  const int nb = (int)((n + kScanTile) / kScanTile);  // covers index n as well
  k_scan_up<V, Load><<<nb, kBlock, 0, s>>>(ld, n, bsum_scratch);
  k_scan_mid<V><<<1, kBlock, 0, s>>>(bsum_scratch, nb);
  k_scan_down<V, Load><<<nb, kBlock, 0, s>>>(ld, n, bsum_scratch, out);
  FGA_HIP(hipGetLastError());
  return FGA_OK;
}

// ------------------------------------------------------------ leaf size L > 1
// With leaf size L a cell is split only while it holds more than L points, so
// the tree keeps exactly the cells whose parent cell holds more than L points;
// a kept cell with at most L points is a leaf at one level below its parent.
// The parent of the cell holding sorted points [a, b] branches at the larger
// of the two boundary LCPs (the neighbours outside the range), and its points
// are the run around [a, b] sharing that many digits.
__device__ inline void prune_mark(const u64* codes, const SegRange& s, int64_t a, int64_t b,
                                  int L, double lroot, BHNode* nd, unsigned* keep) {
  const int dl = a > s.s0 ? lcp_digits(codes[a - 1], codes[a]) : -1;
  const int dr = b + 1 < s.s1 ? lcp_digits(codes[b], codes[b + 1]) : -1;
  const int dp = dl > dr ? dl : dr;
  const int64_t count = b - a + 1;
  if (dp < 0) {  // the root
    *keep = 1u;
    return;
  }
  const int64_t ap = search_left(codes, s.s0, a, dp);
  const int64_t bp = search_right(codes, b, s.s1 - 1, dp);
  const bool kept = bp - ap + 1 > L;
  *keep = kept ? 1u : 0u;
  if (kept && count <= L && count > 1) {  // becomes (or stays) a leaf one level below its parent
    const double l = ldexp(lroot, -(dp + 1));
    nd->l2 = (float)(l * l);
  }
}

// Tree statistics (deepest level, leaves, internal nodes, overflow flag) of
// one block, written to the block's own slot of part; k_stats_fin folds the
// slots. Same-address atomics from every wave of a million-node build
// serialise chip-wide at roughly 10 ns each, which cost over half a
// millisecond per launch. Every thread of the block calls it.
__device__ inline void block_stats(uint4* part, bool leaf, bool internal, int depth, bool over) {
  __shared__ unsigned lds[4][kBlock / kWave];
  const unsigned long long ml = __ballot(leaf), mi = __ballot(internal), mo = __ballot(over);
  int d = depth;
  for (int o = kWave / 2; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o, kWave));
  const int w = (int)threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    lds[0][w] = (unsigned)d;
    lds[1][w] = (unsigned)__popcll(ml);
    lds[2][w] = (unsigned)__popcll(mi);
    lds[3][w] = mo ? 1u : 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    for (int k = 0; k < kBlock / kWave; ++k) {
      r.x = max(r.x, lds[0][k]);
      r.y += lds[1][k];
      r.z += lds[2][k];
      r.w |= lds[3][k];
    }
    part[blockIdx.x] = r;
  }
}

// One block: stats[0] = max(stats[0], deepest), stats[1] += leaves,
// stats[2] += internal nodes, stats[3] |= overflow, over the nb slots.
__global__ __launch_bounds__(kBlock) void k_stats_fin(const uint4* part, int nb, unsigned* stats) {
  __shared__ uint4 lds[kBlock / kWave];
  uint4 r = make_uint4(0u, 0u, 0u, 0u);
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    const uint4 v = part[k];
    r.x = max(r.x, v.x);
    r.y += v.y;
    r.z += v.z;
    r.w |= v.w;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    r.x = max(r.x, (unsigned)__shfl_xor((int)r.x, o, kWave));
    r.y += (unsigned)__shfl_xor((int)r.y, o, kWave);
    r.z += (unsigned)__shfl_xor((int)r.z, o, kWave);
    r.w |= (unsigned)__shfl_xor((int)r.w, o, kWave);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = r;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 1; k < kBlock / kWave; ++k) {
    r.x = max(r.x, lds[k].x);
    r.y += lds[k].y;
    r.z += lds[k].z;
    r.w |= lds[k].w;
  }
  stats[0] = max(stats[0], r.x);
  stats[1] += r.y;
  stats[2] += r.z;
  stats[3] |= r.w;
}

// Copies the kept nodes to their compacted preorder positions; skip pointers
// and segment offsets map through the exclusive scan NI of the keep flags.
__global__ __launch_bounds__(kBlock) void k_compact(const BHNode* in, const unsigned* keep,
                                                    const unsigned* NI, const int* node_off,
                                                    int nseg, unsigned total, BHNode* out,
                                                    uint4* part) {
  const unsigned i = blockIdx.x * kBlock + threadIdx.x;
  bool is_leaf = false, is_int = false;
  if (i < total && keep[i]) {
    int lo = 0, hi = nseg - 1;  // segment of node i
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((unsigned)node_off[mid] <= i) lo = mid;
      else hi = mid - 1;
    }
    const unsigned base = (unsigned)node_off[lo];
    BHNode nd = in[i];
    const unsigned skip_g = base + (unsigned)nd.skip;
    const unsigned ni = NI[i];
    nd.skip = (int)(NI[skip_g] - NI[base]);
    if ((unsigned)nd.skip == ni - NI[base] + 1) {
      is_leaf = true;
      nd.l2 = fabsf(nd.l2);  // a leaf is walked point by point anyway: no twig flag
    } else {
      is_int = true;
    }
    out[ni] = nd;
  }
  block_stats(part, is_leaf, is_int, 0, false);
}

// ------------------------------------------------------------ node emission
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit(const vec4_t<T>* Xs, const u64* codes, const SegRange* sr,
                                                 const SegBox* box, int nseg, int64_t n,
                                                 const unsigned* mask,
                                                 const unsigned char* leaf0, const int* own_d,
                                                 const int* own_a, const int* own_b,
                                                 const unsigned* P, const D4* W, BHNode* nodes,
                                                 unsigned cap, uint4* part, int L,
                                                 unsigned* keep) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool is_int = false, is_leaf = false, over = false;
  int dmax = 0;
  if (k < n) {
    const int sg = find_seg(sr, nseg, k);
    const double lroot = box[sg].lroot;
    // node fields are local to the segment: point indices from its first sorted
    // point, node indices from its root
    const int s0 = (int)sr[sg].s0;
    const int nbase = (int)P[s0];
    const int d = own_d[k];
    if (d >= 0) {  // branching cell owned by separator k
      const int a = own_a[k], b = own_b[k];
      const unsigned idx = P[a] + (unsigned)__popc(mask[a] & ((1u << d) - 1u));
      const D4 s = W[b + 1] + D4{-W[a].m, -W[a].x, -W[a].y, -W[a].z};
      BHNode nd;
      nd.cm = make_float4((float)(s.x / s.m), (float)(s.y / s.m), (float)(s.z / s.m), (float)s.m);
      nd.skip = (int)P[b + 1] - nbase;
      nd.first = a - s0;
      nd.last = b - s0;
      const double l = ldexp(lroot, -d);
      nd.l2 = (float)(l * l);
      // twig: every point of the cell is its own child (all separators inside
      // branch at depth d); flagged by the sign bit of l2. At most 8 points.
      if (b - a < 8) {
        bool twig = true;
        for (int q = a; q < b && twig; ++q) twig = lcp_digits(codes[q], codes[q + 1]) == d;
        if (twig) nd.l2 = -nd.l2;
      }
      if (idx >= cap) {  // more nodes than the array holds: reported, never written
        over = true;
      } else {
        if (L > 1) prune_mark(codes, sr[sg], a, b, L, lroot, &nd, keep + idx);
        nodes[idx] = nd;
      }
      dmax = max(dmax, d);
      is_int = true;
    }
    if (leaf0[k]) {  // leaf: run of identical codes starting at k
      int64_t e = k;
      while (e + 1 < sr[sg].s1 && !leaf0[e + 1]) ++e;
      const unsigned idx = P[k] + (unsigned)__popc(mask[k]);
      BHNode nd;
      if (e == k) {  // singleton: the point itself
        const vec4_t<T> p = Xs[k];
        nd.cm = make_float4((float)p.x, (float)p.y, (float)p.z, (float)p.w);
      } else {
        const D4 s = W[e + 1] + D4{-W[k].m, -W[k].x, -W[k].y, -W[k].z};
        nd.cm = make_float4((float)(s.x / s.m), (float)(s.y / s.m), (float)(s.z / s.m), (float)s.m);
        dmax = kQBits;
      }
      nd.skip = (int)idx + 1 - nbase;
      nd.first = (int)k - s0;
      nd.last = (int)e - s0;
      const double l = ldexp(lroot, -kQBits);  // a leaf of several points is a depth-20 cell
      nd.l2 = (float)(l * l);
      if (idx >= cap) {
        over = true;
      } else {
        if (L > 1) prune_mark(codes, sr[sg], k, e, L, lroot, &nd, keep + idx);
        nodes[idx] = nd;
      }
      is_leaf = true;
    }
  }
  block_stats(part, is_leaf, is_int, dmax, over);
}

__global__ void k_seg_nodes(const SegRange* sr, int nseg, const unsigned* P, int* node_off) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) node_off[s] = (int)P[sr[s].s0];
  if (s == nseg - 1) node_off[nseg] = (int)P[sr[s].s1];
}

__global__ void k_remap_off(const unsigned* NI, int nseg, int* node_off) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= nseg) node_off[s] = (int)NI[node_off[s]];
}

// ------------------------------------------------------------ host driver
// Temporaries of one build, from the caching allocator, returned at scope end.
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t st) : s(st) {}
  ~Scratch() {
    for (void* p : ptrs) pool_free(p, s);
  }
  template <typename P>
  fga_status get(P** out, size_t bytes) {
    void* p = pool_alloc(bytes < 16 ? 16 : bytes, s);
    if (!p) return FGA_E_NOMEM;
    ptrs.push_back(p);
    *out = (P*)p;
    return FGA_OK;
  }
};

// Segmented stable sort of vec4 points by Morton code of their own segment's
// box. On return Xs holds the sorted points, perm_out (if non-null) the
// source index of each sorted point, codes_out (if non-null) the sorted codes.
template <typename T>
fga_status morton_sort(int nseg, const TreeSeg* segs, const vec4_t<T>* X, int64_t ntot,
                       vec4_t<T>* Xs, unsigned* perm_out, u64* codes_out, SegBox* box_dev,
                       Scratch& sc, hipStream_t s) {
  std::vector<SortTile> tiles;
  std::vector<int> seg_tile0(nseg + 1);
  int hist_entries = 0;
  for (int g = 0; g < nseg; ++g) {
    seg_tile0[g] = (int)tiles.size();
    const int nt = (int)((segs[g].n + kSortTile - 1) / kSortTile);
    for (int t = 0; t < nt; ++t) {
      SortTile st;
      st.seg = g;
      st.tile_in_seg = t;
      st.ntiles_seg = nt;
      st.hbase = hist_entries;
      st.start = segs[g].off + (int64_t)t * kSortTile;
      st.count = (int)((segs[g].n - (int64_t)t * kSortTile) < kSortTile
                           ? (segs[g].n - (int64_t)t * kSortTile)
                           : kSortTile);
      st.pad_ = 0;
      tiles.push_back(st);
    }
    hist_entries += 256 * nt;
  }
  seg_tile0[nseg] = (int)tiles.size();
  const int ntiles = (int)tiles.size();
  SortTile* dtiles;
  int* dseg0;
  double* boxpart;
  u64 *k0, *k1;
  unsigned *v0, *v1, *hist;
  FGA_TRY(sc.get(&dtiles, sizeof(SortTile) * ntiles));
  FGA_TRY(sc.get(&dseg0, sizeof(int) * (nseg + 1)));
  FGA_TRY(sc.get(&boxpart, sizeof(double) * 6 * ntiles));
  FGA_TRY(sc.get(&k0, sizeof(u64) * ntot));
  FGA_TRY(sc.get(&k1, sizeof(u64) * ntot));
  FGA_TRY(sc.get(&v0, sizeof(unsigned) * ntot));
  FGA_TRY(sc.get(&v1, sizeof(unsigned) * ntot));
  FGA_TRY(sc.get(&hist, sizeof(unsigned) * hist_entries));
  const int scan_blocks = (hist_entries + kHScanTile - 1) / kHScanTile;
  unsigned* scan_tot;
  FGA_TRY(sc.get(&scan_tot, sizeof(unsigned) * scan_blocks));
  FGA_HIP(hipMemcpyAsync(dtiles, tiles.data(), sizeof(SortTile) * ntiles, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dseg0, seg_tile0.data(), sizeof(int) * (nseg + 1), hipMemcpyHostToDevice, s));
  k_box_part<T><<<ntiles, kBlock, 0, s>>>(X, dtiles, boxpart);
  k_box_fin<<<nseg, kWave, 0, s>>>(boxpart, dseg0, nseg, box_dev);
  k_morton<T><<<ntiles, kBlock, 0, s>>>(X, dtiles, box_dev, k0, v0);
  for (int shift = 0; shift < 3 * kQBits; shift += 8) {
    k_rs_hist<<<ntiles, kBlock, 0, s>>>(k0, dtiles, shift, hist);
    k_scan_tile<<<scan_blocks, kBlock, 0, s>>>(hist, hist_entries, scan_tot);
    if (scan_blocks > 1) {  // one tile is already the whole exclusive scan
      k_scan_u32_1block<<<1, 1024, 0, s>>>(scan_tot, scan_blocks);
      k_scan_add<<<scan_blocks, kBlock, 0, s>>>(hist, hist_entries, scan_tot);
    }
    k_rs_scatter<<<ntiles, kBlock, 0, s>>>(k0, v0, dtiles, shift, hist, k1, v1);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  k_gather4<T><<<(int)((ntot + kBlock - 1) / kBlock), kBlock, 0, s>>>(X, v0, ntot, Xs);
  FGA_HIP(hipGetLastError());
  if (perm_out) FGA_HIP(hipMemcpyAsync(perm_out, v0, sizeof(unsigned) * ntot, hipMemcpyDeviceToDevice, s));
  if (codes_out) FGA_HIP(hipMemcpyAsync(codes_out, k0, sizeof(u64) * ntot, hipMemcpyDeviceToDevice, s));
  return FGA_OK;
}

}  // namespace

// Builds every segment's tree. X (packed vec4, segments at segs[g].off) is
// sorted in place by Morton code. nodes_out receives a new device array;
// node_off_host[g] / [g + 1] bound segment g's nodes (root first); order_out
// (if non-null) receives a new device array sorted position -> original
// position; stats_host = {max depth, leaves, internal}.
template <typename T>
fga_status build_trees(int nseg, const TreeSeg* segs, void* Xpacked, int64_t ntot,
                       int leaf_size, BHNode** nodes_out, int* node_off_host, int** order_out,
                       int* stats_host, hipStream_t s) {
  Scratch sc(s);
  vec4_t<T>* X = (vec4_t<T>*)Xpacked;
  vec4_t<T>* Xs;
  u64* codes;
  SegBox* box;
  unsigned* perm = nullptr;
  FGA_TRY(sc.get(&Xs, sizeof(vec4_t<T>) * ntot));
  FGA_TRY(sc.get(&codes, sizeof(u64) * ntot));
  FGA_TRY(sc.get(&box, sizeof(SegBox) * nseg));
  if (order_out) {
    FGA_TRY(pool_get(&perm, sizeof(unsigned) * ntot, s));
    *order_out = (int*)perm;
  }
  fga_status st = morton_sort<T>(nseg, segs, X, ntot, Xs, perm, codes, box, sc, s);
  if (st != FGA_OK) {
    if (perm) pool_free(perm, s);
    return st;
  }
  FGA_HIP(hipMemcpyAsync(X, Xs, sizeof(vec4_t<T>) * ntot, hipMemcpyDeviceToDevice, s));
  std::vector<SegRange> hr(nseg);
  for (int g = 0; g < nseg; ++g) hr[g] = {segs[g].off, segs[g].off + segs[g].n};
  SegRange* sr;
  unsigned *mask, *cnt, *P, *stats;
  uint4* bpart;
  unsigned char* leaf0;
  int *own_d, *own_a, *own_b, *node_off;
  D4 *W, *bsumD;
  unsigned* bsumU;
  const int nbScan = (int)((ntot + kScanTile) / kScanTile);
  FGA_TRY(sc.get(&sr, sizeof(SegRange) * nseg));
  FGA_TRY(sc.get(&mask, sizeof(unsigned) * ntot));
  FGA_TRY(sc.get(&cnt, sizeof(unsigned) * ntot));
  FGA_TRY(sc.get(&P, sizeof(unsigned) * (ntot + 1)));
  FGA_TRY(sc.get(&stats, sizeof(unsigned) * 4));
  FGA_TRY(sc.get(&bpart, sizeof(uint4) * (size_t)((2 * ntot + kBlock - 1) / kBlock)));
  FGA_TRY(sc.get(&leaf0, ntot));
  FGA_TRY(sc.get(&own_d, sizeof(int) * ntot));
  FGA_TRY(sc.get(&own_a, sizeof(int) * ntot));
  FGA_TRY(sc.get(&own_b, sizeof(int) * ntot));
  FGA_TRY(sc.get(&node_off, sizeof(int) * (nseg + 1)));
  FGA_TRY(sc.get(&W, sizeof(D4) * (ntot + 1)));
  FGA_TRY(sc.get(&bsumD, sizeof(D4) * nbScan));
  FGA_TRY(sc.get(&bsumU, sizeof(unsigned) * nbScan));
  FGA_HIP(hipMemcpyAsync(sr, hr.data(), sizeof(SegRange) * nseg, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemsetAsync(mask, 0, sizeof(unsigned) * ntot, s));
  FGA_HIP(hipMemsetAsync(stats, 0, sizeof(unsigned) * 4, s));
  const int nb = (int)((ntot + kBlock - 1) / kBlock);
  k_topo<<<nb, kBlock, 0, s>>>(codes, sr, nseg, ntot, mask, own_d, own_a, own_b, leaf0);
  k_count<<<nb, kBlock, 0, s>>>(mask, leaf0, ntot, cnt);
  FGA_TRY((exclusive_scan<unsigned, LoadCnt>(LoadCnt{cnt}, ntot, P, bsumU, s)));
  FGA_TRY((exclusive_scan<D4, LoadMass<T>>(LoadMass<T>{X}, ntot, W, bsumD, s)));
  // a compressed octree of n points has at most 2 n - 1 nodes: the node array
  // is sized for that, so the count is not needed on the host before k_emit
  const int L = leaf_size > 1 ? leaf_size : 1;
  unsigned total = (unsigned)(2 * ntot);
  if (L > 1) {  // the leaf-size pass sizes its arrays by the exact count
    FGA_HIP(hipMemcpyAsync(&total, P + ntot, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    FGA_HIP(hipStreamSynchronize(s));
  }
  BHNode* nodes = nullptr;
  if (pool_get(&nodes, sizeof(BHNode) * (total ? total : 1), s) != FGA_OK) {
    if (perm) pool_free(perm, s);
    return FGA_E_NOMEM;
  }
  unsigned* keep = nullptr;
  if (L > 1) {
    FGA_TRY(sc.get(&keep, sizeof(unsigned) * (total + 1)));
    FGA_HIP(hipMemsetAsync(keep, 0, sizeof(unsigned) * (total + 1), s));
  }
  k_emit<T><<<nb, kBlock, 0, s>>>(X, codes, sr, box, nseg, ntot, mask, leaf0, own_d, own_a, own_b, P, W,
                                  nodes, total ? total : 1, bpart, L, keep);
  k_stats_fin<<<1, kBlock, 0, s>>>(bpart, nb, stats);
  k_seg_nodes<<<(nseg + 63) / 64, 64, 0, s>>>(sr, nseg, P, node_off);
  if (L > 1) {  // drop the cells below the leaf size and compact the preorder
    unsigned *NI, *bsumK;
    const int nbK = (int)(((int64_t)total + kScanTile) / kScanTile);
    FGA_TRY(sc.get(&NI, sizeof(unsigned) * (total + 1)));
    FGA_TRY(sc.get(&bsumK, sizeof(unsigned) * nbK));
    FGA_TRY((exclusive_scan<unsigned, LoadCnt>(LoadCnt{keep}, (int64_t)total, NI, bsumK, s)));
    unsigned kept = 0;
    FGA_HIP(hipMemcpyAsync(&kept, NI + total, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    FGA_HIP(hipStreamSynchronize(s));
    BHNode* packed = nullptr;
    if (pool_get(&packed, sizeof(BHNode) * (kept ? kept : 1), s) != FGA_OK) {
      pool_free(nodes, s);
      if (perm) pool_free(perm, s);
      return FGA_E_NOMEM;
    }
    FGA_HIP(hipMemsetAsync(stats + 1, 0, sizeof(unsigned) * 2, s));
    const int nbC = (int)((total + kBlock - 1) / kBlock);
    k_compact<<<nbC, kBlock, 0, s>>>(nodes, keep, NI, node_off, nseg, total, packed, bpart);
    k_stats_fin<<<1, kBlock, 0, s>>>(bpart, nbC, stats);
    k_remap_off<<<(nseg + 64) / 64, 64, 0, s>>>(NI, nseg, node_off);
    FGA_HIP(hipStreamSynchronize(s));
    pool_free(nodes, s);
    nodes = packed;
  }
  unsigned hstats[4];
  hipError_t e1 = hipGetLastError();
  if (e1 == hipSuccess)
    e1 = hipMemcpyAsync(node_off_host, node_off, sizeof(int) * (nseg + 1), hipMemcpyDeviceToHost, s);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(hstats, stats, sizeof(hstats), hipMemcpyDeviceToHost, s);
  if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
  if (e1 != hipSuccess) {
    pool_free(nodes, s);
    if (perm) pool_free(perm, s);
    set_error("tree build failed: %s", hipGetErrorString(e1));
    return FGA_E_DEVICE;
  }
  if (hstats[3]) {
    pool_free(nodes, s);
    if (perm) pool_free(perm, s);
    set_error("tree build: node count above the 2 n - 1 bound");
    return FGA_E_DEVICE;
  }
  stats_host[0] = (int)hstats[0];
  stats_host[1] = (int)hstats[1];
  stats_host[2] = (int)hstats[2];
  *nodes_out = nodes;
  return FGA_OK;
}

// ------------------------------------------------------------ child blocks
namespace {

__device__ inline int seg_of_node(const int* node_off, int nseg, int i) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (node_off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Number of children of every internal node: its children are n + 1 and then
// successive skip pointers until the node's own skip (at most 8).
__global__ __launch_bounds__(kBlock) void k_nchild(const BHNode* pre, int total,
                                                   const int* node_off, int nseg,
                                                   unsigned* nch) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i > total) return;
  if (i == total) {
    nch[i] = 0;
    return;
  }
  const int off = node_off[seg_of_node(node_off, nseg, i)];
  const int loc = i - off;
  const int skip = pre[i].skip;
  unsigned k = 0;
  if (skip > loc + 1)
    for (int c = loc + 1; c < skip && k < 9; c = pre[off + c].skip) ++k;
  nch[i] = k;
}

__device__ inline BHWide to_wide(const BHNode& nd, int child_field) {
  BHWide w;
  w.cm = nd.cm;
  w.first = nd.first;
  w.last = nd.last;
  w.child = child_field;
  w.l2 = nd.l2;
  return w;
}

// Every internal node writes its children's records into its child block
// (block start = 1 + number of children of the segment's earlier nodes);
// segment roots write themselves at their segment's first slot.
__global__ __launch_bounds__(kBlock) void k_relayout(const BHNode* pre, int total,
                                                     const int* node_off, int nseg,
                                                     const unsigned* nch, const unsigned* G,
                                                     BHWide* out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const int off = node_off[seg_of_node(node_off, nseg, i)];
  const int loc = i - off;
  auto child_field = [&](int g) -> int {  // g: global preorder index of a node
    if (nch[g] == 0) return -1;
    const int start = 1 + (int)(G[g] - G[off]);
    return start | (int)((nch[g] - 1u) << kChildShift);
  };
  if (loc == 0) out[off] = to_wide(pre[i], child_field(i));
  if (nch[i] == 0) return;
  const int start = 1 + (int)(G[i] - G[off]);
  int r = 0;
  for (int c = loc + 1; c < pre[i].skip && r < 8; c = pre[off + c].skip, ++r)
    out[off + start + r] = to_wide(pre[off + c], child_field(off + c));
}

}  // namespace

fga_status relayout_wide(const BHNode* pre, int total, int nseg, const int* node_off_host,
                         BHWide** out, hipStream_t s) {
  Scratch sc(s);
  int* doff;
  unsigned *nch, *G, *bsum;
  const int nb = (int)(((int64_t)total + kScanTile) / kScanTile);
  FGA_TRY(sc.get(&doff, sizeof(int) * (nseg + 1)));
  FGA_TRY(sc.get(&nch, sizeof(unsigned) * (total + 1)));
  FGA_TRY(sc.get(&G, sizeof(unsigned) * (total + 1)));
  FGA_TRY(sc.get(&bsum, sizeof(unsigned) * nb));
  FGA_HIP(hipMemcpyAsync(doff, node_off_host, sizeof(int) * (nseg + 1), hipMemcpyHostToDevice, s));
  k_nchild<<<(total + kBlock) / kBlock, kBlock, 0, s>>>(pre, total, doff, nseg, nch);
  FGA_TRY((exclusive_scan<unsigned, LoadCnt>(LoadCnt{nch}, (int64_t)total, G, bsum, s)));
  BHWide* w = nullptr;
  FGA_TRY(pool_get(&w, sizeof(BHWide) * (total ? total : 1), s));
  k_relayout<<<(total + kBlock - 1) / kBlock, kBlock, 0, s>>>(pre, total, doff, nseg, nch, G, w);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    pool_free(w, s);
    set_error("child-block relayout failed: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  *out = w;
  return FGA_OK;
}

// Sorts the template (vec4, one segment per pair) by Morton code in its own
// box, so that a wavefront's particles are spatially close.
template <typename T>
fga_status sort_points_morton(int nseg, const TreeSeg* segs, void* Q, int64_t ntot, int* perm,
                              hipStream_t s) {
  Scratch sc(s);
  vec4_t<T>* Qs;
  SegBox* box;
  FGA_TRY(sc.get(&Qs, sizeof(vec4_t<T>) * ntot));
  FGA_TRY(sc.get(&box, sizeof(SegBox) * nseg));
  FGA_TRY(morton_sort<T>(nseg, segs, (vec4_t<T>*)Q, ntot, Qs, (unsigned*)perm, nullptr, box, sc,
                         s));
  FGA_HIP(hipMemcpyAsync(Q, Qs, sizeof(vec4_t<T>) * ntot, hipMemcpyDeviceToDevice, s));
  return FGA_OK;
}

template fga_status build_trees<float>(int, const TreeSeg*, void*, int64_t, int, BHNode**, int*,
                                       int**, int*, hipStream_t);
template fga_status build_trees<double>(int, const TreeSeg*, void*, int64_t, int, BHNode**, int*,
                                        int**, int*, hipStream_t);
template fga_status sort_points_morton<float>(int, const TreeSeg*, void*, int64_t, int*,
                                             hipStream_t);
template fga_status sort_points_morton<double>(int, const TreeSeg*, void*, int64_t, int*,
                                              hipStream_t);

}  // namespace fga
