// Group tables of the Barnes-Hut group walk, built on the device.
//
// A group is a run of consecutive particles of a Morton-ordered template
// (consecutive in Morton order, hence spatially close) that share one walk
// of the tree. The runs are cut greedily along each segment (one template of
// a batch): a run starts at a particle and takes the following ones, at most
// G in all, while the diagonal of their bounding box stays within tau = f
// times the median diagonal of the segment's aligned blocks of G (f = 0:
// runs of exactly G). Sparse stretches of the order (consecutive particles
// far apart) thus form small groups with small boxes instead of one box that
// opens every node between them.
//
// The greedy chain is sequential by definition; it is evaluated in parallel
// through maps between aligned blocks of G particles (a run is never longer
// than a block, so every block holds at least one run start):
//   1. next(i), the end of the run that would start at particle i (one
//      thread per particle);
//   2. F_b(e), for every block b and every entry offset e (the block's first
//      run start), the entry offset into block b + 1 (one wave per block,
//      a lane per entry follows next());
//   3. H_s = F composed over the 64 blocks of a super-block (one wave per
//      super-block, the maps in LDS);
//   4. the entry of every super-block along the segment (one block per
//      segment), then of every block (one wave per super-block);
//   5. the runs of every block from its entry, compacted into one table.
// Only the block diagonals (for the medians) and the finished table cross
// to the host.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

namespace fga {
namespace {

constexpr int kGMax = 2 * kWave;  // longest run (G = 64 K, K <= 2)
constexpr int kSB = kWave;         // blocks per super-block
constexpr int kSEChunk = 256;      // super-block maps staged in LDS at a time
// Entry value of a block that holds no run start: the last block of a
// segment when the run before it reaches the segment's end.
constexpr unsigned char kNoEntry = 255;

struct GSeg {
  int64_t off;  // first particle of the segment in Q
  int64_t m;    // particles
  int blk0;     // first block of the segment (global block index)
  int sb0;      // first super-block of the segment
};

__device__ inline int seg_of_block(const GSeg* sg, int nseg, int b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sg[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ inline int seg_of_super(const GSeg* sg, int nseg, int s) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sg[mid].sb0 <= s) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__device__ inline int seg_blocks(const GSeg& s, int G) { return (int)((s.m + G - 1) / G); }

// Squared diagonal of the bounding box of every aligned block of G particles
// (one wave per block).
__global__ __launch_bounds__(kBlock) void k_block_diag(const float4* Q, const GSeg* sg, int nseg,
                                                       int nblocks, int G, float* d2) {
  const int b = blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (b >= nblocks) return;  // whole waves leave together
  const GSeg s = sg[seg_of_block(sg, nseg, b)];
  const int64_t first = (int64_t)(b - s.blk0) * G;
  const int c = (int)min((int64_t)G, s.m - first);
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int t = lane; t < c; t += kWave) {
    const float4 p = Q[s.off + first + t];
    lo[0] = fminf(lo[0], p.x); hi[0] = fmaxf(hi[0], p.x);
    lo[1] = fminf(lo[1], p.y); hi[1] = fmaxf(hi[1], p.y);
    lo[2] = fminf(lo[2], p.z); hi[2] = fmaxf(hi[2], p.z);
  }
  for (int o = kWave / 2; o > 0; o >>= 1)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, kWave));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, kWave));
    }
  if (lane == 0) {
    const float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    d2[b] = ex * ex + ey * ey + ez * ez;
  }
}

// next[gi] (segment-local) = end of the greedy run starting at particle gi:
// the particles from gi on while their box stays within tau2, at most G of
// them and not past the segment's end. One thread per particle.
__global__ __launch_bounds__(kBlock) void k_next(const float4* Q, const GSeg* sg, int nseg,
                                                 int64_t ntot, int G, const float* tau2,
                                                 int* next) {
  const int64_t gi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gi >= ntot) return;
  int lo_s = 0, hi_s = nseg - 1;  // the last segment starting at or before gi
  while (lo_s < hi_s) {
    const int mid = (lo_s + hi_s + 1) >> 1;
    if (sg[mid].off <= gi) lo_s = mid;
    else hi_s = mid - 1;
  }
  const GSeg s = sg[lo_s];
  if (gi >= s.off + s.m) return;  // between segments
  const float t2 = tau2[lo_s];
  const int i = (int)(gi - s.off);
  const int e = (int)min((int64_t)i + G, s.m);
  const float4 p = Q[gi];
  float lx = p.x, ly = p.y, lz = p.z, hx = p.x, hy = p.y, hz = p.z;
  int j = i + 1;
  for (; j < e; ++j) {
    const float4 v = Q[s.off + j];
    const float nlx = fminf(lx, v.x), nhx = fmaxf(hx, v.x);
    const float nly = fminf(ly, v.y), nhy = fmaxf(hy, v.y);
    const float nlz = fminf(lz, v.z), nhz = fmaxf(hz, v.z);
    const float ex = nhx - nlx, ey = nhy - nly, ez = nhz - nlz;
    if (ex * ex + ey * ey + ez * ez > t2) break;
    lx = nlx; hx = nhx; ly = nly; hy = nhy; lz = nlz; hz = nhz;
  }
  next[gi] = j;
}

// F[b][e]: entering block b of its segment at offset e (its first run
// start), the chain of runs enters block b + 1 at offset F[b][e] in [0, G),
// or kNoEntry when it reaches the segment's end first. A run is at most G
// long, so every block before the last holds a start. One wave per block,
// entries e = lane, lane + 64.
__global__ __launch_bounds__(kBlock) void k_block_maps(const GSeg* sg, int nseg, int nblocks, int G,
                                                       const int* next, unsigned char* F) {
  const int b = blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (b >= nblocks) return;
  const GSeg s = sg[seg_of_block(sg, nseg, b)];
  const int64_t b0 = (int64_t)(b - s.blk0) * G, b1 = b0 + G;
  for (int e = lane; e < G; e += kWave) {
    int64_t pos = b0 + e;
    while (pos < b1 && pos < s.m) pos = next[s.off + pos];
    F[(int64_t)b * G + e] = pos < s.m ? (unsigned char)(pos - b1) : kNoEntry;
  }
}

// H[sp][e]: the maps of the (up to) 64 blocks of super-block sp composed
// (one wave per super-block, its maps staged in LDS).
__global__ __launch_bounds__(kBlock) void k_super_maps(const GSeg* sg, int nseg, int nsuper, int G,
                                                       const unsigned char* F, unsigned char* H) {
  __shared__ unsigned char lds[kBlock / kWave][kSB * kGMax];
  const int w = (int)threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int sp = blockIdx.x * (kBlock / kWave) + w;
  int fb = 0, nb = 0;
  if (sp < nsuper) {
    const GSeg s = sg[seg_of_super(sg, nseg, sp)];
    fb = s.blk0 + (sp - s.sb0) * kSB;                  // first block
    nb = min(kSB, seg_blocks(s, G) - (sp - s.sb0) * kSB);  // its blocks
    for (int k = lane; k < nb * G; k += kWave) lds[w][k] = F[(int64_t)fb * G + k];
  }
  __syncthreads();
  if (sp >= nsuper) return;
  for (int e0 = lane; e0 < G; e0 += kWave) {
    int e = e0;
    for (int k = 0; k < nb && e != kNoEntry; ++k) e = lds[w][k * G + e];
    H[(int64_t)sp * G + e0] = (unsigned char)e;
  }
}

// Entry offsets of the super-blocks of every segment (one block per segment:
// the first super-block is entered at 0, the next one at H of the previous;
// the maps are staged in LDS kSEChunk at a time and walked by thread 0).
__global__ __launch_bounds__(kBlock) void k_super_entries(const GSeg* sg, int G,
                                                          const unsigned char* H,
                                                          unsigned char* E) {
  __shared__ unsigned char lds[kSEChunk * kGMax];
  const GSeg s = sg[blockIdx.x];
  const int ns = (seg_blocks(s, G) + kSB - 1) / kSB;
  int e = 0;
  for (int c0 = 0; c0 < ns; c0 += kSEChunk) {
    const int nc = min(kSEChunk, ns - c0);
    __syncthreads();  // the previous chunk has been walked
    for (int k = threadIdx.x; k < nc * G; k += kBlock) lds[k] = H[(int64_t)(s.sb0 + c0) * G + k];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = 0; k < nc; ++k) {
        E[s.sb0 + c0 + k] = (unsigned char)e;
        if (e != kNoEntry) e = lds[k * G + e];
      }
  }
}

// Entry offsets of the blocks of every super-block (one wave per
// super-block, its maps staged in LDS, walked by the wave's first lane).
__global__ __launch_bounds__(kBlock) void k_block_entries(const GSeg* sg, int nseg, int nsuper, int G,
                                                          const unsigned char* F,
                                                          const unsigned char* E,
                                                          unsigned char* eb) {
  __shared__ unsigned char lds[kBlock / kWave][kSB * kGMax];
  const int w = (int)threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int sp = blockIdx.x * (kBlock / kWave) + w;
  int fb = 0, nb = 0;
  if (sp < nsuper) {
    const GSeg s = sg[seg_of_super(sg, nseg, sp)];
    fb = s.blk0 + (sp - s.sb0) * kSB;
    nb = min(kSB, seg_blocks(s, G) - (sp - s.sb0) * kSB);
    for (int k = lane; k < nb * G; k += kWave) lds[w][k] = F[(int64_t)fb * G + k];
  }
  __syncthreads();
  if (sp >= nsuper || lane != 0) return;
  int e = E[sp];
  for (int k = 0; k < nb; ++k) {
    eb[fb + k] = (unsigned char)e;
    if (e != kNoEntry) e = lds[w][k * G + e];
  }
}

// The runs that start in every block, from its entry: slots[b G ...] and
// their number cnt[b] (one thread per block).
__global__ __launch_bounds__(kBlock) void k_block_runs(const GSeg* sg, int nseg, int nblocks, int G,
                                                       const int* next, const unsigned char* eb,
                                                       int2* slots, int* cnt) {
  const int b = blockIdx.x * kBlock + (int)threadIdx.x;
  if (b >= nblocks) return;
  const GSeg s = sg[seg_of_block(sg, nseg, b)];
  const int64_t b0 = (int64_t)(b - s.blk0) * G, b1 = min(b0 + G, s.m);
  int64_t pos = eb[b] == kNoEntry ? b1 : b0 + eb[b];
  int k = 0;
  while (pos < b1) {
    const int64_t nx = next[s.off + pos];
    slots[(int64_t)b * G + k] = make_int2((int)pos, (int)(nx - pos));
    ++k;
    pos = nx;
  }
  cnt[b] = k;
}

// Exclusive scan of cnt[0, n) into ofs[0, n] (one block: each thread sums a
// contiguous chunk, the chunk sums are scanned through LDS).
__global__ __launch_bounds__(kBlock) void k_scan_counts(const int* cnt, int n, int* ofs) {
  __shared__ int part[kBlock];
  const int per = (n + kBlock - 1) / kBlock;
  const int a = (int)threadIdx.x * per, e = min(n, a + per);
  int sum = 0;
  for (int i = a; i < e; ++i) sum += cnt[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < kBlock; ++t) {
      const int v = part[t];
      part[t] = run;
      run += v;
    }
    ofs[n] = run;
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int i = a; i < e; ++i) {
    ofs[i] = run;
    run += cnt[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_compact_runs(const int2* slots, const int* cnt,
                                                         const int* ofs, int nblocks, int G,
                                                         int2* table) {
  const int b = blockIdx.x * (kBlock / kWave) + (int)threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (b >= nblocks) return;
  for (int j = lane; j < cnt[b]; j += kWave) table[ofs[b] + j] = slots[(int64_t)b * G + j];
}

__global__ void k_pack_xyz(const float* Y, int64_t m, float4* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = make_float4(Y[3 * i], Y[3 * i + 1], Y[3 * i + 2], 0.f);
}

}  // namespace

fga_status device_groups_xyz(const float* Y, int64_t m, int G, double f, std::vector<int2>& out,
                             hipStream_t s) {
  float4* Q = nullptr;
  FGA_TRY(pool_get(&Q, sizeof(float4) * (size_t)m, s));
  k_pack_xyz<<<(int)((m + kBlock - 1) / kBlock), kBlock, 0, s>>>(Y, m, Q);
  fga_status st = FGA_OK;
  if (hipGetLastError() != hipSuccess) {
    set_error("group tables: pack launch failed");
    st = FGA_E_DEVICE;
  }
  std::vector<std::vector<int2>> tabs;
  const int64_t zero = 0;
  if (st == FGA_OK) st = device_groups(Q, 1, &zero, &m, G, f, tabs, s);
  pool_free(Q, s);
  if (st == FGA_OK) out = std::move(tabs[0]);
  return st;
}

fga_status device_groups(const float4* Q, int nseg, const int64_t* off, const int64_t* m, int G,
                         double f, std::vector<std::vector<int2>>& out, hipStream_t s) {
  out.assign(nseg, {});
  if (G < 1 || G > kGMax) {
    set_error("group tables: run length %d outside [1, %d]", G, kGMax);
    return FGA_E_INVALID_ARG;
  }
  std::vector<GSeg> hs(nseg);
  int nblocks = 0, nsuper = 0;
  int64_t ntot = 0;
  for (int k = 0; k < nseg; ++k) {
    const int nb = (int)((m[k] + G - 1) / G);
    hs[k] = {off[k], m[k], nblocks, nsuper};
    nblocks += nb;
    nsuper += (nb + kSB - 1) / kSB;
    ntot = std::max(ntot, off[k] + m[k]);
  }
  if (nblocks == 0) return FGA_OK;
  GSeg* sg = nullptr;
  float *d2 = nullptr, *tau2 = nullptr;
  int *next = nullptr, *cnt = nullptr, *ofs = nullptr;
  unsigned char *F = nullptr, *H = nullptr, *E = nullptr, *eb = nullptr;
  int2 *slots = nullptr, *table = nullptr;
  fga_status st = FGA_OK;
  auto get = [&](auto** p, size_t bytes) {
    if (st == FGA_OK) st = pool_get(p, bytes < 16 ? 16 : bytes, s);
  };
  get(&sg, sizeof(GSeg) * nseg);
  get(&d2, sizeof(float) * nblocks);
  get(&tau2, sizeof(float) * nseg);
  get(&next, sizeof(int) * ntot);
  get(&F, (size_t)nblocks * G);
  get(&H, (size_t)nsuper * G);
  get(&E, (size_t)nsuper);
  get(&eb, (size_t)nblocks);
  get(&slots, sizeof(int2) * (size_t)nblocks * G);
  get(&table, sizeof(int2) * (size_t)nblocks * G);
  get(&cnt, sizeof(int) * nblocks);
  get(&ofs, sizeof(int) * (nblocks + 1));
  const int wgrid = (nblocks + kBlock / kWave - 1) / (kBlock / kWave);  // a wave per block
  const int sgrid = (nsuper + kBlock / kWave - 1) / (kBlock / kWave);   // a wave per super-block
  std::vector<float> htau(nseg, std::numeric_limits<float>::infinity());
  std::vector<int> hofs;
  hipError_t e = hipSuccess;
  if (st == FGA_OK) {
    e = hipMemcpyAsync(sg, hs.data(), sizeof(GSeg) * nseg, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && f > 0) {
      // tau per segment from the median diagonal of its aligned blocks
      k_block_diag<<<wgrid, kBlock, 0, s>>>(Q, sg, nseg, nblocks, G, d2);
      std::vector<float> hd(nblocks);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), d2, sizeof(float) * nblocks, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      for (int k = 0; k < nseg && e == hipSuccess; ++k) {
        const int b0 = hs[k].blk0, nb = (k + 1 < nseg ? hs[k + 1].blk0 : nblocks) - b0;
        if (nb == 0) continue;
        std::nth_element(hd.begin() + b0, hd.begin() + b0 + nb / 2, hd.begin() + b0 + nb);
        const float med = hd[b0 + nb / 2];
        if (med > 0) htau[k] = (float)(f * f) * med;
      }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(tau2, htau.data(), sizeof(float) * nseg, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      k_next<<<(int)((ntot + kBlock - 1) / kBlock), kBlock, 0, s>>>(Q, sg, nseg, ntot, G, tau2, next);
      k_block_maps<<<wgrid, kBlock, 0, s>>>(sg, nseg, nblocks, G, next, F);
      k_super_maps<<<sgrid, kBlock, 0, s>>>(sg, nseg, nsuper, G, F, H);
      k_super_entries<<<nseg, kBlock, 0, s>>>(sg, G, H, E);
      k_block_entries<<<sgrid, kBlock, 0, s>>>(sg, nseg, nsuper, G, F, E, eb);
      k_block_runs<<<(nblocks + kBlock - 1) / kBlock, kBlock, 0, s>>>(sg, nseg, nblocks, G, next, eb, slots, cnt);
      k_scan_counts<<<1, kBlock, 0, s>>>(cnt, nblocks, ofs);
      k_compact_runs<<<wgrid, kBlock, 0, s>>>(slots, cnt, ofs, nblocks, G, table);
      e = hipGetLastError();
    }
    hofs.resize(nblocks + 1);
    if (e == hipSuccess) e = hipMemcpyAsync(hofs.data(), ofs, sizeof(int) * (nblocks + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::vector<int2> ht;
    if (e == hipSuccess) {
      ht.resize(hofs[nblocks]);
      e = hipMemcpyAsync(ht.data(), table, sizeof(int2) * ht.size(), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
      for (int k = 0; k < nseg; ++k) {
        const int g0 = hofs[hs[k].blk0], g1 = hofs[k + 1 < nseg ? hs[k + 1].blk0 : nblocks];
        out[k].assign(ht.begin() + g0, ht.begin() + g1);
      }
  }
  for (void* p : {(void*)sg, (void*)d2, (void*)tau2, (void*)next, (void*)F, (void*)H, (void*)E,
                  (void*)eb, (void*)slots, (void*)table, (void*)cnt, (void*)ofs})
    if (p) pool_free(p, s);
  if (st != FGA_OK) return st;
  if (e != hipSuccess) {
    set_error("group tables: %s", hipGetErrorString(e));
    return FGA_E_DEVICE;
  }
  return FGA_OK;
}

}  // namespace fga
