// Block-level reductions and prefix sums used by several kernels.
#pragma once
#include "common.h"

namespace fga {

// Sum of K doubles over a block of kBlock threads; the result is valid in
// thread 0. Fixed shuffle/LDS order, so it is deterministic.
template <int K>
__device__ inline void block_sum(double (&v)[K], double* lds /* >= K * kBlock/kWave */) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    v[k] = x;
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[w * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int ww = 0; ww < kBlock / kWave; ++ww) s += lds[ww * K + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

template <int K>
__device__ inline void block_minmax(double (&mn)[K], double (&mx)[K], double* lds) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a = mn[k], b = mx[k];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      a = fmin(a, __shfl_xor(a, o, kWave));
      b = fmax(b, __shfl_xor(b, o, kWave));
    }
    mn[k] = a;
    mx[k] = b;
  }
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      lds[w * 2 * K + k] = mn[k];
      lds[w * 2 * K + K + k] = mx[k];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = lds[k], b = lds[K + k];
      for (int ww = 1; ww < kBlock / kWave; ++ww) {
        a = fmin(a, lds[ww * 2 * K + k]);
        b = fmax(b, lds[ww * 2 * K + K + k]);
      }
      mn[k] = a;
      mx[k] = b;
    }
  }
  __syncthreads();
}

// Inclusive prefix sum over a wave (Hillis-Steele with shuffles).
template <typename T>
__device__ inline T wave_incl_scan(T x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

// Inclusive prefix sum / maximum over a wave with DPP moves (no LDS round
// trips): shifts by 1, 2, 4 and 8 within rows of 16 lanes, then the last lane
// of row 0 and of row 2 broadcast to the next row (row_bcast:15, rows 1 and
// 3), then lane 31 to rows 2 and 3 (row_bcast:31). Lanes shifted in from
// outside a row read 0, the identity of both operations (unsigned maximum),
// so each step compiles to one DPP add or max. Must be called with all 64
// lanes active.
__device__ inline int wave_incl_sum_dpp(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, true);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, true);  // row_bcast:31
  return x;
}
__device__ inline unsigned wave_incl_max_u32(unsigned x) {
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true));
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true));
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true));
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true));
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, true));
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, true));
  return x;
}

// Exclusive prefix sum over the block; returns the block total in *total.
template <typename T>
__device__ inline T block_excl_scan(T x, T* lds /* kBlock/kWave */, T* total) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  T inc = wave_incl_scan(x);
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  T base = T(0), tot = T(0);
  for (int ww = 0; ww < kBlock / kWave; ++ww) {
    if (ww < w) base += lds[ww];
    tot += lds[ww];
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

// Wave-wide minimum of an unsigned value, broadcast as a uniform value. Must be
// called with all 64 lanes active. Butterfly within rows of 16 lanes with DPP
// (quad_perm swaps, half-row and row mirrors), then the four row results are
// combined with lane reads.
__device__ inline unsigned wave_min_u32(unsigned v) {
  unsigned t;
  t = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  v = min(v, t);
  t = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  v = min(v, t);
  t = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v = min(v, t);
  t = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  v = min(v, t);
  unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return min(min(r0, r1), min(r2, r3));
}

}  // namespace fga
