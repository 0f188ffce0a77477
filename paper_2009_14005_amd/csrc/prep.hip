// Step a0 of the hot path, once per registration: the Appendix A
// normalisation (Eqs. A.1-A.3) and the smooth-particle masses S = N o B
// (Eq. Normalized_IntrinsicVol for N, Eq. RBF_function for B when landmark
// correspondences are given, B = 1 otherwise; Eq. FinalSPM), then packing
// of both clouds into the vec4 layouts the force kernels read.
//
// All reductions are two-stage and deterministic: one block per chunk of
// kChunk points writes partial values, and one block per cloud (or pair)
// combines the partials of its chunks in chunk order. Every cloud of every
// pair is handled by the same launches, so a batch of registrations costs
// the same number of launches as one.
#include <math.h>

#include <vector>

#include "common.h"
#include "reduce.h"
#include "rigid.h"

namespace fga {
namespace {

constexpr int kChunk = kBlock * 16;  // points per chunk
constexpr int kPart = 12;            // doubles of partial data per chunk

struct Seg {                // one cloud
  const void* p;            // input n x 3
  int64_t n;
  int chunk0, nchunk;       // its chunks
  int pair;                 // owning pair
  int is_y;                 // 1 = template
  int64_t out_off;          // offset of its packed output (points)
  int hist_off;             // offset of its histogram (cells)
  int lm_off, lm_cnt;       // its landmark anchors (RBF masses); none: B = 1
};
struct Chunk {
  int seg;
  int pad_;
  int64_t start, count;
};
struct SegStats {           // device, per cloud
  double mean[3];
  double lo[3], hi[3];      // box of the normalised coordinates
  double niv_sum;           // sum of the unnormalised masses N o B
  unsigned nonfinite;
  unsigned lm_singular;     // the RBF collocation system had no usable pivot
};
struct PairStats {          // device, per pair
  double l, r;              // Eq. (A.2)
  double mu0[3];            // mean of the normalised template
};

struct PrepConsts {
  double a, b;
  int dims;                 // 3, or 2 for planar clouds embedded at z = 0
  double rbf_inv_s2;        // 1 / sigma^2 of the RBF kernel Phi(s) = exp(-s^2 / sigma^2)
  double rbf_beta;          // B at a landmark anchor
  double v_ball;            // volume of one point's ball, Eq. (Normalized_IntrinsicVol)
  int rho;
  int mass_mode;
  int identity;             // 1: no normalisation (fga_masses on raw points)
  int damping;
  double eta, dt;
};

template <typename Tin>
__device__ inline void load3(const void* p, int64_t i, double* v) {
  const Tin* q = (const Tin*)p + 3 * i;
  v[0] = (double)q[0];
  v[1] = (double)q[1];
  v[2] = (double)q[2];
}

// Eq. (A.3): ((p - mean - l) (b - a)) / (r - l) + a, evaluated in that order.
__device__ inline double norm1(double p, double mean, double l, double r, double a, double b) {
  return ((p - mean) - l) * (b - a) / (r - l) + a;
}

// ---------------------------------------------------------------- stage A
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_sum(const Seg* segs, const Chunk* chunks,
                                                double* part) {
  __shared__ double lds[4 * kBlock / kWave];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    load3<Tin>(sg.p, ch.start + k, x);
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) v[3] += 1.0;
    v[0] += x[0];
    v[1] += x[1];
    v[2] += x[2];
  }
  block_sum<4>(v, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[blockIdx.x * kPart + k] = v[k];
}

// One wave combines a cloud's chunk partials: lane j takes chunks j, j + 64,
// ..., then a butterfly over the lanes (a fixed order: deterministic).
__device__ inline double wave_sum_d(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ inline double wave_min_d(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ inline double wave_max_d(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__global__ __launch_bounds__(kWave) void k_fin_mean(const Seg* segs, const double* part,
                                                    SegStats* ss) {
  const Seg sg = segs[blockIdx.x];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = (int)threadIdx.x; c < sg.nchunk; c += kWave)
    for (int k = 0; k < 4; ++k) s[k] += part[(sg.chunk0 + c) * kPart + k];
  for (int k = 0; k < 4; ++k) s[k] = wave_sum_d(s[k]);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) ss[blockIdx.x].mean[k] = s[k] / (double)sg.n;
    ss[blockIdx.x].nonfinite = (unsigned)s[3];
    ss[blockIdx.x].lm_singular = 0u;  // set by the collocation solve, if the cloud has landmarks
  }
}

// ---------------------------------------------------------------- stage B
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_minmax(const Seg* segs, const Chunk* chunks,
                                                   const SegStats* ss, double* part) {
  __shared__ double lds[2 * kBlock / kWave];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const double* mean = ss[ch.seg].mean;
  double mn[1] = {INFINITY}, mx[1] = {-INFINITY};
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    load3<Tin>(sg.p, ch.start + k, x);
    for (int a = 0; a < 3; ++a) {
      const double d = x[a] - mean[a];
      mn[0] = fmin(mn[0], d);
      mx[0] = fmax(mx[0], d);
    }
  }
  block_minmax<1>(mn, mx, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x * kPart + 0] = mn[0];
    part[blockIdx.x * kPart + 1] = mx[0];
  }
}

// Eq. (A.2): l and r over both clouds of a pair (segments 2p and 2p + 1).
__global__ __launch_bounds__(kWave) void k_fin_lr(const Seg* segs, const double* part,
                                                  PairStats* ps, PrepConsts c) {
  const int p = blockIdx.x;
  double l = INFINITY, r = -INFINITY;
  for (int s = 2 * p; s < 2 * p + 2; ++s)
    for (int k = (int)threadIdx.x; k < segs[s].nchunk; k += kWave) {
      l = fmin(l, part[(segs[s].chunk0 + k) * kPart + 0]);
      r = fmax(r, part[(segs[s].chunk0 + k) * kPart + 1]);
    }
  l = wave_min_d(l);
  r = wave_max_d(r);
  if (threadIdx.x != 0) return;
  ps[p].l = l;
  ps[p].r = r;
  // mean of the normalised template: Eq. (A.3) applied to a zero centred coordinate
  const double m0 = (0.0 - l) * (c.b - c.a) / (r - l) + c.a;
  for (int a = 0; a < 3; ++a) ps[p].mu0[a] = m0;
}

template <typename Tin>
__device__ inline void normalised(const Seg& sg, const SegStats& st, const PairStats* ps,
                                  const PrepConsts& c, int64_t i, double* x) {
  load3<Tin>(sg.p, i, x);
  if (c.identity) return;
  const PairStats& pr = ps[sg.pair];
  for (int a = 0; a < 3; ++a) x[a] = norm1(x[a], st.mean[a], pr.l, pr.r, c.a, c.b);
}

// ------------------------------------------------------- RBF landmarks
// Eq. (RBF_function): B(p) = 1 + sum_c lambda_c exp(-|p - a_c|^2 / sigma^2)
// over the cloud's anchors a_c (x, y, z, lambda_c), B = 1 without anchors.
__device__ inline double rbf_B(const double* x, const double4* lmk, const Seg& sg, double inv_s2) {
  double b = 1.0;
  for (int k = 0; k < sg.lm_cnt; ++k) {
    const double4 a = lmk[sg.lm_off + k];
    const double dx = x[0] - a.x, dy = x[1] - a.y, dz = x[2] - a.z;
    b += a.w * exp(-(dx * dx + dy * dy + dz * dz) * inv_s2);
  }
  return b;
}

// The collocation system of one cloud (one block per cloud): anchors in the
// frame the masses are computed in, Phi_cc' lambda = (beta - 1) 1, solved by
// Gaussian elimination without pivoting (Phi is symmetric positive definite
// for distinct anchors); one thread per row, the back substitution on one.
constexpr int kMaxLandmarks = 64;
template <typename Tin>
__global__ __launch_bounds__(kMaxLandmarks) void k_rbf_solve(const Seg* segs, const SegStats* ss,
                                                             const PairStats* ps, PrepConsts c,
                                                             const int64_t* lm_idx, double4* lmk,
                                                             SegStats* ss_out) {
  __shared__ double A[kMaxLandmarks][kMaxLandmarks + 1];
  __shared__ double rhs[kMaxLandmarks], anc[kMaxLandmarks][3];
  __shared__ int bad;
  const Seg sg = segs[blockIdx.x];
  const int m = sg.lm_cnt, i = (int)threadIdx.x;
  if (m == 0) return;
  const SegStats st = ss[blockIdx.x];
  if (i == 0) bad = 0;
  if (i < m) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, lm_idx[sg.lm_off + i], x);
    for (int a = 0; a < 3; ++a) anc[i][a] = x[a];
  }
  __syncthreads();
  if (i < m) {
    for (int j = 0; j < m; ++j) {
      const double dx = anc[i][0] - anc[j][0], dy = anc[i][1] - anc[j][1], dz = anc[i][2] - anc[j][2];
      A[i][j] = exp(-(dx * dx + dy * dy + dz * dz) * c.rbf_inv_s2);
    }
    rhs[i] = c.rbf_beta - 1.0;
  }
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    const double piv = A[k][k];
    if (!(piv > 1e-12)) {  // coincident or nearly coincident anchors
      if (i == 0) bad = 1;
      break;
    }
    if (i > k && i < m) {
      const double f = A[i][k] / piv;
      for (int j = k; j < m; ++j) A[i][j] -= f * A[k][j];
      rhs[i] -= f * rhs[k];
    }
  }
  __syncthreads();
  if (i == 0) {
    if (!bad) {
      for (int k = m - 1; k >= 0; --k) {
        double v = rhs[k];
        for (int j = k + 1; j < m; ++j) v -= A[k][j] * rhs[j];
        rhs[k] = v / A[k][k];
      }
    }
    ss_out[blockIdx.x].lm_singular = bad ? 1u : 0u;
  }
  __syncthreads();
  if (i < m) lmk[sg.lm_off + i] = make_double4(anc[i][0], anc[i][1], anc[i][2], bad ? 0.0 : rhs[i]);
}

// ---------------------------------------------------------------- stage C
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_box(const Seg* segs, const Chunk* chunks,
                                                const SegStats* ss, const PairStats* ps,
                                                PrepConsts c, double* part) {
  __shared__ double lds[6 * kBlock / kWave];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, ch.start + k, x);
    for (int a = 0; a < 3; ++a) {
      mn[a] = fmin(mn[a], x[a]);
      mx[a] = fmax(mx[a], x[a]);
    }
  }
  block_minmax<3>(mn, mx, lds);
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) {
      part[blockIdx.x * kPart + a] = mn[a];
      part[blockIdx.x * kPart + 3 + a] = mx[a];
    }
}

__global__ __launch_bounds__(kWave) void k_fin_box(const Seg* segs, const double* part, SegStats* ss) {
  const Seg sg = segs[blockIdx.x];
  for (int a = 0; a < 3; ++a) {
    double mn = INFINITY, mx = -INFINITY;
    for (int k = (int)threadIdx.x; k < sg.nchunk; k += kWave) {
      mn = fmin(mn, part[(sg.chunk0 + k) * kPart + a]);
      mx = fmax(mx, part[(sg.chunk0 + k) * kPart + 3 + a]);
    }
    mn = wave_min_d(mn);
    mx = wave_max_d(mx);
    if (threadIdx.x == 0) {
      ss[blockIdx.x].lo[a] = mn;
      ss[blockIdx.x].hi[a] = mx;
    }
  }
}

// NIV lattice cell of a point: min(floor(rho (p - lo) / ext), rho - 1) per
// axis, a zero-extent axis counting as extent 1.
__device__ inline int niv_cell(const double* x, const SegStats& st, int rho) {
  int idx = 0;
  for (int a = 0; a < 3; ++a) {
    double ext = st.hi[a] - st.lo[a];
    if (!(ext > 0.0)) ext = 1.0;
    double f = floor(((double)rho * (x[a] - st.lo[a])) / ext);
    int q = f < 0.0 ? 0 : (f > (double)(rho - 1) ? rho - 1 : (int)f);
    idx = idx * rho + q;
  }
  return idx;
}

__device__ inline double niv_vcell(const SegStats& st, int rho, int dims) {
  double v = 1.0;
  for (int a = 0; a < dims; ++a) {
    double ext = st.hi[a] - st.lo[a];
    if (!(ext > 0.0)) ext = 1.0;
    v *= ext / (double)rho;
  }
  return v;
}

// NIV value V_cell / min(n_c V_ball, V_cell).
__device__ inline double niv_value(unsigned n_c, double v_cell, double v_ball) {
  return v_cell / fmin((double)n_c * v_ball, v_cell);
}

// ---------------------------------------------------------------- stage D
// Counts per lattice cell. Up to 16^3 cells the block counts its chunk in
// LDS and adds only its non-zero cells to the global histogram (the points of
// a scan crowd into few cells, where global atomics would queue up).
constexpr int kHistLds = 4096;
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_hist(const Seg* segs, const Chunk* chunks,
                                                 const SegStats* ss, const PairStats* ps,
                                                 PrepConsts c, unsigned* hist) {
  __shared__ unsigned lh[kHistLds];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  const int cells = c.rho * c.rho * c.rho;
  if (cells > kHistLds) {
    for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
      double x[3];
      normalised<Tin>(sg, st, ps, c, ch.start + k, x);
      atomicAdd(&hist[sg.hist_off + niv_cell(x, st, c.rho)], 1u);
    }
    return;
  }
  for (int k = (int)threadIdx.x; k < cells; k += kBlock) lh[k] = 0u;
  __syncthreads();
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, ch.start + k, x);
    atomicAdd(&lh[niv_cell(x, st, c.rho)], 1u);
  }
  __syncthreads();
  for (int k = (int)threadIdx.x; k < cells; k += kBlock)
    if (lh[k]) atomicAdd(&hist[sg.hist_off + k], lh[k]);
}

// ---------------------------------------------------------------- stage E
// Unnormalised mass N o B of a point (N = 1 in uniform mode).
__device__ inline double spm_value(const double* x, const Seg& sg, const SegStats& st,
                                   const PrepConsts& c, const unsigned* hist, const double4* lmk) {
  const double nv = c.mass_mode == FGA_MASS_UNIFORM
                        ? 1.0
                        : niv_value(hist[sg.hist_off + niv_cell(x, st, c.rho)], niv_vcell(st, c.rho, c.dims), c.v_ball);
  return sg.lm_cnt ? nv * rbf_B(x, lmk, sg, c.rbf_inv_s2) : nv;
}

template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_nivsum(const Seg* segs, const Chunk* chunks,
                                                   const SegStats* ss, const PairStats* ps,
                                                   PrepConsts c, const unsigned* hist,
                                                   const double4* lmk, double* part) {
  __shared__ double lds[kBlock / kWave];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  double v[1] = {0.0};
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, ch.start + k, x);
    v[0] += spm_value(x, sg, st, c, hist, lmk);
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x * kPart] = v[0];
}

__global__ __launch_bounds__(kWave) void k_fin_niv(const Seg* segs, const double* part, SegStats* ss) {
  const Seg sg = segs[blockIdx.x];
  double s = 0.0;
  for (int k = (int)threadIdx.x; k < sg.nchunk; k += kWave) s += part[(sg.chunk0 + k) * kPart];
  s = wave_sum_d(s);
  if (threadIdx.x == 0) ss[blockIdx.x].niv_sum = s;
}

// ---------------------------------------------------------------- stage F
// Reference -> (x, y, z, m) with sum m = 1. Template -> (q, c) with
// q = y_n - mu0 and c the per-particle damping coefficient: eta (fraction
// damping) or eta dt / m_Y (literal damping, m_Y normalised to mean 1).
template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void k_pack(const Seg* segs, const Chunk* chunks,
                                                 const SegStats* ss, const PairStats* ps,
                                                 PrepConsts c, const unsigned* hist,
                                                 const double4* lmk, vec4_t<T>* outX,
                                                 vec4_t<T>* outQ) {
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, ch.start + k, x);
    double w;
    if (c.mass_mode == FGA_MASS_UNIFORM && sg.lm_cnt == 0) {
      w = sg.is_y ? 1.0 : 1.0 / (double)sg.n;
    } else {
      const double nv = spm_value(x, sg, st, c, hist, lmk);
      w = sg.is_y ? nv / (st.niv_sum / (double)sg.n) : nv / st.niv_sum;
    }
    if (!sg.is_y) {
      outX[sg.out_off + ch.start + k] = make4<T>((T)x[0], (T)x[1], (T)x[2], (T)w);
    } else {
      const double* mu0 = ps[sg.pair].mu0;
      const double cc = c.damping == FGA_DAMP_LITERAL ? c.eta * c.dt / w : c.eta;
      outQ[sg.out_off + ch.start + k] =
          make4<T>((T)(x[0] - mu0[0]), (T)(x[1] - mu0[1]), (T)(x[2] - mu0[2]), (T)cc);
    }
  }
}

// ---------------------------------------------------------------- stage G
// S0 = sum q q^T of the stored (rounded) template coordinates.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_s0(const Seg* segs, const Chunk* chunks,
                                               const vec4_t<T>* Q, double* part) {
  __shared__ double lds[9 * kBlock / kWave];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (sg.is_y) {
    for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
      const vec4_t<T> q = Q[sg.out_off + ch.start + k];
      const double qq[3] = {(double)q.x, (double)q.y, (double)q.z};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) v[3 * a + b] += qq[a] * qq[b];
    }
  }
  block_sum<9>(v, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 9; ++k) part[blockIdx.x * kPart + k] = v[k];
}

__global__ __launch_bounds__(kWave) void k_fin_state(const Seg* segs, const double* part,
                                                     const PairStats* ps, RigidState* st,
                                                     double tol, int max_iter, double rank_tol,
                                                     int dims) {
  const int p = blockIdx.x;
  const Seg sg = segs[2 * p + 1];
  double S0[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = (int)threadIdx.x; k < sg.nchunk; k += kWave)
    for (int e = 0; e < 9; ++e) S0[e] += part[(sg.chunk0 + k) * kPart + e];
  for (int e = 0; e < 9; ++e) S0[e] = wave_sum_d(S0[e]);
  if (threadIdx.x != 0) return;
  rigid_init(st[p], S0, ps[p].mu0, (int)sg.n, tol, max_iter, rank_tol, dims);
}

// masses_only: write the normalised masses N o B of one raw cloud.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_write_masses(const Seg* segs, const Chunk* chunks,
                                                         const SegStats* ss, PrepConsts c,
                                                         const unsigned* hist, const double4* lmk,
                                                         int norm, Tin* out) {
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  const double scale = norm == 0 ? st.niv_sum : st.niv_sum / (double)sg.n;
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    load3<Tin>(sg.p, ch.start + k, x);
    out[ch.start + k] = (Tin)(spm_value(x, sg, st, c, hist, lmk) / scale);
  }
}

// ---------------------------------------------------------------- host side
struct Plan {
  std::vector<Seg> segs;
  std::vector<Chunk> chunks;
  std::vector<int64_t> lm;  // landmark point indices of every cloud, in cloud order
  int hist_cells = 0;
};

void plan_add(Plan& pl, const void* p, int64_t n, int pair, int is_y, int64_t out_off, int rho,
              const int64_t* lm = nullptr, int n_lm = 0) {
  Seg s;
  s.lm_off = (int)pl.lm.size();
  s.lm_cnt = lm ? n_lm : 0;
  for (int k = 0; k < s.lm_cnt; ++k) pl.lm.push_back(lm[k]);
  s.p = p;
  s.n = n;
  s.chunk0 = (int)pl.chunks.size();
  s.nchunk = (int)((n + kChunk - 1) / kChunk);
  s.pair = pair;
  s.is_y = is_y;
  s.out_off = out_off;
  s.hist_off = pl.hist_cells;
  pl.hist_cells += rho * rho * rho;
  for (int k = 0; k < s.nchunk; ++k) {
    Chunk c;
    c.seg = (int)pl.segs.size();
    c.pad_ = 0;
    c.start = (int64_t)k * kChunk;
    c.count = (n - c.start) < kChunk ? (n - c.start) : kChunk;
    pl.chunks.push_back(c);
  }
  pl.segs.push_back(s);
}

struct DevBufs {
  void* mem = nullptr;
  hipStream_t s = nullptr;
  ~DevBufs() {
    if (mem) pool_free(mem, s);
  }
};

PrepConsts make_consts(const fga_params& p, int identity, int dims = 3) {
  PrepConsts c;
  c.a = p.a;
  c.b = p.b;
  c.dims = dims;
  c.rbf_inv_s2 = 1.0 / (p.rbf_sigma * p.rbf_sigma);
  c.rbf_beta = p.rbf_weight;
  const double rb = (p.b - p.a) / (2.0 * (double)p.max_depth * (double)p.rho);
  // one point's ball (Eq. Normalized_IntrinsicVol): a disc in D = 2
  c.v_ball = dims == 2 ? M_PI * (rb * rb) : 4.0 / 3.0 * M_PI * (rb * rb * rb);
  c.rho = p.rho;
  c.mass_mode = p.mass_mode;
  c.identity = identity;
  c.damping = p.damping;
  c.eta = p.eta;
  c.dt = p.dt;
  return c;
}

template <typename Tin, typename T>
fga_status prep_impl(int npairs, const CloudIn* X, const CloudIn* Y, const fga_params& p,
                     PrepOut* out, NormInfo* info, hipStream_t s, int dims) {
  Plan pl;
  int64_t xoff = 0, yoff = 0;
  for (int k = 0; k < npairs; ++k) {
    plan_add(pl, X[k].p, X[k].n, k, 0, xoff, p.rho, X[k].lm, X[k].n_lm);
    plan_add(pl, Y[k].p, Y[k].n, k, 1, yoff, p.rho, Y[k].lm, Y[k].n_lm);
    xoff += X[k].n;
    yoff += Y[k].n;
  }
  const int nseg = (int)pl.segs.size(), nch = (int)pl.chunks.size();
  // one device block for all scratch
  size_t o_seg = 0, o_ch = o_seg + sizeof(Seg) * nseg, o_part = o_ch + sizeof(Chunk) * nch;
  o_part = (o_part + 255) & ~(size_t)255;
  size_t o_ss = o_part + sizeof(double) * kPart * nch;
  size_t o_ps = o_ss + sizeof(SegStats) * nseg;
  size_t o_hist = o_ps + sizeof(PairStats) * npairs;
  size_t o_lmi = (o_hist + sizeof(unsigned) * pl.hist_cells + 255) & ~(size_t)255;
  size_t o_lmk = o_lmi + sizeof(int64_t) * pl.lm.size();
  size_t total = o_lmk + sizeof(double4) * pl.lm.size();
  DevBufs buf;
  buf.s = s;
  FGA_TRY(pool_get(&buf.mem, total, s));
  char* base = (char*)buf.mem;
  Seg* dseg = (Seg*)(base + o_seg);
  Chunk* dch = (Chunk*)(base + o_ch);
  double* part = (double*)(base + o_part);
  SegStats* ss = (SegStats*)(base + o_ss);
  PairStats* ps = (PairStats*)(base + o_ps);
  unsigned* hist = (unsigned*)(base + o_hist);
  int64_t* lmi = (int64_t*)(base + o_lmi);
  double4* lmk = (double4*)(base + o_lmk);
  const bool any_lm = !pl.lm.empty();
  if (any_lm)
    FGA_HIP(hipMemcpyAsync(lmi, pl.lm.data(), sizeof(int64_t) * pl.lm.size(), hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dseg, pl.segs.data(), sizeof(Seg) * nseg, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dch, pl.chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemsetAsync(hist, 0, sizeof(unsigned) * pl.hist_cells, s));
  const PrepConsts c = make_consts(p, 0, dims);
  k_sum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, part);
  k_fin_mean<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_minmax<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, part);
  k_fin_lr<<<npairs, 64, 0, s>>>(dseg, part, ps, c);
  k_box<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, part);
  k_fin_box<<<nseg, 64, 0, s>>>(dseg, part, ss);
  if (any_lm) k_rbf_solve<Tin><<<nseg, kMaxLandmarks, 0, s>>>(dseg, ss, ps, c, lmi, lmk, ss);
  if (p.mass_mode == FGA_MASS_NIV) k_hist<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, hist);
  if (p.mass_mode == FGA_MASS_NIV || any_lm) {
    k_nivsum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, hist, lmk, part);
    k_fin_niv<<<nseg, 64, 0, s>>>(dseg, part, ss);
  }
  k_pack<Tin, T><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, hist, lmk, (vec4_t<T>*)out->X,
                                        (vec4_t<T>*)out->Q);
  k_s0<T><<<nch, kBlock, 0, s>>>(dseg, dch, (const vec4_t<T>*)out->Q, part);
  // FP32 template coordinates carry ~1e-7 relative rounding, so a collinear
  // template shows singular-value ratios of that order
  const double rank_tol = sizeof(T) == 8 ? 1e-12 : 1e-6;
  k_fin_state<<<npairs, 64, 0, s>>>(dseg, part, ps, out->st, p.tol, p.max_iter, rank_tol, dims);
  FGA_HIP(hipGetLastError());
  // host copies for validation and de-normalisation (one sync per prep)
  std::vector<SegStats> hss(nseg);
  std::vector<PairStats> hps(npairs);
  FGA_HIP(hipMemcpyAsync(hss.data(), ss, sizeof(SegStats) * nseg, hipMemcpyDeviceToHost, s));
  FGA_HIP(hipMemcpyAsync(hps.data(), ps, sizeof(PairStats) * npairs, hipMemcpyDeviceToHost, s));
  FGA_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < npairs; ++k) {
    const SegStats& sx = hss[2 * k];
    const SegStats& sy = hss[2 * k + 1];
    if (sx.nonfinite || sy.nonfinite) {
      set_error("pair %d: %u non-finite reference and %u non-finite template values", k,
                sx.nonfinite, sy.nonfinite);
      return FGA_E_NONFINITE;
    }
    if (sx.lm_singular || sy.lm_singular) {
      set_error("pair %d: landmark points (nearly) coincide within the RBF width: the "
                "collocation system is singular", k);
      return FGA_E_DEGENERATE;
    }
    if (!(hps[k].r > hps[k].l)) {
      set_error("pair %d: both clouds have zero extent (r == l in Eq. A.2)", k);
      return FGA_E_DEGENERATE;
    }
    for (int a = 0; a < 3; ++a) {
      info[k].xbar[a] = sx.mean[a];
      info[k].ybar[a] = sy.mean[a];
    }
    info[k].l = hps[k].l;
    info[k].r = hps[k].r;
    info[k].a = p.a;
    info[k].b = p.b;
  }
  return FGA_OK;
}

template <typename Tin>
fga_status masses_impl(const void* pts, int64_t n, const int64_t* lm, int n_lm,
                       const fga_params& p, int norm, void* out, hipStream_t s) {
  Plan pl;
  plan_add(pl, pts, n, 0, 0, 0, p.rho, lm, n_lm);
  const int nseg = 1, nch = (int)pl.chunks.size();
  size_t o_seg = 0, o_ch = sizeof(Seg), o_part = o_ch + sizeof(Chunk) * nch;
  o_part = (o_part + 255) & ~(size_t)255;
  size_t o_ss = o_part + sizeof(double) * kPart * nch;
  size_t o_hist = o_ss + sizeof(SegStats);
  size_t o_lmi = (o_hist + sizeof(unsigned) * pl.hist_cells + 255) & ~(size_t)255;
  size_t o_lmk = o_lmi + sizeof(int64_t) * pl.lm.size();
  size_t total = o_lmk + sizeof(double4) * pl.lm.size();
  DevBufs buf;
  buf.s = s;
  FGA_TRY(pool_get(&buf.mem, total, s));
  char* base = (char*)buf.mem;
  Seg* dseg = (Seg*)(base + o_seg);
  Chunk* dch = (Chunk*)(base + o_ch);
  double* part = (double*)(base + o_part);
  SegStats* ss = (SegStats*)(base + o_ss);
  unsigned* hist = (unsigned*)(base + o_hist);
  int64_t* lmi = (int64_t*)(base + o_lmi);
  double4* lmk = (double4*)(base + o_lmk);
  if (!pl.lm.empty())
    FGA_HIP(hipMemcpyAsync(lmi, pl.lm.data(), sizeof(int64_t) * pl.lm.size(), hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dseg, pl.segs.data(), sizeof(Seg), hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dch, pl.chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemsetAsync(hist, 0, sizeof(unsigned) * pl.hist_cells, s));
  FGA_HIP(hipMemsetAsync(ss, 0, sizeof(SegStats), s));
  const PrepConsts c = make_consts(p, 1);
  k_sum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, part);
  k_fin_mean<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_box<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, nullptr, c, part);
  k_fin_box<<<nseg, 64, 0, s>>>(dseg, part, ss);
  if (!pl.lm.empty()) k_rbf_solve<Tin><<<nseg, kMaxLandmarks, 0, s>>>(dseg, ss, nullptr, c, lmi, lmk, ss);
  if (p.mass_mode == FGA_MASS_NIV) k_hist<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, nullptr, c, hist);
  k_nivsum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, nullptr, c, hist, lmk, part);
  k_fin_niv<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_write_masses<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, c, hist, lmk, norm, (Tin*)out);
  FGA_HIP(hipGetLastError());
  SegStats hss;
  FGA_HIP(hipMemcpyAsync(&hss, ss, sizeof(SegStats), hipMemcpyDeviceToHost, s));
  FGA_HIP(hipStreamSynchronize(s));
  if (hss.nonfinite) {
    set_error("%u non-finite coordinates", hss.nonfinite);
    return FGA_E_NONFINITE;
  }
  if (hss.lm_singular) {
    set_error("landmark points (nearly) coincide within the RBF width: the collocation system is singular");
    return FGA_E_DEGENERATE;
  }
  return FGA_OK;
}

}  // namespace

fga_status prep_pairs(int npairs, const CloudIn* X, const CloudIn* Y, fga_dtype dt,
                      const fga_params& p, PrepOut* out, NormInfo* info, hipStream_t s, int dims) {
  const bool f64 = p.precision == FGA_PREC_FP64;
  if (dt == FGA_F32)
    return f64 ? prep_impl<float, double>(npairs, X, Y, p, out, info, s, dims)
               : prep_impl<float, float>(npairs, X, Y, p, out, info, s, dims);
  return f64 ? prep_impl<double, double>(npairs, X, Y, p, out, info, s, dims)
             : prep_impl<double, float>(npairs, X, Y, p, out, info, s, dims);
}

fga_status masses_only(const void* pts, fga_dtype dt, int64_t n, const int64_t* lm, int n_lm,
                       const fga_params& p, int norm, void* out, hipStream_t s) {
  return dt == FGA_F32 ? masses_impl<float>(pts, n, lm, n_lm, p, norm, out, s)
                       : masses_impl<double>(pts, n, lm, n_lm, p, norm, out, s);
}

}  // namespace fga
