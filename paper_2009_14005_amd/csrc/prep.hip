// Step a0 of the hot path, once per registration: the Appendix A
// normalisation (Eqs. A.1-A.3) and the smooth-particle masses (Eq.
// Normalized_IntrinsicVol, Eq. FinalSPM with B = 1), then packing of both
// clouds into the vec4 layouts the force kernels read.
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
};
struct Chunk {
  int seg;
  int pad_;
  int64_t start, count;
};
struct SegStats {           // device, per cloud
  double mean[3];
  double lo[3], hi[3];      // box of the normalised coordinates
  double niv_sum;
  unsigned nonfinite;
  int pad_;
};
struct PairStats {          // device, per pair
  double l, r;              // Eq. (A.2)
  double mu0[3];            // mean of the normalised template
};

struct PrepConsts {
  double a, b;
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

__global__ __launch_bounds__(kBlock) void k_fin_mean(const Seg* segs, const double* part,
                                                     SegStats* ss) {
  const Seg sg = segs[blockIdx.x];
  if (threadIdx.x == 0) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < sg.nchunk; ++c)
      for (int k = 0; k < 4; ++k) s[k] += part[(sg.chunk0 + c) * kPart + k];
    for (int k = 0; k < 3; ++k) ss[blockIdx.x].mean[k] = s[k] / (double)sg.n;
    ss[blockIdx.x].nonfinite = (unsigned)s[3];
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
__global__ void k_fin_lr(const Seg* segs, const double* part, PairStats* ps, PrepConsts c) {
  if (threadIdx.x != 0) return;
  const int p = blockIdx.x;
  double l = INFINITY, r = -INFINITY;
  for (int s = 2 * p; s < 2 * p + 2; ++s)
    for (int k = 0; k < segs[s].nchunk; ++k) {
      l = fmin(l, part[(segs[s].chunk0 + k) * kPart + 0]);
      r = fmax(r, part[(segs[s].chunk0 + k) * kPart + 1]);
    }
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

__global__ void k_fin_box(const Seg* segs, const double* part, SegStats* ss) {
  if (threadIdx.x != 0) return;
  const Seg sg = segs[blockIdx.x];
  for (int a = 0; a < 3; ++a) {
    double mn = INFINITY, mx = -INFINITY;
    for (int k = 0; k < sg.nchunk; ++k) {
      mn = fmin(mn, part[(sg.chunk0 + k) * kPart + a]);
      mx = fmax(mx, part[(sg.chunk0 + k) * kPart + 3 + a]);
    }
    ss[blockIdx.x].lo[a] = mn;
    ss[blockIdx.x].hi[a] = mx;
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

__device__ inline double niv_vcell(const SegStats& st, int rho) {
  double v = 1.0;
  for (int a = 0; a < 3; ++a) {
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
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_nivsum(const Seg* segs, const Chunk* chunks,
                                                   const SegStats* ss, const PairStats* ps,
                                                   PrepConsts c, const unsigned* hist,
                                                   double* part) {
  __shared__ double lds[kBlock / kWave];
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  const double vc = niv_vcell(st, c.rho);
  double v[1] = {0.0};
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, ch.start + k, x);
    v[0] += niv_value(hist[sg.hist_off + niv_cell(x, st, c.rho)], vc, c.v_ball);
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x * kPart] = v[0];
}

__global__ void k_fin_niv(const Seg* segs, const double* part, SegStats* ss) {
  if (threadIdx.x != 0) return;
  const Seg sg = segs[blockIdx.x];
  double s = 0.0;
  for (int k = 0; k < sg.nchunk; ++k) s += part[(sg.chunk0 + k) * kPart];
  ss[blockIdx.x].niv_sum = s;
}

// ---------------------------------------------------------------- stage F
// Reference -> (x, y, z, m) with sum m = 1. Template -> (q, c) with
// q = y_n - mu0 and c the per-particle damping coefficient: eta (fraction
// damping) or eta dt / m_Y (literal damping, m_Y normalised to mean 1).
template <typename Tin, typename T>
__global__ __launch_bounds__(kBlock) void k_pack(const Seg* segs, const Chunk* chunks,
                                                 const SegStats* ss, const PairStats* ps,
                                                 PrepConsts c, const unsigned* hist,
                                                 vec4_t<T>* outX, vec4_t<T>* outQ) {
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  const double vc = niv_vcell(st, c.rho);
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    normalised<Tin>(sg, st, ps, c, ch.start + k, x);
    double w;
    if (c.mass_mode == FGA_MASS_UNIFORM) {
      w = sg.is_y ? 1.0 : 1.0 / (double)sg.n;
    } else {
      const double nv = niv_value(hist[sg.hist_off + niv_cell(x, st, c.rho)], vc, c.v_ball);
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

__global__ void k_fin_state(const Seg* segs, const double* part, const PairStats* ps,
                            RigidState* st, double tol, int max_iter, double rank_tol) {
  if (threadIdx.x != 0) return;
  const int p = blockIdx.x;
  const Seg sg = segs[2 * p + 1];
  double S0[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < sg.nchunk; ++k)
    for (int e = 0; e < 9; ++e) S0[e] += part[(sg.chunk0 + k) * kPart + e];
  rigid_init(st[p], S0, ps[p].mu0, (int)sg.n, tol, max_iter, rank_tol);
}

// masses_only: write the normalised NIV values of one raw cloud.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_write_masses(const Seg* segs, const Chunk* chunks,
                                                         const SegStats* ss, PrepConsts c,
                                                         const unsigned* hist, int norm,
                                                         Tin* out) {
  const Chunk ch = chunks[blockIdx.x];
  const Seg sg = segs[ch.seg];
  const SegStats st = ss[ch.seg];
  const double vc = niv_vcell(st, c.rho);
  const double scale = norm == 0 ? st.niv_sum : st.niv_sum / (double)sg.n;
  for (int64_t k = threadIdx.x; k < ch.count; k += kBlock) {
    double x[3];
    load3<Tin>(sg.p, ch.start + k, x);
    out[ch.start + k] = (Tin)(niv_value(hist[sg.hist_off + niv_cell(x, st, c.rho)], vc, c.v_ball) / scale);
  }
}

// ---------------------------------------------------------------- host side
struct Plan {
  std::vector<Seg> segs;
  std::vector<Chunk> chunks;
  int hist_cells = 0;
};

void plan_add(Plan& pl, const void* p, int64_t n, int pair, int is_y, int64_t out_off, int rho) {
  Seg s;
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

PrepConsts make_consts(const fga_params& p, int identity) {
  PrepConsts c;
  c.a = p.a;
  c.b = p.b;
  const double rb = (p.b - p.a) / (2.0 * (double)p.max_depth * (double)p.rho);
  c.v_ball = 4.0 / 3.0 * M_PI * (rb * rb * rb);
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
                     PrepOut* out, NormInfo* info, hipStream_t s) {
  Plan pl;
  int64_t xoff = 0, yoff = 0;
  for (int k = 0; k < npairs; ++k) {
    plan_add(pl, X[k].p, X[k].n, k, 0, xoff, p.rho);
    plan_add(pl, Y[k].p, Y[k].n, k, 1, yoff, p.rho);
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
  size_t total = o_hist + sizeof(unsigned) * pl.hist_cells;
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
  FGA_HIP(hipMemcpyAsync(dseg, pl.segs.data(), sizeof(Seg) * nseg, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dch, pl.chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemsetAsync(hist, 0, sizeof(unsigned) * pl.hist_cells, s));
  const PrepConsts c = make_consts(p, 0);
  k_sum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, part);
  k_fin_mean<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_minmax<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, part);
  k_fin_lr<<<npairs, 64, 0, s>>>(dseg, part, ps, c);
  k_box<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, part);
  k_fin_box<<<nseg, 64, 0, s>>>(dseg, part, ss);
  if (p.mass_mode == FGA_MASS_NIV) {
    k_hist<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, hist);
    k_nivsum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, hist, part);
    k_fin_niv<<<nseg, 64, 0, s>>>(dseg, part, ss);
  }
  k_pack<Tin, T><<<nch, kBlock, 0, s>>>(dseg, dch, ss, ps, c, hist, (vec4_t<T>*)out->X,
                                        (vec4_t<T>*)out->Q);
  k_s0<T><<<nch, kBlock, 0, s>>>(dseg, dch, (const vec4_t<T>*)out->Q, part);
  // FP32 template coordinates carry ~1e-7 relative rounding, so a collinear
  // template shows singular-value ratios of that order
  const double rank_tol = sizeof(T) == 8 ? 1e-12 : 1e-6;
  k_fin_state<<<npairs, 64, 0, s>>>(dseg, part, ps, out->st, p.tol, p.max_iter, rank_tol);
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
fga_status masses_impl(const void* pts, int64_t n, const fga_params& p, int norm, void* out,
                       hipStream_t s) {
  Plan pl;
  plan_add(pl, pts, n, 0, 0, 0, p.rho);
  const int nseg = 1, nch = (int)pl.chunks.size();
  size_t o_seg = 0, o_ch = sizeof(Seg), o_part = o_ch + sizeof(Chunk) * nch;
  o_part = (o_part + 255) & ~(size_t)255;
  size_t o_ss = o_part + sizeof(double) * kPart * nch;
  size_t o_hist = o_ss + sizeof(SegStats);
  size_t total = o_hist + sizeof(unsigned) * pl.hist_cells;
  DevBufs buf;
  buf.s = s;
  FGA_TRY(pool_get(&buf.mem, total, s));
  char* base = (char*)buf.mem;
  Seg* dseg = (Seg*)(base + o_seg);
  Chunk* dch = (Chunk*)(base + o_ch);
  double* part = (double*)(base + o_part);
  SegStats* ss = (SegStats*)(base + o_ss);
  unsigned* hist = (unsigned*)(base + o_hist);
  FGA_HIP(hipMemcpyAsync(dseg, pl.segs.data(), sizeof(Seg), hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemcpyAsync(dch, pl.chunks.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
  FGA_HIP(hipMemsetAsync(hist, 0, sizeof(unsigned) * pl.hist_cells, s));
  FGA_HIP(hipMemsetAsync(ss, 0, sizeof(SegStats), s));
  const PrepConsts c = make_consts(p, 1);
  k_sum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, part);
  k_fin_mean<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_box<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, nullptr, c, part);
  k_fin_box<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_hist<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, nullptr, c, hist);
  k_nivsum<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, nullptr, c, hist, part);
  k_fin_niv<<<nseg, 64, 0, s>>>(dseg, part, ss);
  k_write_masses<Tin><<<nch, kBlock, 0, s>>>(dseg, dch, ss, c, hist, norm, (Tin*)out);
  FGA_HIP(hipGetLastError());
  SegStats hss;
  FGA_HIP(hipMemcpyAsync(&hss, ss, sizeof(SegStats), hipMemcpyDeviceToHost, s));
  FGA_HIP(hipStreamSynchronize(s));
  if (hss.nonfinite) {
    set_error("%u non-finite coordinates", hss.nonfinite);
    return FGA_E_NONFINITE;
  }
  return FGA_OK;
}

}  // namespace

fga_status prep_pairs(int npairs, const CloudIn* X, const CloudIn* Y, fga_dtype dt,
                      const fga_params& p, PrepOut* out, NormInfo* info, hipStream_t s) {
  const bool f64 = p.precision == FGA_PREC_FP64;
  if (dt == FGA_F32)
    return f64 ? prep_impl<float, double>(npairs, X, Y, p, out, info, s)
               : prep_impl<float, float>(npairs, X, Y, p, out, info, s);
  return f64 ? prep_impl<double, double>(npairs, X, Y, p, out, info, s)
             : prep_impl<double, float>(npairs, X, Y, p, out, info, s);
}

fga_status masses_only(const void* pts, fga_dtype dt, int64_t n, const fga_params& p, int norm,
                       void* out, hipStream_t s) {
  return dt == FGA_F32 ? masses_impl<float>(pts, n, p, norm, out, s)
                       : masses_impl<double>(pts, n, p, norm, out, s);
}

}  // namespace fga
