/*
 * fga.h — C ABI of the MI355X-native Fast Gravitational Approach (FGA) library.
 *
 * FGA (arXiv 2009.14005) registers a template point set Y (M x 3) to a
 * reference point set X (N x 3) by letting the static reference pull every
 * template particle with a softened gravitational force (Eq. GAForce),
 * integrating a damped second-order ODE (Eqs. GAForceDissipative,
 * TotalGAForce, PreviousVelocity) and projecting the particle displacements
 * onto one rigid motion with the Kabsch solution (Eqs. R_Kabsch, transEst),
 * iterated as in Alg. 2. The pull is evaluated either as the exact all-pairs
 * sum or with the Barnes-Hut octree of Alg. 1 and the BHForce traversal of
 * Alg. 2 (acceptance criterion Eq. MAC).
 *
 * Conventions for every entry point:
 *   - Point arrays are contiguous row-major n x 3 DEVICE arrays of the given
 *     dtype (float or double). Mass arrays are contiguous DEVICE vectors of
 *     the same dtype. The caller owns every buffer passed in.
 *   - R (row-major 3x3), t (3) and reports are HOST memory, FP64.
 *     Registration results satisfy X ~= R * Y + t in the caller's coordinates.
 *   - `stream` is a hipStream_t (NULL = the default stream). Work is queued on
 *     it; functions that return host results synchronise that stream.
 *   - Every function returns an fga_status and never aborts. Argument checks
 *     happen on the host before any device work. A non-OK status leaves a
 *     thread-local message readable with fga_last_error().
 *   - Non-convergence is not an error: the report carries converged = 0.
 *   - One library instance per process drives the current HIP device. States
 *     are not thread-safe; distinct states may run on distinct streams.
 */
#ifndef FGA_H
#define FGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FGA_OK = 0,
  FGA_E_INVALID_ARG = 1, /* null pointer, bad size or out-of-range parameter */
  FGA_E_NOMEM = 2,       /* device allocation failed */
  FGA_E_DEVICE = 3,      /* HIP runtime or kernel error */
  FGA_E_NONFINITE = 4,   /* NaN or Inf in the input points or masses */
  FGA_E_DEGENERATE = 5,  /* zero-extent input, or a collinear template */
  FGA_E_UNSUPPORTED = 6  /* valid request the library does not implement */
} fga_status;

typedef enum { FGA_F32 = 0, FGA_F64 = 1 } fga_dtype;

/* Damping of Eq. (PreviousVelocity).
 * FRACTION: v' = (1 - eta) v + dt g, the friction removing the fraction eta of
 *           the particle momentum per step (Sec. n-Body Simulations).
 * LITERAL:  v' = v + dt (F - eta v) / m_Y, Eqs. GAForceDissipative-PreviousVelocity. */
typedef enum { FGA_DAMP_FRACTION = 0, FGA_DAMP_LITERAL = 1 } fga_damping;

/* Velocity carried between iterations.
 * RIGID:    the realised rigid displacement of the previous step over dt.
 * PARTICLE: the unconstrained per-particle velocity v' of Eq. PreviousVelocity. */
typedef enum { FGA_VEL_RIGID = 0, FGA_VEL_PARTICLE = 1 } fga_velocity;

/* Masses (Sec. Smooth-Particle Mass Function, Eq. FinalSPM with B = 1):
 * NIV normalised intrinsic volume, or UNIFORM (the constant-NIV case). */
typedef enum { FGA_MASS_NIV = 0, FGA_MASS_UNIFORM = 1 } fga_mass_mode;

/* Arithmetic of the force sum. The displacement moments, the rigid state and
 * the Kabsch step are FP64 in every mode except FP32_ALL.
 * FP32:       FP32 positions and forces, plain per-lane accumulation.
 * FP32_KAHAN: FP32 positions and forces, tile sums added with Kahan compensation
 *             (direct sum: tiles of 64 reference points; group walk: each
 *             flushed interaction list). The per-particle Barnes-Hut walk
 *             accumulates plainly in every FP32 mode.
 * FP64:       FP64 positions and forces (requires FGA_F64 data).
 * FP32_ALL:   like FP32, and the per-particle moments are also summed in FP32. */
typedef enum {
  FGA_PREC_FP32 = 0,
  FGA_PREC_FP32_KAHAN = 1,
  FGA_PREC_FP64 = 2,
  FGA_PREC_FP32_ALL = 3
} fga_precision;

typedef struct {
  double G, eps, eta, dt; /* 66.7, 0.2, 0.2, 0.1 (Sec. Baseline Methods and Parameter Settings) */
  double theta;           /* MAC opening parameter; 0 = direct all-pairs sum */
  double a, b;            /* normalisation range [a, b] = [-5, 5] (Appendix A) */
  int rho;                /* NIV lattice cells per axis, 16 */
  int max_depth;          /* octree depth limit, 20 (Sec. BH tree, step iii) */
  int max_iter;           /* iteration cap */
  double tol;             /* stop when ||T_k - T_{k-1}||_F^2 < tol on a shrinking step
                             (Alg. 2, threshold 1e-4 on the norm: tol = 1e-8);
                             tol <= 0 runs exactly max_iter iterations */
  int damping;            /* fga_damping */
  int velocity;           /* fga_velocity */
  int mass_mode;          /* fga_mass_mode */
  int precision;          /* fga_precision */
  int leaf_size;          /* BH leaf size L: cells with at most L points are not split.
                             1 = Alg. 1 exactly (singleton leaves); 2..64 sum more points
                             exactly (at least Alg. 1's accuracy) for fewer node visits;
                             0 = chosen by the autotuner among 1, 2, 4, 8 and 16 (FP32
                             Barnes-Hut; FP64 and fga_forces use 1) */
  int tile;               /* work split of one iteration, 0..255: reference ranges per template
                             tile of 256 particles, or for the group walk the most parts a
                             heavy group is split into (the largest power of two <= tile);
                             0 = autotuned per shape class and cached */
  int check_every;        /* host checks the convergence flag every k iterations (0 = 16) */
  int group_width;        /* BH traversal (FP32 only): 1 = per-particle, every particle makes
                             the Alg. 2 accept/open decisions itself; 64 or 128 = the
                             particles of a wave (consecutive in Morton order) share one walk,
                             a node being accepted only if the MAC holds for the group's whole
                             bounding box (at least as accurate as per-particle); 32 = groups
                             of at most 32 such particles, each held twice over the wave's
                             lanes (the two copies split the interaction list); 0 = chosen
                             by the autotuner among 1, 64 and 128 (and 32 for planar sets,
                             fga_register_2d). FP64 uses 1. The choice changes
                             which nodes are accepted, so with 0 the result of identical
                             inputs can differ (within the MAC's accuracy) between processes
                             whose timings made different choices; FGA_TUNE_CACHE pins them. */
  double rbf_sigma;       /* width sigma of the RBF kernel exp(-s^2 / sigma^2) of the landmark
                             masses (Eq. RBF_function), in the normalised frame; 0.03 */
  double rbf_weight;      /* value of the RBF weight B at a landmark point; away from every
                             landmark B returns to the landmark-free value 1; 100 */
  int reserved[4];        /* zero */
} fga_params;

typedef struct {
  int iters;              /* iterations performed */
  int converged;          /* 1 if the tolerance was met before max_iter */
  double last_dT2;        /* ||T_k - T_{k-1}||_F^2 of the last iteration (normalised frame) */
  long long interactions; /* force interactions evaluated (accepted nodes + leaf points) */
  double ms_total;        /* wall time of the call in milliseconds */
  int traversal;          /* force kernel in use: 0 = direct sum (theta = 0), 1 = per-particle
                             Barnes-Hut walk, 32, 64 or 128 = group walk of groups of at most
                             that many particles */
  int leaf_size;          /* leaf size of the Barnes-Hut tree in use (0 for the direct sum) */
} fga_report;

typedef struct fga_state fga_state;
typedef struct fga_tree fga_tree;

/* Fills *p with the paper's parameter settings (G = 66.7, eps = 0.2,
 * eta = 0.2, dt = 0.1, theta = 0.6, [a,b] = [-5,5], rho = 16, depth 20), 200
 * iterations, tol = 1e-8, fraction damping, rigid velocity, NIV masses,
 * FP32 with Kahan tiles, leaf size 1. */
fga_status fga_default_params(fga_params* p);

/* Message of the last non-OK status on this thread ("" if none). */
const char* fga_last_error(void);

/* Library version string. */
const char* fga_version(void);

/* Smooth-particle masses of one point set, Eq. (Normalized_IntrinsicVol)
 * with B = 1 (Eq. FinalSPM): the set's bounding box is split into p->rho
 * cells per axis; every point gets V_cell / min(n_c V_ball, V_cell) with
 * n_c the count of its cell and V_ball the volume of a ball of radius
 * (b - a) / (2 max_depth rho). norm = 0 scales the result to sum 1, norm = 1
 * to mean 1. pts: n x 3 device, masses_out: n device values of dtype dt. */
fga_status fga_masses(const void* pts, fga_dtype dt, int64_t n, const fga_params* p, int norm,
                      void* masses_out, void* stream);

/* Smooth-particle masses with landmark points, Eq. (FinalSPM) S = N o B: N as
 * in fga_masses, B the RBF interpolation of Eq. (RBF_function) over the
 * landmark points pts[landmarks[k]], B(p) = 1 + sum_k lambda_k exp(-|p - a_k|^2 /
 * sigma^2) with lambda from the collocation system B(a_k) = p->rbf_weight
 * (solved on the device). landmarks: host array of n_landmarks indices in
 * [0, n), at most 64; no landmarks gives fga_masses. Landmarks closer than the
 * RBF width make the system singular: FGA_E_DEGENERATE. Coordinates are those
 * of pts (no normalisation). */
fga_status fga_masses_landmarks(const void* pts, fga_dtype dt, int64_t n, const int64_t* landmarks,
                                int n_landmarks, const fga_params* p, int norm, void* masses_out,
                                void* stream);

/* Gravitational force on every template particle, Eq. (GAForce):
 *   F_i = -G sum_j mX_j mY_i (y_i - x_j) / (|y_i - x_j|^2 + eps^2)^(3/2).
 * theta == 0: exact all-pairs sum. theta > 0: Barnes-Hut (Alg. 1 tree built
 * on X here, Alg. 2 BHForce). Y: m x 3, X: n x 3, mX: n, mY: m or NULL (= 1),
 * F_out: m x 3, all device arrays of dtype dt. interactions (host, may be
 * NULL) receives the number of interactions evaluated. Uses p->G, p->eps,
 * p->precision, p->leaf_size. */
fga_status fga_forces(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                      const void* mY, fga_dtype dt, double theta, const fga_params* p,
                      void* F_out, long long* interactions, void* stream);

/* Size of the static device scratch of fga_forces_direct_noalloc (64 MiB per GPU). */
#define FGA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* fga_forces with theta = 0 (the exact all-pairs sum of Eq. GAForce) for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same kernels, with
 * their scratch (the packed reference and the per-range partial forces,
 * about 16 n + 12 m r bytes in FP32 for r reference ranges) in a fixed
 * FGA_NOALLOC_SCRATCH_BYTES device array that each GPU holds from the
 * library's first call there until the process ends. No allocation of any
 * kind and no synchronisation: the work is queued on `stream` and F_out is
 * ready when it completes; launch errors are reported, kernel faults surface
 * at the caller's next synchronisation. Sizes whose scratch exceeds the array
 * return FGA_E_INVALID_ARG before any device work. Every call on one GPU uses
 * that GPU's single array, so calls that overlap in time on one GPU (other
 * streams, other threads) race and must be ordered by the caller; calls on
 * one stream are ordered by it. Arguments as in fga_forces. */
fga_status fga_forces_direct_noalloc(const void* Y, int64_t m, const void* X, int64_t n,
                                     const void* mX, const void* mY, fga_dtype dt,
                                     const fga_params* p, void* F_out, void* stream);

/* Plummer energy of the template in the reference's field, the energy whose
 * negative gradient is Eq. (GAForce) (a convergence diagnostic; Eq.
 * GPE_Energy_GA prints |r| + eps where the force implies sqrt(|r|^2 + eps^2)):
 *   E = -G sum_i mY_i sum_j mX_j / sqrt(|y_i - x_j|^2 + eps^2).
 * theta == 0: exact double sum; theta > 0: the Alg. 2 traversal of the Alg. 1
 * tree built here on X, an accepted node contributing M / sqrt(r^2 + eps^2).
 * Arguments as in fga_forces; E (host) receives the FP64 total, summed in a
 * fixed order (terms in the data's precision, tiles and totals in FP64). */
fga_status fga_energy(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                      const void* mY, fga_dtype dt, double theta, const fga_params* p, double* E,
                      long long* interactions, void* stream);

/* D = 2 (Alg. 1's split with 2^D = 4 children per cell: the quadtree). Point
 * sets are n x 2 device arrays; they are embedded at z = 0, where the octree
 * build splits only the two planar axes (a quadtree with the planar box
 * diagonal), forces stay in the plane, the NIV lattice has rho^2 cells with
 * disc areas for the point balls, and the rigid step is the 2 x 2 Kabsch
 * rotation. fga_forces_2d: as fga_forces, F_out m x 2. fga_register_2d:
 * R row-major 2 x 2 and t (2), host, X ~= R Y + t. */
fga_status fga_forces_2d(const void* Y, int64_t m, const void* X, int64_t n, const void* mX,
                         const void* mY, fga_dtype dt, double theta, const fga_params* p,
                         void* F_out, long long* interactions, void* stream);
fga_status fga_register_2d(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                           const fga_params* p, double R[4], double t[2], fga_report* rep,
                           void* stream);

/* Registration state for Alg. 2: normalises (Appendix A), computes masses,
 * builds the BH tree once if p->theta > 0, and sets T = [I | 0]. The state
 * owns device copies; X and Y may be freed after the call returns. */
fga_status fga_state_create(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                            const fga_params* p, void* stream, fga_state** out);

/* fga_state_create with prior correspondences (Alg. 2's landmarks C):
 * X[lm_X[k]] <-> Y[lm_Y[k]], k < n_landmarks <= 64, host arrays. The masses
 * become S = N o B (Eq. FinalSPM) with B of Eq. (RBF_function) anchored at the
 * normalised landmark points of each cloud (the reference's at X[lm_X], the
 * template's at Y[lm_Y]); sigma = p->rbf_sigma in the normalised frame. */
fga_status fga_state_create_landmarks(const void* X, int64_t n, const void* Y, int64_t m,
                                      fga_dtype dt, const int64_t* lm_X, const int64_t* lm_Y,
                                      int n_landmarks, const fga_params* p, void* stream,
                                      fga_state** out);

/* Runs n_iters iterations of the Alg. 2 loop body (forces, damped velocity,
 * displacements, Kabsch step, template update) on the state's stream. Stops
 * early only if p->tol > 0 and the tolerance is met. */
fga_status fga_step(fga_state* st, int n_iters);

/* fga_step for exactly n_iters >= 1 iterations (no early stop) with HIP events
 * recorded on the state's stream around the two launches of every iteration:
 * ms[0] receives the summed duration of the force launches (template pose,
 * Eq. GAForce forces, the damped ODE step and the per-block displacement
 * moments), ms[1] that of the reduction launches (moment sum and the Kabsch
 * step of Eqs. R_Kabsch and transEst). A registration's first iteration that
 * measures the group walk's costs, if still pending, runs first, untimed.
 * ms is host memory. Synchronises the stream. */
fga_status fga_step_profile(fga_state* st, int n_iters, double ms[2]);

/* Current transform in the caller's coordinates (de-normalised as in
 * Appendix A) and an optional report. R, t, rep are host memory; rep may be NULL. */
fga_status fga_state_get(const fga_state* st, double R[9], double t[3], fga_report* rep);

/* Current transform in the normalised frame (Yn -> Xn), host memory. */
fga_status fga_state_get_normalised(const fga_state* st, double R[9], double t[3]);

/* Serialises the dynamic state (FP64 rigid state, per-particle velocities in
 * particle mode) into buf. Call with buf = NULL to query *len. */
fga_status fga_state_save(const fga_state* st, void* buf, size_t* len);

/* Restores a state saved from a state created with the same inputs and parameters. */
fga_status fga_state_load(fga_state* st, const void* buf, size_t len);

void fga_state_destroy(fga_state* st);

/* Whole Alg. 2 registration of Y to X: normalise, masses, tree (theta > 0),
 * iterate to convergence or max_iter, de-normalise. */
fga_status fga_register(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                        const fga_params* p, double R[9], double t[3], fga_report* rep,
                        void* stream);

/* fga_register with landmark correspondences (see fga_state_create_landmarks). */
fga_status fga_register_landmarks(const void* X, int64_t n, const void* Y, int64_t m, fga_dtype dt,
                                  const int64_t* lm_X, const int64_t* lm_Y, int n_landmarks,
                                  const fga_params* p, double R[9], double t[3], fga_report* rep,
                                  void* stream);

/* npairs independent registrations run together: one set of launches builds
 * every pair's tree, and every iteration is one persistent launch over a work
 * queue replayed from a HIP graph. With FP32 Barnes-Hut (and group_width != 1)
 * the queue holds blocks of the group walk (one particle per lane, groups
 * bounded by twice the median box, heavy groups split over several waves by
 * the cost one measuring iteration finds, heaviest first); otherwise (pair,
 * template tile, reference range) items of the per-particle walk or the direct
 * sum. Each pair stops by the Alg. 2 rule on its own. X[k], Y[k] are device
 * arrays of n[k] x 3 and m[k] x 3 points. R: npairs x 9, t: npairs x 3, reps:
 * npairs (may be NULL), host memory. */
fga_status fga_register_batch(int npairs, const void* const* X, const int64_t* n,
                              const void* const* Y, const int64_t* m, fga_dtype dt,
                              const fga_params* p, double* R, double* t, fga_report* reps,
                              void* stream);

/* Frame-to-frame registration of a sequence of scans (the LiDAR odometry
 * application): frame k+1 (template) is registered to frame k (reference) for
 * every k < nframes - 1, all pairs in one fga_register_batch call (every
 * frame's tree is built once, as the reference of its pair), and the relative
 * transforms are composed into the pose of every frame in frame 0's
 * coordinates: T_0 = [I | 0], T_{k+1} = T_k T_rel(k), in FP64 on the host.
 * frames[k]: device array of sizes[k] x 3 points. R_rel, t_rel: (nframes - 1)
 * x 9 and x 3 with frame_k ~= R_rel(k) frame_{k+1} + t_rel(k); R_abs, t_abs:
 * nframes x 9 and x 3 (both may be NULL); reps: nframes - 1 or NULL. All
 * results are host memory. */
fga_status fga_register_sequence(int nframes, const void* const* frames, const int64_t* sizes,
                                 fga_dtype dt, const fga_params* p, double* R_rel, double* t_rel,
                                 double* R_abs, double* t_abs, fga_report* reps, void* stream);

/* The library keeps the device buffers of finished calls in a cache and reuses
 * them (a registration needs a few dozen buffers; allocating and freeing them
 * each time costs more than a small registration). Returns every idle cached
 * buffer to the device; buffers still in use by queued work stay cached.
 * Thread-safe. */
fga_status fga_trim_cache(void);

/* ---- inspection entry points (used by tests and tools) ---- */

/* Builds the compressed octree of Alg. 1 on X (n x 3) with masses mX (n),
 * device arrays of dtype dt. Chains of single-child cells are collapsed to
 * their deepest cell, which gives the same accept/open outcome and force. */
fga_status fga_tree_create(const void* X, const void* mX, int64_t n, fga_dtype dt,
                           const fga_params* p, void* stream, fga_tree** out);

/* info[0] = nodes, info[1] = leaves, info[2] = internal nodes, info[3] = max depth. */
fga_status fga_tree_info(const fga_tree* tr, int64_t info[4]);

/* Copies the tree to host memory. Nodes are in depth-first preorder.
 *   com_mass: nodes x 4 (x, y, z, mass), float
 *   ints:     nodes x 4 (skip, first, last, depth), int32; skip is the preorder
 *             index after the node's subtree; [first, last] the node's points in
 *             sorted order; a leaf has skip == index + 1.
 *   order:    n, int32: order[k] = input index of the k-th sorted point.
 * Any pointer may be NULL. */
fga_status fga_tree_export(const fga_tree* tr, float* com_mass, int32_t* ints, int32_t* order);

void fga_tree_destroy(fga_tree* tr);

/* Group runs of the Barnes-Hut group walk for the points Y (m x 3, FP32, device
 * pointer), taken in the given order (the library cuts the template in its
 * body-frame Morton order): greedy runs of at most G (32, 64 or 128)
 * consecutive points, each ending before the diagonal of its bounding box
 * would exceed f times the median diagonal of the aligned runs of G points
 * (f = 0: runs of exactly G). runs_out (host, 2 x cap int32) receives
 * (first, count) per run and *n_runs their number; FGA_E_INVALID_ARG when
 * there are more than cap runs (*n_runs is set either way). */
fga_status fga_group_runs(const void* Y, int64_t m, int G, double f, int32_t* runs_out, int64_t cap,
                          int64_t* n_runs, void* stream);

/* Host evaluation of the FP64 Kabsch solution used on the device: given
 * C = hat(Y_D)^T hat(Y) (row-major 3x3), writes R = U diag(1,1,sgn det(U V^T)) V^T
 * (Eq. R_Kabsch). Returns FGA_E_DEGENERATE when rank(C) < 2. */
fga_status fga_kabsch(const double C[9], double R[9]);

#ifdef __cplusplus
}
#endif
#endif /* FGA_H */
