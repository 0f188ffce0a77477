/*
 * FP64 CPU oracle for the Fast Gravitational Approach (FGA) force evaluation.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * HIP path is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table
 * or helper with the GPU library.
 *
 * Contents (paper: "Fast Gravitational Approach for Rigid Point Set
 * Registration with Ordinary Differential Equations", arXiv 2009.14005):
 *   - oracle_direct_forces : Eq. (GAForce), the all-pairs gravitational force
 *                            on each template particle, written out as the
 *                            plain double loop.
 *   - oracle_bh_build      : Alg. 1 (Build BH tree), recursive 2^D split of
 *                            the reference bounding box, uncompressed.
 *   - oracle_bh_build_leaf : the same split stopped at cells of at most L
 *                            points (L = 1 is Alg. 1 itself), the leaf-size
 *                            variant of the tree that the GPU path can build.
 *   - oracle_bh_forces     : Alg. 2, function BHForce, recursive descent with
 *                            the multipole acceptance criterion Eq. (MAC).
 *   - oracle_gpe           : Plummer potential energy, a diagnostic whose
 *                            negative gradient is Eq. (GAForce).
 *   - oracle_direct_forces_2d, oracle_bh_build_dims : the same in D = 2 (the
 *                            quadtree of Alg. 1's general 2^D split).
 *   - oracle_bh_gpe        : the Plummer energy with the BHForce traversal
 *                            (accepted nodes contribute M / sqrt(r^2 + eps^2)).
 *
 * Readings of the paper used here (all listed in the design notes):
 *   - Cell membership: per-axis integer quantisation of the tight bounding
 *     box, q = min(floor(2^20 (p - lo) / (hi - lo)), 2^20 - 1); a zero-extent
 *     axis gives q = 0. At depth k a point goes to the upper half of an axis
 *     when bit (19 - k) of q is set. This is the midpoint split of Alg. 1 with
 *     points on a split plane assigned to the upper child.
 *   - Depth limit: cells are split while they hold at least two points and
 *     their depth is below 20; a depth-20 cell is a leaf that keeps all its
 *     points (Alg. 1 literally gives such cells no mass).
 *   - Node length l is the diagonal of the node's box (Alg. 1).
 *   - BHForce: a node is accepted when l / r < theta with r the distance from
 *     the query to the node's centre of mass (Eq. MAC); r = 0 therefore never
 *     accepts. A leaf that is not accepted contributes the exact Eq. (GAForce)
 *     sum over its points; an internal node that is not accepted recurses into
 *     its non-empty children and the results are simply added.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC fga_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QBITS 20          /* maximum tree depth d = 20 (Sec. BH tree, step iii) */

/* ------------------------------------------------------------------ forces */

/* Eq. (GAForce): F_i = -G sum_j mX_j mY_i (y_i - x_j) / (|y_i - x_j|^2 + eps^2)^(3/2).
 * Y: m x 3, X: n x 3, row-major. mY may be NULL (all ones). F: m x 3 out. */
void oracle_direct_forces(const double* Y, long m, const double* X, long n,
                          const double* mX, const double* mY, double G, double eps,
                          double* F) {
  const double eps2 = eps * eps;
  long i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < m; ++i) {
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (long j = 0; j < n; ++j) {
      double dx = Y[3 * i + 0] - X[3 * j + 0];
      double dy = Y[3 * i + 1] - X[3 * j + 1];
      double dz = Y[3 * i + 2] - X[3 * j + 2];
      double r2 = dx * dx + dy * dy + dz * dz + eps2;
      double w = mX[j] / (r2 * sqrt(r2));
      fx += w * dx;
      fy += w * dy;
      fz += w * dz;
    }
    double my = mY ? mY[i] : 1.0;
    F[3 * i + 0] = -G * my * fx;
    F[3 * i + 1] = -G * my * fy;
    F[3 * i + 2] = -G * my * fz;
  }
}

/* Eq. (GAForce) in D = 2: Y m x 2, X n x 2, F m x 2. */
void oracle_direct_forces_2d(const double* Y, long m, const double* X, long n,
                             const double* mX, const double* mY, double G, double eps,
                             double* F) {
  const double eps2 = eps * eps;
  long i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < m; ++i) {
    double fx = 0.0, fy = 0.0;
    for (long j = 0; j < n; ++j) {
      double dx = Y[2 * i + 0] - X[2 * j + 0];
      double dy = Y[2 * i + 1] - X[2 * j + 1];
      double r2 = dx * dx + dy * dy + eps2;
      double w = mX[j] / (r2 * sqrt(r2));
      fx += w * dx;
      fy += w * dy;
    }
    double my = mY ? mY[i] : 1.0;
    F[2 * i + 0] = -G * my * fx;
    F[2 * i + 1] = -G * my * fy;
  }
}

/* Plummer potential E = -G sum_i sum_j mY_i mX_j / sqrt(|y_i - x_j|^2 + eps^2).
 * Its negative gradient with respect to y_i is Eq. (GAForce). Diagnostic only. */
double oracle_gpe(const double* Y, long m, const double* X, long n, const double* mX,
                  const double* mY, double G, double eps) {
  double e = 0.0;
  long i;
#pragma omp parallel for reduction(+ : e) schedule(static)
  for (i = 0; i < m; ++i) {
    double s = 0.0;
    for (long j = 0; j < n; ++j) {
      double dx = Y[3 * i + 0] - X[3 * j + 0];
      double dy = Y[3 * i + 1] - X[3 * j + 1];
      double dz = Y[3 * i + 2] - X[3 * j + 2];
      s += mX[j] / sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
    }
    e += (mY ? mY[i] : 1.0) * s;
  }
  return -G * e;
}

/* ------------------------------------------------------------ Alg. 1 tree */

typedef struct onode {
  int depth;
  long npts;             /* number of reference points inside the cell */
  long* pts;             /* their indices (owned by the tree's index pool) */
  double l;              /* diagonal of the cell's box */
  double mass;           /* sum of the point masses */
  double com[3];         /* centre of mass (first D entries) */
  struct onode* child[8];/* NULL = empty child cell */
  int nchild;            /* number of non-empty children (0 for a leaf) */
} onode;

typedef struct otree {
  onode* root;
  long n;
  const double* X;       /* borrowed; caller keeps X and mX alive */
  const double* mX;
  unsigned* q;           /* n x 3 quantised coordinates */
  double lo[3], hi[3];
  long n_nodes, n_leaves, n_internal, n_branching, max_depth;
  long leaf;             /* cells with at most this many points are leaves (Alg. 1: 1) */
  int dims;              /* D = 3 (octree) or 2 (quadtree); points are n x D */
  long* pool;            /* index storage: one slice per depth level */
} otree;

static onode* new_node(int depth, long* pts, long npts) {
  onode* nd = (onode*)calloc(1, sizeof(onode));
  nd->depth = depth;
  nd->pts = pts;
  nd->npts = npts;
  return nd;
}

/* CreateChild of Alg. 1 for a cell holding npts >= 1 points. */
static void create_child(otree* t, onode* nd, const double diag_root) {
  /* Node length: the box diagonal. A cell at depth k has every side halved k
   * times, so its diagonal is the root diagonal times 2^-k. */
  nd->l = ldexp(diag_root, -nd->depth);
  /* mass and centre of mass of the points inside the cell */
  const int D = t->dims;
  double m = 0.0, c[3] = {0.0, 0.0, 0.0};
  for (long k = 0; k < nd->npts; ++k) {
    long j = nd->pts[k];
    double w = t->mX[j];
    m += w;
    for (int a = 0; a < D; ++a) c[a] += w * t->X[D * j + a];
  }
  nd->mass = m;
  for (int a = 0; a < D; ++a) nd->com[a] = c[a] / m;
  t->n_nodes++;
  if (nd->depth > t->max_depth) t->max_depth = nd->depth;
  /* Alg. 1 splits a cell while it holds more than one point; the leaf-size
   * variant stops at cells of at most `leaf` points. Depth-20 cells are leaves. */
  if (nd->npts <= t->leaf || nd->depth >= QBITS) {
    t->n_leaves++;
    return;
  }
  t->n_internal++;
  /* split at the midpoint: bucket the points by the next quantisation bit of
   * each of the D axes (2^D children) */
  const int bit = QBITS - 1 - nd->depth;
  const int nch = 1 << D;
  long cnt[8] = {0};
  for (long k = 0; k < nd->npts; ++k) {
    long j = nd->pts[k];
    int o = 0;
    for (int a = 0; a < D; ++a) o = o << 1 | (int)((t->q[D * j + a] >> bit) & 1u);
    cnt[o]++;
  }
  long start[8];
  long acc = 0;
  for (int o = 0; o < nch; ++o) {
    start[o] = acc;
    acc += cnt[o];
  }
  /* stable partition into the child order, in a scratch copy */
  long* tmp = (long*)malloc(sizeof(long) * nd->npts);
  long pos[8];
  memcpy(pos, start, sizeof pos);
  for (long k = 0; k < nd->npts; ++k) {
    long j = nd->pts[k];
    int o = 0;
    for (int a = 0; a < D; ++a) o = o << 1 | (int)((t->q[D * j + a] >> bit) & 1u);
    tmp[pos[o]++] = j;
  }
  memcpy(nd->pts, tmp, sizeof(long) * nd->npts);
  free(tmp);
  int nonempty = 0;
  for (int o = 0; o < nch; ++o) {
    if (cnt[o] == 0) continue;  /* empty cell: CreateChild does nothing */
    onode* c = new_node(nd->depth + 1, nd->pts + start[o], cnt[o]);
    nd->child[o] = c;
    nonempty++;
    create_child(t, c, diag_root);
  }
  nd->nchild = nonempty;
  if (nonempty >= 2) t->n_branching++;
}

/* Alg. 1 with leaves of at most `leaf` points (leaf = 1: Alg. 1 itself) on
 * the reference X (n x 3) with masses mX. Returns an opaque handle, or NULL
 * for n < 1 or leaf < 1. */
void* oracle_bh_build_dims(const double* X, const double* mX, long n, long leaf, int dims) {
  if (n < 1 || leaf < 1 || (dims != 2 && dims != 3)) return NULL;
  const int D = dims;
  otree* t = (otree*)calloc(1, sizeof(otree));
  t->n = n;
  t->leaf = leaf;
  t->dims = D;
  t->X = X;
  t->mX = mX;
  for (int a = 0; a < D; ++a) {
    t->lo[a] = X[a];
    t->hi[a] = X[a];
  }
  for (long j = 1; j < n; ++j)
    for (int a = 0; a < D; ++a) {
      if (X[D * j + a] < t->lo[a]) t->lo[a] = X[D * j + a];
      if (X[D * j + a] > t->hi[a]) t->hi[a] = X[D * j + a];
    }
  t->q = (unsigned*)malloc(sizeof(unsigned) * D * n);
  const double cells = ldexp(1.0, QBITS);
  for (long j = 0; j < n; ++j)
    for (int a = 0; a < D; ++a) {
      double ext = t->hi[a] - t->lo[a];
      unsigned q = 0;
      if (ext > 0.0) {
        double f = floor((X[D * j + a] - t->lo[a]) / ext * cells);
        q = f >= cells - 1.0 ? (1u << QBITS) - 1u : (unsigned)f;
      }
      t->q[D * j + a] = q;
    }
  t->pool = (long*)malloc(sizeof(long) * n);
  for (long j = 0; j < n; ++j) t->pool[j] = j;
  double d2 = 0.0;
  for (int a = 0; a < t->dims; ++a) d2 += (t->hi[a] - t->lo[a]) * (t->hi[a] - t->lo[a]);
  t->root = new_node(0, t->pool, n);
  create_child(t, t->root, sqrt(d2));
  return t;
}

/* Alg. 1 in D = 3 with leaves of at most `leaf` points. */
void* oracle_bh_build_leaf(const double* X, const double* mX, long n, long leaf) {
  return oracle_bh_build_dims(X, mX, n, leaf, 3);
}

/* Alg. 1: build the BH tree on the reference X (n x 3) with masses mX. */
void* oracle_bh_build(const double* X, const double* mX, long n) {
  return oracle_bh_build_leaf(X, mX, n, 1);
}

static void free_node(onode* nd) {
  if (!nd) return;
  for (int o = 0; o < 8; ++o) free_node(nd->child[o]);
  free(nd);
}

void oracle_bh_free(void* h) {
  otree* t = (otree*)h;
  if (!t) return;
  free_node(t->root);
  free(t->q);
  free(t->pool);
  free(t);
}

/* Tree statistics: [nodes, leaves, internal, branching internal, max depth]. */
void oracle_bh_stats(const void* h, long* out5) {
  const otree* t = (const otree*)h;
  out5[0] = t->n_nodes;
  out5[1] = t->n_leaves;
  out5[2] = t->n_internal;
  out5[3] = t->n_branching;
  out5[4] = t->max_depth;
}

/* Root mass and centre of mass: out4 = [mass, cx, cy, cz]. */
void oracle_bh_root(const void* h, double* out4) {
  const otree* t = (const otree*)h;
  out4[0] = t->root->mass;
  for (int a = 0; a < 3; ++a) out4[1 + a] = a < t->dims ? t->root->com[a] : 0.0;
}

/* Leaf membership: leaf_id[j] = index of the leaf holding reference point j,
 * leaves numbered in depth-first child order. Returns the number of leaves. */
static void label_leaves(const onode* nd, long* leaf_id, long* next) {
  if (nd->nchild == 0) {
    for (long k = 0; k < nd->npts; ++k) leaf_id[nd->pts[k]] = *next;
    (*next)++;
    return;
  }
  for (int o = 0; o < 8; ++o)
    if (nd->child[o]) label_leaves(nd->child[o], leaf_id, next);
}

long oracle_bh_leaves(const void* h, long* leaf_id) {
  const otree* t = (const otree*)h;
  long next = 0;
  label_leaves(t->root, leaf_id, &next);
  return next;
}

/* Quantised coordinates (n x D) used for cell membership. */
void oracle_bh_quant(const void* h, unsigned* q_out) {
  const otree* t = (const otree*)h;
  memcpy(q_out, t->q, sizeof(unsigned) * t->dims * t->n);
}

/* ----------------------------------------------------------- Alg. 2 BHForce */

typedef struct bh_ctx {
  const otree* t;
  double theta, eps2;
} bh_ctx;

/* Adds sum_j m_j (x_j - y) / (|y - x_j|^2 + eps^2)^(3/2) of node nd to acc
 * (the force per unit template mass and per unit G). cnt counts interactions:
 * one per accepted node and one per leaf point summed exactly. */
static void bh_force(const bh_ctx* c, const onode* nd, const double* y, double acc[3],
                     long* cnt) {
  if (nd == NULL || nd->npts == 0) return;  /* empty node: no contribution */
  const int D = c->t->dims;
  double d[3] = {0.0, 0.0, 0.0};
  double rr = 0.0;
  for (int a = 0; a < D; ++a) {
    d[a] = y[a] - nd->com[a];
    rr += d[a] * d[a];
  }
  const double r = sqrt(rr);
  if (nd->l / r < c->theta) {  /* Eq. (MAC): far enough, use the node's CoM */
    double r2 = r * r + c->eps2;
    double w = nd->mass / (r2 * sqrt(r2));
    for (int a = 0; a < D; ++a) acc[a] -= w * d[a];
    (*cnt)++;
    return;
  }
  if (nd->nchild == 0) {  /* leaf that is not accepted: exact sum over its points */
    for (long k = 0; k < nd->npts; ++k) {
      long j = nd->pts[k];
      double e[3] = {0.0, 0.0, 0.0};
      double r2 = 0.0;
      for (int a = 0; a < D; ++a) {
        e[a] = y[a] - c->t->X[D * j + a];
        r2 += e[a] * e[a];
      }
      r2 += c->eps2;
      double w = c->t->mX[j] / (r2 * sqrt(r2));
      for (int a = 0; a < D; ++a) acc[a] -= w * e[a];
      (*cnt)++;
    }
    return;
  }
  for (int o = 0; o < 8; ++o) bh_force(c, nd->child[o], y, acc, cnt);
}

/* Plummer energy of one template particle through the same traversal: an
 * accepted node contributes mass / sqrt(r^2 + eps^2), a leaf that is not
 * accepted the exact sum over its points. Returns the sum (per unit G and
 * template mass, sign not applied). */
static double bh_pot(const bh_ctx* c, const onode* nd, const double* y, long* cnt) {
  if (nd == NULL || nd->npts == 0) return 0.0;
  const int D = c->t->dims;
  double rr = 0.0;
  for (int a = 0; a < D; ++a) rr += (y[a] - nd->com[a]) * (y[a] - nd->com[a]);
  const double r = sqrt(rr);
  if (nd->l / r < c->theta) {
    (*cnt)++;
    return nd->mass / sqrt(rr + c->eps2);
  }
  double s = 0.0;
  if (nd->nchild == 0) {
    for (long k = 0; k < nd->npts; ++k) {
      long j = nd->pts[k];
      double r2 = 0.0;
      for (int a = 0; a < D; ++a) r2 += (y[a] - c->t->X[D * j + a]) * (y[a] - c->t->X[D * j + a]);
      s += c->t->mX[j] / sqrt(r2 + c->eps2);
      (*cnt)++;
    }
    return s;
  }
  for (int o = 0; o < 8; ++o) s += bh_pot(c, nd->child[o], y, cnt);
  return s;
}

/* Alg. 2: for every template particle, F_k = G mY_k * BHForce(root, Y_k).
 * Y: m x 3. mY may be NULL (ones). F: m x 3 out. interactions: total count
 * (may be NULL). */
void oracle_bh_forces(const void* h, const double* Y, long m, const double* mY, double G,
                      double eps, double theta, double* F, long* interactions) {
  const otree* t = (const otree*)h;
  bh_ctx c = {t, theta, eps * eps};
  long total = 0;
  long i;
  const int D = t->dims;
#pragma omp parallel for reduction(+ : total) schedule(dynamic, 64)
  for (i = 0; i < m; ++i) {
    double acc[3] = {0.0, 0.0, 0.0};
    long cnt = 0;
    bh_force(&c, t->root, Y + D * i, acc, &cnt);
    double s = G * (mY ? mY[i] : 1.0);
    for (int a = 0; a < D; ++a) F[D * i + a] = s * acc[a];
    total += cnt;
  }
  if (interactions) *interactions = total;
}

/* Plummer energy E = -G sum_i mY_i (BH potential at y_i) with the Alg. 2
 * traversal; Y m x D. interactions (may be NULL) as in oracle_bh_forces. */
double oracle_bh_gpe(const void* h, const double* Y, long m, const double* mY, double G,
                     double eps, double theta, long* interactions) {
  const otree* t = (const otree*)h;
  bh_ctx c = {t, theta, eps * eps};
  long total = 0;
  double e = 0.0;
  long i;
  const int D = t->dims;
#pragma omp parallel for reduction(+ : total, e) schedule(dynamic, 64)
  for (i = 0; i < m; ++i) {
    long cnt = 0;
    e += (mY ? mY[i] : 1.0) * bh_pot(&c, t->root, Y + D * i, &cnt);
    total += cnt;
  }
  if (interactions) *interactions = total;
  return -G * e;
}
