// FP64 rigid step of the FGA loop body: Kabsch rotation (Eq. R_Kabsch),
// translation (Eq. transEst) and the template update / composition of Alg. 2.
// Compiled for both host and device: the device runs it once per iteration in
// the last block of the reduction launch; the host entry fga_kabsch exposes
// the same solver for tests.
#pragma once
#include <math.h>

#include "common.h"

namespace fga {

#define FGA_HD __host__ __device__ inline

FGA_HD void m3_mul(const double* A, const double* B, double* C) {  // C = A B
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
FGA_HD void m3_mul_bt(const double* A, const double* B, double* C) {  // C = A B^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
}
FGA_HD double m3_det(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// One Jacobi rotation of columns P < Q of W (and of V alongside) that makes
// them orthogonal; false if they already are, to 1e-15 relative (cosine of
// their angle, compared squared). The column dot product carries rounding of
// a few ulps (2.2e-16 each), so a tighter threshold is usually never met and
// the sweeps run to their cap; at 1e-15 a cold solve ends after 3 to 5
// sweeps. P and Q are compile-time so that W and V stay in registers.
template <int P, int Q>
FGA_HD bool jacobi_rotate(double* W, double* V) {
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = 0; i < 3; ++i) {
    al += W[3 * i + P] * W[3 * i + P];
    be += W[3 * i + Q] * W[3 * i + Q];
    ga += W[3 * i + P] * W[3 * i + Q];
  }
  if (ga * ga <= 1e-30 * (al * be)) return false;
  const double ze = (be - al) / (2.0 * ga);
  const double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
  const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
  for (int i = 0; i < 3; ++i) {
    const double wp = W[3 * i + P], wq = W[3 * i + Q];
    W[3 * i + P] = c * wp - sn * wq;
    W[3 * i + Q] = sn * wp + c * wq;
    const double vp = V[3 * i + P], vq = V[3 * i + Q];
    V[3 * i + P] = c * vp - sn * vq;
    V[3 * i + Q] = sn * vp + c * vq;
  }
  return true;
}

// Swaps columns P and Q of W and V and entries P and Q of nrm.
template <int P, int Q>
FGA_HD void swap_columns(double* W, double* V, double* nrm) {
  for (int i = 0; i < 3; ++i) {
    double t = W[3 * i + P];
    W[3 * i + P] = W[3 * i + Q];
    W[3 * i + Q] = t;
    t = V[3 * i + P];
    V[3 * i + P] = V[3 * i + Q];
    V[3 * i + Q] = t;
  }
  const double t = nrm[P];
  nrm[P] = nrm[Q];
  nrm[Q] = t;
}

// One-sided (Hestenes) Jacobi SVD of a 3x3 matrix: A = U diag(s) V^T with
// s sorted in descending order. Columns of W = A V are rotated pairwise, in
// the order (0,1), (0,2), (1,2), until they are mutually orthogonal; then
// s_k = |W_k| and U_k = W_k / s_k. Columns belonging to zero singular values
// are left as zero in U. Every array index is a compile-time constant, so the
// device keeps the whole solve in registers. V0 (orthogonal, or NULL for the
// identity) is the starting V: W = A V0. The right singular vectors of a
// matrix close to A make W nearly orthogonal from the start, so fewer sweeps
// are needed; the factors are the same up to rounding and column signs.
FGA_HD void svd3(const double* A, double* U, double* s, double* V, const double* V0 = nullptr) {
  double W[9];
  if (V0) {
    for (int k = 0; k < 9; ++k) V[k] = V0[k];
    m3_mul(A, V0, W);
  } else {
    for (int k = 0; k < 9; ++k) W[k] = A[k];
    for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
  }
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = jacobi_rotate<0, 1>(W, V);
    rotated = jacobi_rotate<0, 2>(W, V) || rotated;
    rotated = jacobi_rotate<1, 2>(W, V) || rotated;
    if (!rotated) break;
  }
  double nrm[3];
  for (int k = 0; k < 3; ++k)
    nrm[k] = sqrt(W[k] * W[k] + W[3 + k] * W[3 + k] + W[6 + k] * W[6 + k]);
  // sort columns by singular value, descending (three compare-swaps; equal
  // values keep their order)
  if (nrm[0] < nrm[1]) swap_columns<0, 1>(W, V, nrm);
  if (nrm[1] < nrm[2]) swap_columns<1, 2>(W, V, nrm);
  if (nrm[0] < nrm[1]) swap_columns<0, 1>(W, V, nrm);
  for (int k = 0; k < 3; ++k) {
    s[k] = nrm[k];
    const double inv = nrm[k] > 0.0 ? 1.0 / nrm[k] : 0.0;
    for (int i = 0; i < 3; ++i) U[3 * i + k] = W[3 * i + k] * inv;
  }
}

// Eq. (R_Kabsch): C = U S V^T, R = U diag(1, 1, sgn det(U V^T)) V^T, sgn(0) = +1.
// For rank(C) = 2 the third left singular vector is completed as U_0 x U_1.
// Returns 0, or 1 when rank(C) < 2 (collinear template: R is then undefined
// and set to the identity). A singular value below rank_tol * s_0 counts as
// zero; rank_tol reflects the precision the template is stored in. Vw, if
// given, starts the SVD (see svd3) and receives its V.
FGA_HD int kabsch3(const double* C, double* R, double rank_tol = 1e-13, double* Vw = nullptr) {
  double U[9], s[3], V[9];
  svd3(C, U, s, V, Vw);
  if (Vw)
    for (int k = 0; k < 9; ++k) Vw[k] = V[k];
  const double tiny = rank_tol * s[0];
  if (!(s[0] > 0.0) || s[1] <= tiny) {
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    return 1;
  }
  if (s[2] <= tiny) {  // rank 2: complete U with the cross product of its first two columns
    U[2] = U[3] * U[7] - U[6] * U[4];
    U[5] = U[6] * U[1] - U[0] * U[7];
    U[8] = U[0] * U[4] - U[3] * U[1];
  }
  const double d = m3_det(U) * m3_det(V) < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = U[3 * i] * V[3 * j] + U[3 * i + 1] * V[3 * j + 1] + d * U[3 * i + 2] * V[3 * j + 2];
  return 0;
}

// Eq. (R_Kabsch) in D = 2 for a planar C (its third row and column zero):
// the rotation about z that maximises tr(R^T C), angle atan2(C10 - C01, C00 + C11).
// Returns 1 (R = I) when both terms vanish (no rotation is determined).
FGA_HD int kabsch2(const double* C, double* R, double rank_tol) {
  const double sn = C[3] - C[1], cs = C[0] + C[4];
  const double h = sqrt(sn * sn + cs * cs);
  const double scale = fabs(C[0]) + fabs(C[1]) + fabs(C[3]) + fabs(C[4]);
  for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
  if (!(h > rank_tol * scale)) return 1;
  R[0] = cs / h;
  R[1] = -sn / h;
  R[3] = sn / h;
  R[4] = cs / h;
  return 0;
}

// One Alg. 2 rigid step from the reduced displacement moments.
//   mom[0..2]  = sum_i d_i
//   mom[3..11] = P = sum_i d_i q_i^T (row-major, P[a][b] = sum d_a q_b)
// With hat(y_i) = R q_i (the centred template) the Kabsch matrix is
//   C = hat(Y_D)^T hat(Y) = sum (hat y_i + d_i - dbar) hat y_i^T = (R S0 + P) R^T,
// because sum_i hat y_i = 0. Then R_s from Eq. (R_Kabsch), mu_D = mu + dbar,
// t_s = mu_D - R_s mu (Eq. transEst), R <- R_s R, t <- R_s t + t_s, mu <- mu_D.
// The rigid velocity of the next step is (y_new - y)/dt = A q + b.
FGA_HD void rigid_update(RigidState& s, const double* mom, double dt) {
  const double invm = 1.0 / (double)s.m;
  const double dbar[3] = {mom[0] * invm, mom[1] * invm, mom[2] * invm};
  double RS0[9], C[9], Rs[9];
  m3_mul(s.R, s.S0, RS0);
  for (int k = 0; k < 9; ++k) RS0[k] += mom[3 + k];
  m3_mul_bt(RS0, s.R, C);
  if (s.dims == 2 ? kabsch2(C, Rs, s.rank_tol) : kabsch3(C, Rs, s.rank_tol, s.Vw)) s.flags |= 1;
  double muD[3], ts[3], Rn[9], tn[3];
  for (int a = 0; a < 3; ++a) muD[a] = s.mu[a] + dbar[a];
  for (int a = 0; a < 3; ++a)
    ts[a] = muD[a] - (Rs[3 * a] * s.mu[0] + Rs[3 * a + 1] * s.mu[1] + Rs[3 * a + 2] * s.mu[2]);
  m3_mul(Rs, s.R, Rn);
  for (int a = 0; a < 3; ++a)
    tn[a] = Rs[3 * a] * s.t[0] + Rs[3 * a + 1] * s.t[1] + Rs[3 * a + 2] * s.t[2] + ts[a];
  // keep R orthonormal: one Newton-Schulz step R <- R (3 I - R^T R) / 2
  {
    double RtR[9], Kc[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        RtR[3 * i + j] = Rn[i] * Rn[j] + Rn[3 + i] * Rn[3 + j] + Rn[6 + i] * Rn[6 + j];
    for (int k = 0; k < 9; ++k) Kc[k] = ((k % 4 == 0) ? 1.5 : 0.0) - 0.5 * RtR[k];
    double Ro[9];
    m3_mul(Rn, Kc, Ro);
    for (int k = 0; k < 9; ++k) Rn[k] = Ro[k];
  }
  double dT2 = 0.0;
  for (int k = 0; k < 9; ++k) dT2 += (Rn[k] - s.R[k]) * (Rn[k] - s.R[k]);
  for (int a = 0; a < 3; ++a) dT2 += (tn[a] - s.t[a]) * (tn[a] - s.t[a]);
  const double invdt = 1.0 / dt;
  for (int k = 0; k < 9; ++k) s.A[k] = (Rn[k] - s.R[k]) * invdt;
  for (int a = 0; a < 3; ++a) s.b[a] = (muD[a] - s.mu[a]) * invdt;
  for (int k = 0; k < 9; ++k) s.R[k] = Rn[k];
  for (int a = 0; a < 3; ++a) {
    s.t[a] = tn[a];
    s.mu[a] = muD[a];
  }
  // stop rule of Alg. 2: the step fell below tol while shrinking (the motion
  // starts from rest, so the first, accelerating steps are small as well)
  if (s.tol > 0.0 && dT2 < s.tol && s.iter > 0 && dT2 < s.dT2) s.converged = 1;
  s.dT2 = dT2;
  s.iter += 1;
  if (s.iter >= s.max_iter) s.converged = s.converged ? 1 : 2;  // 2 = stopped at the cap
  for (int k = 0; k < 9; ++k) {
    s.fR[k] = (float)s.R[k];
    s.fA[k] = (float)s.A[k];
  }
  for (int a = 0; a < 3; ++a) {
    s.fmu[a] = (float)s.mu[a];
    s.fb[a] = (float)s.b[a];
  }
}

// Initial state: T = [I | 0] (Alg. 2 initialisation), zero velocity.
FGA_HD void rigid_init(RigidState& s, const double* S0, const double* mu0, int m, double tol,
                       int max_iter, double rank_tol, int dims = 3) {
  for (int k = 0; k < 9; ++k) {
    s.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    s.A[k] = 0.0;
    s.S0[k] = S0[k];
    s.Vw[k] = (k % 4 == 0) ? 1.0 : 0.0;
    s.fR[k] = (float)s.R[k];
    s.fA[k] = 0.0f;
  }
  for (int a = 0; a < 3; ++a) {
    s.t[a] = 0.0;
    s.mu[a] = mu0[a];
    s.mu0[a] = mu0[a];
    s.b[a] = 0.0;
    s.fmu[a] = (float)mu0[a];
    s.fb[a] = 0.0f;
  }
  s.dT2 = 0.0;
  s.tol = tol;
  s.rank_tol = rank_tol;
  s.interactions = 0;
  s.iter = 0;
  s.converged = 0;
  s.m = m;
  s.flags = 0;
  s.max_iter = max_iter;
  s.dims = dims;
}

}  // namespace fga
