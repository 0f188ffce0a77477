/* Exercises the FP64 oracle's C part (tree builds in D = 2 and 3 with several
 * leaf sizes, Barnes-Hut forces and energies, direct sums) on seeded random
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer.
 * Exits 0 when every result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_direct_forces(const double*, long, const double*, long, const double*, const double*,
                          double, double, double*);
void oracle_direct_forces_2d(const double*, long, const double*, long, const double*,
                             const double*, double, double, double*);
double oracle_gpe(const double*, long, const double*, long, const double*, const double*, double,
                  double);
void* oracle_bh_build_dims(const double*, const double*, long, long, int);
void oracle_bh_free(void*);
void oracle_bh_forces(const void*, const double*, long, const double*, double, double, double,
                      double*, long*);
double oracle_bh_gpe(const void*, const double*, long, const double*, double, double, double, long*);
long oracle_bh_leaves(const void*, long*);
void oracle_bh_stats(const void*, long*);

static unsigned long long rs = 88172645463325252ull;
static double urand(void) {
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return (double)(rs >> 11) / 9007199254740992.0;
}

int main(void) {
  const long n = 700, m = 300;
  double* X = malloc(sizeof(double) * 3 * (n + 4));
  double* Y = malloc(sizeof(double) * 3 * m);
  double* mX = malloc(sizeof(double) * (n + 4));
  double* F = malloc(sizeof(double) * 3 * m);
  long* ids = malloc(sizeof(long) * (n + 4));
  for (long i = 0; i < 3 * n; ++i) X[i] = urand();
  for (long i = 0; i < 3 * 4; ++i) X[3 * n + i] = X[i];  /* duplicates: depth-20 leaves */
  for (long i = 0; i < 3 * m; ++i) Y[i] = urand() * 1.5 - 0.25;
  for (long i = 0; i < n + 4; ++i) mX[i] = 0.5 + urand();
  int bad = 0;
  for (int D = 2; D <= 3; ++D)
    for (long leaf = 1; leaf <= 16; leaf *= 4) {
      void* t = oracle_bh_build_dims(X, mX, n + 4, leaf, D);
      long st[5], cnt = 0;
      oracle_bh_stats(t, st);
      if (oracle_bh_leaves(t, ids) < 1) bad = 1;
      for (int k = 0; k < 3; ++k) {
        const double th = k == 0 ? 0.0 : (k == 1 ? 0.5 : 1e9);
        oracle_bh_forces(t, Y, m, NULL, 66.7, 0.2, th, F, &cnt);
        for (long i = 0; i < D * m; ++i) bad |= !isfinite(F[i]);
        bad |= !isfinite(oracle_bh_gpe(t, Y, m, NULL, 66.7, 0.2, th, &cnt));
      }
      oracle_bh_free(t);
    }
  oracle_direct_forces(Y, m, X, n, mX, NULL, 66.7, 0.2, F);
  for (long i = 0; i < 3 * m; ++i) bad |= !isfinite(F[i]);
  oracle_direct_forces_2d(Y, m, X, n, mX, NULL, 66.7, 0.2, F);
  bad |= !isfinite(oracle_gpe(Y, m, X, n, mX, NULL, 66.7, 0.2));
  free(X);
  free(Y);
  free(mX);
  free(F);
  free(ids);
  printf(bad ? "non-finite result\n" : "oracle driver ok\n");
  return bad;
}
