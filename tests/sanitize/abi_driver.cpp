// Calls the C ABI's host paths — argument validation of every entry point
// (fake pointers, rejected before any device call) and the host Kabsch
// solver — in a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer. Exits 0 when every call returns the expected
// status.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "fga.h"

static int fails = 0;
static void expect(fga_status got, fga_status want, const char* what) {
  if (got != want) {
    std::printf("%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, fga_last_error());
    ++fails;
  }
}

int main() {
  fga_params p;
  expect(fga_default_params(&p), FGA_OK, "default params");
  void* fake = reinterpret_cast<void*>(0x1000);
  double R[9], t[3], E = 0.0;
  long long cnt = 0;
  const int64_t idx[2] = {0, 99};
  expect(fga_forces(fake, 0, fake, 10, fake, nullptr, FGA_F32, 0.5, &p, fake, &cnt, nullptr),
         FGA_E_INVALID_ARG, "forces m = 0");
  expect(fga_forces(fake, 10, fake, 10, fake, nullptr, FGA_F32, -1.0, &p, fake, &cnt, nullptr),
         FGA_E_INVALID_ARG, "forces theta < 0");
  expect(fga_energy(fake, 10, fake, 10, nullptr, nullptr, FGA_F32, 0.0, &p, &E, &cnt, nullptr),
         FGA_E_INVALID_ARG, "energy mX NULL");
  expect(fga_masses_landmarks(fake, FGA_F32, 10, idx, 2, &p, 0, fake, nullptr), FGA_E_INVALID_ARG,
         "landmark index out of range");
  expect(fga_register(fake, 10, nullptr, 10, FGA_F32, &p, R, t, nullptr, nullptr), FGA_E_INVALID_ARG,
         "register Y NULL");
  expect(fga_forces_direct_noalloc(fake, 1 << 20, fake, 1 << 23, fake, nullptr, FGA_F32, &p, fake,
                                   nullptr),
         FGA_E_INVALID_ARG, "no-alloc scratch too small");
  fga_params q = p;
  q.eta = 1.5;
  expect(fga_register(fake, 10, fake, 10, FGA_F32, &q, R, t, nullptr, nullptr), FGA_E_INVALID_ARG,
         "fraction damping eta > 1");
  q = p;
  q.group_width = 48;
  expect(fga_register(fake, 10, fake, 10, FGA_F32, &q, R, t, nullptr, nullptr), FGA_E_INVALID_ARG,
         "group_width 48");
  const void* frames[1] = {fake};
  const int64_t sizes[1] = {10};
  expect(fga_register_sequence(1, frames, sizes, FGA_F32, &p, R, t, nullptr, nullptr, nullptr, nullptr),
         FGA_E_INVALID_ARG, "sequence of one frame");
  // host Kabsch solver: a rotation about z by 0.3 rad is recovered from C = R S
  const double c = std::cos(0.3), s = std::sin(0.3);
  const double C[9] = {2 * c, -1 * s, 0, 2 * s, 1 * c, 0, 0, 0, 0.5};
  expect(fga_kabsch(C, R), FGA_OK, "kabsch");
  if (std::fabs(R[0] - c) > 1e-12 || std::fabs(R[3] - s) > 1e-12) {
    std::printf("kabsch: wrong rotation\n");
    ++fails;
  }
  const double C1[9] = {1, 0, 0, 0, 0, 0, 0, 0, 0};
  expect(fga_kabsch(C1, R), FGA_E_DEGENERATE, "kabsch rank 1");
  std::printf(fails ? "abi driver: %d failures\n" : "abi driver ok\n", fails);
  return fails;
}
