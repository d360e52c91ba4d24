/* Host-only checks of the library's parameter derivation and validation
 * (dpse_derive, dpse_workspace_size, dpse_status_string), meant to run in a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer on the host code.
 * Draws parameter sets from a mix of valid and invalid values (zero,
 * negative, NaN, infinite, huge, odd or non-power-of-two sizes, every flag
 * combination) with a fixed xorshift generator; for every accepted set it
 * checks the derived quantities against the rules of the C ABI's header.
 * Exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dpse.h"

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) {
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return rs;
}
static double unif(void) { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }

static double pick_pos(double lo, double hi) {
  switch (next() % 12) {
    case 0: return 0.0;
    case 1: return -unif() * hi;
    case 2: return NAN;
    case 3: return INFINITY;
    case 4: return 1e300;
    default: return lo + (hi - lo) * unif();
  }
}

static int pick_n(int lo, int hi) {
  switch (next() % 16) {
    case 0: return (int)(next() % 3000) - 500;  /* anything, often not a power of two */
    case 1: return hi * 2;
    default: {
      int v = lo;
      int steps = (int)(next() % 6);
      for (int i = 0; i < steps && v * 2 <= hi; ++i) v *= 2;
      return v;
    }
  }
}

static int fails = 0;
#define CHECK(c, msg)                                             \
  do {                                                            \
    if (!(c)) {                                                   \
      if (fails < 20) fprintf(stderr, "check failed: %s\n", msg); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(int argc, char** argv) {
  const int iters = argc > 1 ? atoi(argv[1]) : 4000;
  int accepted = 0, rejected = 0;
  for (int it = 0; it < iters; ++it) {
    dpse_params p;
    memset(&p, 0, sizeof(p));
    const int nxy = pick_n(32, 1024);
    const double h = 0.05 + unif();
    p.Nx = nxy;
    p.Ny = (next() % 4) ? nxy : pick_n(32, 1024);
    p.Lx = (next() % 6) ? p.Nx * h : pick_pos(1.0, 100.0);
    p.Ly = (next() % 6) ? p.Ny * h : pick_pos(1.0, 100.0);
    p.H = (next() % 6) ? 4.0 + 60.0 * unif() : pick_pos(0.1, 100.0);
    p.eps = (next() % 6) ? 1.0 : pick_pos(0.01, 50.0);
    p.eps_bottom = (next() % 3) ? p.eps : pick_pos(0.01, 50.0);
    p.eps_top = (next() % 3) ? p.eps : pick_pos(0.01, 50.0);
    p.xi = (next() % 6) ? 0.5 + 3.0 * unif() : pick_pos(0.01, 10.0);
    p.g_w = (next() % 4) ? 0.0 : pick_pos(0.0, 0.2);
    p.Nz = (next() % 8) ? pick_n(32, 1024) + 1 : pick_n(16, 2048);
    p.support = (next() % 3) ? 0 : (int)(next() % 40) - 4;
    p.r_cut = (next() % 3) ? 0.0 : pick_pos(0.1, 10.0);
    p.delta = (next() % 3) ? 0.0 : pick_pos(1e-8, 1e-2);
    p.precision = (next() % 8) ? (int)(next() % 2) : (int)(next() % 5) - 2;
    /* mostly the flags that combine with any slab (gauge, cap, deterministic),
       sometimes any combination of solver flags, rarely an unknown bit */
    p.flags = (next() % 3) ? (int)(next() % 4) | ((next() % 2) ? DPSE_DETERMINISTIC : 0) : (int)(next() % 64);
    if (next() % 16 == 0) p.flags |= 1 << (int)(next() % 31);

    dpse_info info;
    memset(&info, 0xA5, sizeof(info));
    const int st = dpse_derive(&p, &info);
    const int64_t max_n = (next() % 5) ? (int64_t)(next() % 100000) + 1 : (int64_t)(next() % 4) - 1;
    int64_t bytes = -1;
    const int sw = dpse_workspace_size(&p, max_n, &bytes);
    CHECK(dpse_status_string(st) != NULL && dpse_status_string((int)(next() % 64) - 8) != NULL, "status string");
    if (st != DPSE_OK) {
      CHECK(st == DPSE_EINVAL, "derive returns EINVAL or OK");
      CHECK(sw != DPSE_OK, "workspace size refused for refused parameters");
      ++rejected;
      continue;
    }
    ++accepted;
    CHECK(isfinite(p.Lx) && p.Lx > 0 && isfinite(p.Ly) && p.Ly > 0 && isfinite(p.H) && p.H > 0,
          "accepted lengths are positive and finite");
    CHECK(p.Nx >= 32 && p.Nx <= 1024 && (p.Nx & (p.Nx - 1)) == 0, "Nx a power of two in [32, 1024]");
    CHECK(p.Ny >= 32 && p.Ny <= 1024 && (p.Ny & (p.Ny - 1)) == 0, "Ny a power of two in [32, 1024]");
    CHECK(fabs(info.h - p.Lx / p.Nx) <= 1e-12 * info.h, "h = Lx / Nx");
    CHECK(fabs(p.Ly / p.Ny - info.h) <= 1e-12 * info.h, "equal spacings");
    CHECK(info.support >= 2 && info.support <= 32 && info.support % 2 == 0, "even support <= 32");
    CHECK(fabs(info.H_E - info.support * info.h / 2) <= 1e-12 * info.H_E, "H_E = n_g h / 2");
    CHECK(fabs(info.g_t * info.g_t - (1.0 / (4 * p.xi * p.xi) + p.g_w * p.g_w)) <= 1e-12 * info.g_t * info.g_t,
          "g_t^2 = 1/(4 xi^2) + g_w^2");
    CHECK(info.z_lo < info.z_hi, "domain ordered");
    CHECK(info.r_cut > 0 && info.r_cut < 0.5 * fmin(p.Lx, p.Ly), "cutoff inside half the box");
    CHECK(info.n_modes == p.Ny * (p.Nx / 2 + 1), "half-spectrum modes");
    CHECK(info.workspace_bytes == 0 && info.max_n == 0 && info.table_bytes == 0, "derive touches no device");
    if (max_n >= 1 && max_n <= ((int64_t)1 << 28)) {
      CHECK(sw == DPSE_OK && bytes > 0 && bytes % 256 == 0, "workspace size for a valid max_n");
    } else {
      CHECK(sw == DPSE_EINVAL, "workspace size refuses max_n out of range");
    }
  }
  printf("derive_fuzz: %d accepted, %d rejected, %d failed checks\n", accepted, rejected, fails);
  return fails ? 1 : 0;
}
