/* The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
 * oracle's source is included, then both enumerations (plain loop and
 * chaining mesh) run on random catalogues -- auto and cross, xi and wp,
 * periodic and not, first edge 0 and positive, coincident points, a single
 * point, none -- and must agree; invalid arguments must return their error
 * codes.  Test infrastructure, like the oracle itself. */
#include "../../oracle/oracle.c"

#include <stdio.h>

static int g_fail = 0;
#define CHECK(c)                                                           \
  do {                                                                     \
    if (!(c)) {                                                            \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);      \
      g_fail = 1;                                                          \
    }                                                                      \
  } while (0)

static uint64_t s_state = 88172645463325252ull;
static double urand(void) { /* xorshift64*: inputs only */
  s_state ^= s_state >> 12;
  s_state ^= s_state << 25;
  s_state ^= s_state >> 27;
  return (double)((s_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static void fill(double *p, int64_t n, double lo, double ext) {
  for (int64_t i = 0; i < n; i++) p[i] = lo + urand() * ext;
}

int main(void) {
  enum { N1 = 700, N2 = 500 };
  static double x1[N1], y1[N1], z1[N1], w1[N1], x2[N2], y2[N2], z2[N2], w2[N2];
  const double L = 60.0;
  for (int trial = 0; trial < 24; trial++) {
    const int mode = trial & 1, periodic = (trial >> 1) & 1, autoc = (trial >> 2) & 1;
    const int64_t n1 = trial % 6 == 5 ? 1 : (trial % 6 == 4 ? 0 : N1);
    fill(x1, N1, 0, L), fill(y1, N1, 0, L), fill(z1, N1, 0, L), fill(w1, N1, 0.5, 1.0);
    fill(x2, N2, 0, L), fill(y2, N2, 0, L), fill(z2, N2, 0, L), fill(w2, N2, 0.5, 1.0);
    for (int i = 0; i < 40 && n1 > 80; i++) { /* coincident points */
      x1[i] = x1[i + 40];
      y1[i] = y1[i + 40];
      z1[i] = z1[i + 40];
    }
    double edges[9] = {trial % 3 == 0 ? 0.0 : 0.3, 0.7, 1.5, 3.0, 5.0, 8.0, 12.0, 17.0, 22.0};
    uint64_t ca[8 * 7], cb[8 * 7];
    double wa[8 * 7], wb[8 * 7], ra[8 * 7], rb[8 * 7];
    for (int grid = 0; grid <= 1; grid++) {
      const int rc = oracle_count(mode, autoc, n1, x1, y1, z1, w1, N2, x2, y2, z2, w2, periodic, L,
                                  edges, 9, 13.0, 7, grid, 2, grid ? cb : ca, grid ? wb : wa,
                                  grid ? rb : ra);
      CHECK(rc == ORACLE_OK);
    }
    const int nout = 8 * (mode ? 7 : 1);
    for (int k = 0; k < nout; k++) {
      CHECK(ca[k] == cb[k]);
      CHECK(fabs(wa[k] - wb[k]) <= 1e-12 * fabs(wa[k]) + 1e-300);
      CHECK(fabs(ra[k] - rb[k]) <= 1e-12 * fabs(ra[k]) + 1e-300);
    }
  }
  uint64_t c[4];
  double e2[2] = {1.0, 1.0};
  CHECK(oracle_count(ORACLE_XI, 1, N1, x1, y1, z1, NULL, 0, NULL, NULL, NULL, NULL, 0, 0.0, e2, 2,
                     0.0, 1, 1, 1, c, NULL, NULL) == ORACLE_ERR_ARG);
  double e3[2] = {0.5, 1.0};
  x1[3] = L + 1.0;
  CHECK(oracle_count(ORACLE_XI, 1, N1, x1, y1, z1, NULL, 0, NULL, NULL, NULL, NULL, 1, L, e3, 2,
                     0.0, 1, 1, 1, c, NULL, NULL) == ORACLE_ERR_OUT_OF_BOX);
  x1[3] = NAN;
  CHECK(oracle_count(ORACLE_XI, 1, N1, x1, y1, z1, NULL, 0, NULL, NULL, NULL, NULL, 0, 0.0, e3, 2,
                     0.0, 1, 1, 1, c, NULL, NULL) == ORACLE_ERR_NONFINITE);
  CHECK(oracle_count(ORACLE_WP, 1, 4, y1, y1, y1, NULL, 0, NULL, NULL, NULL, NULL, 0, 0.0, e3, 2,
                     -1.0, 1, 1, 1, c, NULL, NULL) == ORACLE_ERR_ARG);
  if (!g_fail) printf("oracle checks passed\n");
  return g_fail;
}
