// Host-side checks of libcountpairs under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only: the build passes each
// -fsanitize= after -Xarch_host).  The library's host source is included so
// its internal helpers can be driven directly: argument validation of every
// entry point, the binning tables and the binary32 error bound, the grid
// geometry, the column split of the queue items, the estimators and the
// tuning cache.  No device work is needed: on a machine without a GPU the
// first HIP call of a valid request fails cleanly with CP_ERR_DEVICE.
#include "../../paper_1911_08275_amd/csrc/api.hip"

#include <cstdio>
#include <cstdlib>

using namespace cp;

static int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);     \
      g_fail = 1;                                                         \
    }                                                                     \
  } while (0)

static void check_validation() {
  cp_options o;
  cp_default_options(&o);
  double x[4] = {1, 2, 3, 4};
  cp_points p{4, x, x, x, nullptr, CP_F64};
  uint64_t n[64];
  double w[64], r[64];
  const double good[3] = {0.5, 1.0, 2.0};
  CHECK(countpairs_xi(nullptr, good, 3, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_xi(&p, good, 1, &o, n, w, r) == CP_ERR_INVALID_ARG);
  const double dup[3] = {0.5, 0.5, 2.0}, neg[2] = {-1.0, 1.0}, nan_[2] = {0.0, NAN};
  CHECK(countpairs_xi(&p, dup, 3, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_xi(&p, neg, 2, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_xi(&p, nan_, 2, &o, n, w, r) == CP_ERR_INVALID_ARG);
  double many[80];
  for (int k = 0; k < 80; k++) many[k] = 0.1 * (k + 1);
  CHECK(countpairs_xi(&p, many, 80, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_xi(&p, good, 3, nullptr, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_xi(&p, good, 3, &o, nullptr, w, r) == CP_ERR_INVALID_ARG);
  cp_options bad = o;
  bad.precision = 9;
  CHECK(countpairs_xi(&p, good, 3, &bad, n, w, r) == CP_ERR_INVALID_ARG);
  bad = o;
  bad.periodic = 1;
  bad.boxsize = -1;
  CHECK(countpairs_xi(&p, good, 3, &bad, n, w, r) == CP_ERR_INVALID_ARG);
  bad = o;
  bad.need_ravg = 1;
  CHECK(countpairs_xi(&p, good, 3, &bad, n, nullptr, r) == CP_ERR_INVALID_ARG);
  bad = o;
  bad.refine[1] = -2;
  CHECK(countpairs_xi(&p, good, 3, &bad, n, w, r) == CP_ERR_INVALID_ARG);
  bad = o;
  bad.no_prune = 3;
  CHECK(countpairs_xi(&p, good, 3, &bad, n, w, r) == CP_ERR_INVALID_ARG);
  cp_points q = p;
  q.n = -5;
  CHECK(countpairs_xi(&q, good, 3, &o, n, w, r) == CP_ERR_INVALID_ARG);
  q = p;
  q.dtype = 7;
  CHECK(countpairs_xi(&q, good, 3, &o, n, w, r) == CP_ERR_INVALID_ARG);
  q = p;
  q.y = nullptr;
  CHECK(countpairs_xi(&q, good, 3, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_wp(&p, good, 3, 0.0, 4, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_wp(&p, good, 3, 10.0, 0, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_wp(&p, good, 3, 10.0, 100000, &o, n, w, r) == CP_ERR_INVALID_ARG);
  CHECK(countpairs_cross(&p, nullptr, good, 3, &o, n, w, r) == CP_ERR_INVALID_ARG);
  cp_options wso = o;
  wso.workspace = x;
  CHECK(countpairs_xi_noalloc(&p, good, 3, &wso, n, w, r) == CP_ERR_INVALID_ARG);
  // no points: zero counts without device work
  cp_points e0{0, nullptr, nullptr, nullptr, nullptr, CP_F64};
  n[0] = n[1] = 7;
  CHECK(countpairs_xi(&e0, good, 3, &o, n, w, r) == CP_OK);
  CHECK(n[0] == 0 && n[1] == 0);
  // a valid request: device work (CP_OK on a GPU, CP_ERR_DEVICE without)
  const int rc = countpairs_xi(&p, good, 3, &o, n, w, r);
  CHECK(rc == CP_OK || rc == CP_ERR_DEVICE);
  CHECK(strlen(countpairs_last_error()) > 0 || rc == CP_OK);
  for (int c = -8; c <= 1; c++) CHECK(countpairs_strerror(c) != nullptr);
  cp_plan *pl = nullptr;
  CHECK(cp_plan_create(&p, 0, good, 3, nullptr, 0, 0.0, 1, &o, &pl) == CP_ERR_INVALID_ARG);
  CHECK(cp_plan_create(&p, 1, good, 3, nullptr, 0, 0.0, 1, &o, &pl) == CP_ERR_INVALID_ARG);
  CHECK(cp_plan_destroy(nullptr) == CP_OK);
  CHECK(countpairs_workspace_size(0, 1000, 0, good, 3, 0.0, 1, &o) > 0);
  CHECK(countpairs_workspace_size(3, 1000, 2000, good, 3, 40.0, 40, &o) > 0);
  CHECK(countpairs_workspace_size(0, -1, 0, good, 3, 0.0, 1, &o) == 0);
}

static void check_binning() {
  // edges from zero, tight log spacing, wide spans; both precisions, both
  // statistics; the tables must build or fail cleanly
  for (int mode = XI; mode <= WP; mode++)
    for (int prec = F64; prec <= F32R; prec++)
      for (int variant = 0; variant < 5; variant++) {
        double e[61];
        int ne = 15;
        for (int k = 0; k < ne; k++) e[k] = 0.1 * std::pow(250.0, k / 14.0);
        if (variant == 1) e[0] = 0.0;
        if (variant == 2) {
          ne = 61;
          for (int k = 0; k < ne; k++) e[k] = 1e-3 * std::pow(1e6, k / 60.0);
        }
        if (variant == 3) {
          ne = 3;
          e[0] = 10.0;
          e[1] = 10.0 + 1e-9;
          e[2] = 10.0 + 2e-9;
        }
        if (variant == 4) {
          ne = 2;
          e[0] = 0.0;
          e[1] = 1e-30;
        }
        const double lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
        const int ref[3] = {2, 2, 2};
        Geometry g = choose_geometry(mode, true, 420.0, lo, ext, e[ne - 1], 40.0, ref, 1000000);
        Binning B;
        const int rc = make_binning(mode, prec, e, ne, 40.0, 40, g, 420.0, B);
        CHECK(rc == CP_OK || rc == CP_ERR_INVALID_ARG);
        if (rc == CP_OK) {
          CHECK(B.t64.e.size() >= 1 && B.t64.e.size() <= kTabMax);
          CHECK(B.E.size() == ne);
          for (int k = 1; k < ne; k++) CHECK(B.E[k] >= B.E[k - 1]);
        }
      }
}

static void check_geometry() {
  const double lo[3] = {-5.0, 3.0, 0.0};
  for (int periodic = 0; periodic <= 1; periodic++)
    for (double R : {0.01, 1.0, 25.0, 100.0, 300.0, 1e6})
      for (int r = 0; r <= 9; r++) {
        const double ext[3] = {420.0, periodic ? 420.0 : 1e-12, periodic ? 420.0 : 0.0};
        const int ref[3] = {r, (r + 1) % 10, 8};
        for (int64_t npts : {(int64_t)0, (int64_t)1, (int64_t)1000, (int64_t)1000000000}) {
          Geometry g = choose_geometry(r % 2 ? XI : WP, periodic, 420.0, lo, ext, R, R * 1.5,
                                       ref, npts);
          for (int a = 0; a < 3; a++) {
            CHECK(g.n[a] >= 1 && g.n[a] <= kMaxAxisCells);
            CHECK(g.r[a] >= 0 && g.r[a] <= 8);
            CHECK(!periodic || g.wrap[a] || g.n[a] >= 2 * g.r[a] + 1);
          }
          CHECK(g.maxspan >= 1);
          PairParams P;
          memset(&P, 0, sizeof(P));
          for (int chunk : {10, 70, 100, 140, 1000}) {
            split_columns(g, r % 2 == 0, R, R, (double)npts, 2.0, chunk, P);
            CHECK(P.nsplit >= 1 && P.nsplit <= kMaxChunks);
            for (int k = 0; k < P.nsplit; k++) CHECK(P.chunk[k] < P.chunk[k + 1]);
          }
        }
      }
}

static void check_estimators() {
  const double e[4] = {1.0, 2.0, 5.0, 10.0};
  double rr[3 * 8];
  CHECK(cp_rr_periodic_xi(1000, 100.0, e, 4, CP_ORDERED, rr) == CP_OK);
  CHECK(cp_rr_periodic_xi(1000, 10.0, e, 4, CP_ORDERED, rr) == CP_ERR_INVALID_ARG);
  CHECK(cp_rr_periodic_xi(1000, 100.0, nullptr, 4, CP_ORDERED, rr) == CP_ERR_INVALID_ARG);
  CHECK(cp_rr_periodic_wp(1000, 100.0, e, 4, 20.0, 8, CP_UNIQUE, rr) == CP_OK);
  CHECK(cp_rr_periodic_wp(1000, 100.0, e, 4, 80.0, 8, CP_UNIQUE, rr) == CP_ERR_INVALID_ARG);
  uint64_t dd[3] = {10, 20, 30};
  double xi[3];
  CHECK(cp_xi_natural(dd, 1.0, rr, 1.0, 3, xi) == CP_OK);
  CHECK(cp_xi_natural(dd, 0.0, rr, 1.0, 3, xi) == CP_ERR_INVALID_ARG);
  double x2[3 * 8] = {0}, wp[3];
  CHECK(cp_wp_integrate(x2, 3, 8, 20.0, wp) == CP_OK);
  CHECK(cp_wp_integrate(x2, 3, 0, 20.0, wp) == CP_ERR_INVALID_ARG);
}

static void check_tune_cache(const char *dir) {
  const std::string path = std::string(dir) + "/at.json";
  FILE *f = fopen(path.c_str(), "w");
  CHECK(f != nullptr);
  if (!f) return;
  fprintf(f, "{\n \"good\": {\"refine\": [2, 3, 1], \"chunk_pct\": 70, \"waves\": 2, \"ms\": 1.5},\n");
  fprintf(f, " \"bad refine\": {\"refine\": [0, 3, 1], \"chunk_pct\": 70, \"waves\": 2, \"ms\": 1.5},\n");
  fprintf(f, " \"truncated\": {\"refine\": [2, 3\n \"\n garbage \" \"\" {{{ \n");
  std::string longline(5000, 'x');
  fprintf(f, "\"%s\": {}\n}\n", longline.c_str());
  fclose(f);
  setenv("CP_AUTOTUNE_CACHE", path.c_str(), 1);
  TuneChoice t;
  CHECK(tune_lookup("good", t) && t.refine[1] == 3 && t.chunk_pct == 70 && t.waves == 2);
  CHECK(!tune_lookup("bad refine", t));
  CHECK(!tune_lookup("truncated", t));
  TuneChoice u;
  u.refine[0] = 4;
  u.ms = 2.25;
  tune_store("new/key", u);
  setenv("CP_AUTOTUNE_CACHE", (path + ".other").c_str(), 1);
  CHECK(!tune_lookup("good", t));            // another file, another cache
  setenv("CP_AUTOTUNE_CACHE", path.c_str(), 1);
  CHECK(tune_lookup("new/key", t) && t.refine[0] == 4);
  CHECK(tune_lookup("good", t));
}

int main(int argc, char **argv) {
  check_validation();
  check_binning();
  check_geometry();
  check_estimators();
  check_tune_cache(argc > 1 ? argv[1] : "/tmp");
  if (!g_fail) printf("host checks passed\n");
  return g_fail;
}
