/*
 * countpairs.h - C ABI of the MI355X (gfx950) gridded pair-counting library.
 *
 * Operation (Sinha & Garrison, "Corrfunc: blazing fast correlation functions
 * with AVX512F SIMD intrinsics"):
 *   - Section 1.1, Code 1: the pair count is the histogram, over separation
 *     bins, of all pairs (i, j) with R_min <= sep < R_max; each pair adds one
 *     to its bin's count and its weight to the bin's weight sum.
 *   - Section 1.1, eqn:separations: xi(r) bins r = |p_j - p_i|; wp(rp) bins
 *     rp = sqrt(dx^2 + dy^2) and keeps pi = |dz| < pi_max (line of sight z).
 *   - Section 1.2 and Section 2.1: points are gridded into cells; only
 *     neighbouring cell pairs are searched; for an auto-count only unique
 *     pairs are searched and the total is doubled.
 *   - Section 2.2: cell pairs whose minimum possible separation (from the
 *     cells' bounding boxes) is at least R_max are skipped.
 *
 * Conventions shared by every entry point (all readings of the paper):
 *   - separations are compared squared: bin k holds E_k <= s < E_{k+1} with
 *     E_k = fl64(e_k * e_k) and s = ((dx*dx + dy*dy) + dz*dz) evaluated in
 *     binary64 without fused multiply-add; d = p_j - p_i per axis, wrapped to
 *     the minimum image when periodic (d > L/2 -> d - L, d < -L/2 -> d + L).
 *   - wp output is the 2-D histogram [rp bin][pi bin], rp-major, with pi bins
 *     q_l <= pi < q_{l+1}, q_l = fl64(l * fl64(pi_max / npibins)) for
 *     0 < l < npibins, q_0 = 0 and q_npibins = pi_max.
 *   - counts are exact.  CP_PREC_FP32_RECHECK evaluates distances in binary32
 *     with a derived error bound and re-evaluates in binary64 every pair whose
 *     binary32 value could lie on the other side of an edge, so its counts are
 *     identical to CP_PREC_FP64's (cp_stats.precision tells which precision
 *     a call ran; see there for the cases that run binary64).
 *   - weighted outputs: wsum_k = sum of w_i * w_j, ravg_k = sum of
 *     w_i * w_j * sep / wsum_k (sep = r for xi, rp for wp; 0 for empty bins).
 *     They are binary64 sums in an unspecified order (relative error far
 *     below 1e-12 for the supported sizes).  Absent weights mean w = 1.
 *
 * Memory: position and weight arrays are DEVICE pointers, owned by the
 * caller, read-only for the call and not retained after it returns.  Edges
 * and all outputs are HOST pointers.  Every countpairs_* call enqueues its
 * work on options->stream (NULL: the null stream) and synchronises that
 * stream before returning, so the status covers errors found on the device.
 * Calls on different host threads with different streams are independent;
 * each thread keeps its own cached device scratch buffers unless the caller
 * supplies a workspace.
 *
 * Errors: every entry point returns CP_OK (0) or a negative CP_ERR_* code;
 * countpairs_last_error() returns a thread-local message for the last failure.
 * No call frees caller memory; no C++ exception crosses this boundary.
 */
#ifndef COUNTPAIRS_H
#define COUNTPAIRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element type of cp_points.x/y/z */
enum { CP_F64 = 0, CP_F32 = 1 };
/* arithmetic of the distance evaluation */
enum { CP_PREC_FP64 = 0, CP_PREC_FP32_RECHECK = 1 };
/* auto-count convention: ordered pairs (each unordered pair counted twice,
 * as Section 2.1 obtains by doubling the unique-pair total) or unique
 * pairs (each unordered pair once) */
enum { CP_ORDERED = 0, CP_UNIQUE = 1 };

enum {
  CP_OK = 0,
  CP_ERR_INVALID_ARG = -1, /* bad edges, sizes, enums, box, null pointers */
  CP_ERR_OUT_OF_BOX = -2,  /* periodic coordinate outside [0, boxsize) */
  CP_ERR_NONFINITE = -3,   /* NaN or Inf in positions or weights */
  CP_ERR_NOMEM = -4,       /* allocation failed or workspace too small */
  CP_ERR_DEVICE = -5,      /* HIP runtime error (see countpairs_last_error) */
  CP_ERR_INTERNAL = -6     /* a device-side consistency check failed */
};

/* A point set: n points, SoA coordinates (CP_F64: double, CP_F32: float),
 * optional binary64 weights (NULL: unweighted).  Device pointers. */
typedef struct {
  int64_t n;
  const void *x, *y, *z;
  const double *w;
  int dtype;
} cp_points;

typedef struct {
  int precision;          /* CP_PREC_FP64 or CP_PREC_FP32_RECHECK */
  int periodic;           /* 1: cube [0, boxsize)^3, minimum-image separations */
  double boxsize;         /* side of the periodic cube (ignored otherwise) */
  int refine[3];          /* cells per R_max (pi_max along z for wp) per axis
                             (Section 3.1 bin_refine_factors).  All three 0: the
                             library chooses the refine factors, the queue
                             items' work-chunk target and the waves per
                             workgroup by timing candidates on the call's own
                             data (best of three whole calls each, coordinate
                             descent), and caches the choice per workload
                             signature (statistic, precision, weights, periodic,
                             log2 of the point counts and of the expected
                             neighbours per point, pi_max / R_max) in memory and
                             in a JSON file: $CP_AUTOTUNE_CACHE, else
                             $HOME/.cache/paper_1911_08275_amd/autotune.json.
                             The first call of a signature runs about 24 timed
                             calls.  CP_AUTOTUNE=0 in the environment switches
                             tuning off (refine 2,2,2).  Counts do not depend
                             on the choice. */
  int need_ravg;          /* 1: fill wsum and ravg */
  int count_mode;         /* CP_ORDERED (default) or CP_UNIQUE, auto-counts only */
  void *stream;           /* hipStream_t; NULL = null stream */
  void *workspace;        /* optional device scratch owned by the caller */
  size_t workspace_bytes; /* its size; too small -> CP_ERR_NOMEM */
  int no_prune;           /* 1: switch off the bounding-box tests of Section 2.2
                             (no cell pair is skipped, no z-window, no whole-unit
                             count): every pair of every cell within the refine
                             reach is evaluated.  For ablations and for checking
                             that pruning is exact; 0 (default) prunes. */
} cp_options;

/* Diagnostics of the last successful call on the calling thread. */
typedef struct {
  uint64_t candidates;       /* pair separations evaluated on the device */
  uint64_t rechecks;         /* binary32 pairs re-evaluated in binary64 */
  uint64_t cell_pairs;       /* (tile, cell) work units searched */
  uint64_t cell_pairs_pruned;/* units skipped by the bounding-box test */
  uint64_t tiles;            /* primary tiles of <= 64 points */
  int grid[3];               /* cells per axis */
  int refine[3];             /* refine factors used */
  float ms_grid;             /* device time of the cell build (ms) */
  float ms_pairs;            /* device time of the pair kernel (ms) */
  float ms_total;            /* device time of the whole call (ms) */
  int precision;             /* CP_PREC_* the pair kernel actually ran.  Binary64
                                runs whatever was asked for (a) on a grid with a
                                single wrapped cell on some axis (box under
                                three cells of reach: per-pair minimum images)
                                and (b) for weighted xi (need_ravg), where every
                                counted pair needs its binary64 separation and
                                the binary64 kernel is faster on gfx950; the
                                environment variable CP_XI_WEIGHTED_BINARY32=1
                                selects the binary32 screen for (b) instead
                                (candidates screened in binary32, the surviving
                                pairs evaluated in binary64: same counts) */
  int tuned;                 /* launch settings: 0 given by the caller (refine
                                set), 1 tuned during this call, 2 taken from
                                the tuning cache, 3 library defaults (tuning
                                switched off, or a cache miss in
                                countpairs_xi_noalloc) */
  int chunk_pct;             /* work-chunk target of the queue items, percent
                                of the library's estimate */
  int waves;                 /* waves per pair-kernel workgroup */
} cp_stats;

/* Fill *o with defaults: FP32 recheck, non-periodic, refine 0 (tuned by the
 * library), no ravg, ordered counts, null stream, library scratch. */
void cp_default_options(cp_options *o);

/*
 * xi(r) auto-count of d (Section 1.1 eqn:separations, first case).
 *   edges   2 <= nedges <= 61 host doubles (at most 60 bins), finite, strictly
 *           increasing, edges[0] >= 0
 *   npairs  nedges-1 host uint64 counts (required)
 *   wsum, ravg  nedges-1 host doubles each, written when need_ravg (then required)
 * Fewer than two points give zero counts and CP_OK.
 */
int countpairs_xi(const cp_points *d, const double *edges, int nedges,
                  const cp_options *o, uint64_t *npairs, double *wsum,
                  double *ravg);

/*
 * wp auto-count: 2-D histogram xi(rp, pi) (Section 1.1 eqn:separations,
 * second case; pi_max filter), line of sight z.
 *   rp_edges  as edges above, bins in rp
 *   pimax     > 0; 1 <= npibins <= 256 equal pi bins in [0, pimax)
 *   npairs    (nedges-1) * npibins host uint64, rp-major
 *   wsum, rpavg  same shape, when need_ravg
 * Each wave of the pair kernel keeps the whole 2-D histogram in LDS:
 * (nedges + 1) * npibins * 4 bytes, plus 16 bytes per entry when need_ravg,
 * must stay under ~159 KB (fewer waves per workgroup are used as it grows);
 * beyond that the call fails with CP_ERR_INVALID_ARG.
 */
int countpairs_wp(const cp_points *d, const double *rp_edges, int nedges,
                  double pimax, int npibins, const cp_options *o,
                  uint64_t *npairs, double *wsum, double *rpavg);

/*
 * countpairs_xi without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * countpairs_xi, except:
 *   - its device scratch is a static array of the library (64 MiB per device,
 *     held by every device the library runs on until the process ends), not
 *     the thread's cached buffers; a call that needs more (roughly more than
 *     500 000 points, depending on the grid) fails with CP_ERR_NOMEM and a
 *     message giving both sizes;
 *   - o->workspace must be NULL (CP_ERR_INVALID_ARG otherwise);
 *   - it creates no HIP events, so the ms_* fields of countpairs_last_stats
 *     are 0; it calls no hipMalloc/hipFree and no other allocating routine;
 *   - every call on one device shares that device's scratch: calls that
 *     overlap on one device (two host threads, or two streams) race and give
 *     undefined results.  The call still synchronises o->stream before it
 *     returns, so calls made one after the other are safe.
 */
int countpairs_xi_noalloc(const cp_points *d, const double *edges, int nedges,
                          const cp_options *o, uint64_t *npairs, double *wsum,
                          double *ravg);

/*
 * xi(r) cross-count: every ordered pair (i in d1, j in d2) (Section 1.1: the
 * DR and RR terms of survey geometries; Section 2.1: no symmetry for cross
 * correlations).  count_mode is ignored.  Pair weight w1_i * w2_j.
 */
int countpairs_cross(const cp_points *d1, const cp_points *d2,
                     const double *edges, int nedges, const cp_options *o,
                     uint64_t *npairs, double *wsum, double *ravg);

/* wp cross-count (same conventions as countpairs_wp and countpairs_cross). */
int countpairs_cross_wp(const cp_points *d1, const cp_points *d2,
                        const double *rp_edges, int nedges, double pimax,
                        int npibins, const cp_options *o, uint64_t *npairs,
                        double *wsum, double *rpavg);

/* Device scratch (bytes) a call on n1 (+ n2 for cross) points needs at most,
 * for a caller-supplied workspace.  kind: 0 xi, 1 wp, 2 cross, 3 cross_wp. */
size_t countpairs_workspace_size(int kind, int64_t n1, int64_t n2,
                                 const double *edges, int nedges, double pimax,
                                 int npibins, const cp_options *o);

const char *countpairs_strerror(int code);
const char *countpairs_last_error(void);
int countpairs_last_stats(cp_stats *out);

/*
 * Batched plan: many catalogues of uneven size counted together (Section 1.1
 * motivates many correlation-function evaluations, e.g. inside MCMC).  All
 * catalogues share the periodic box, the bins and the precision; plans
 * count pairs only (the catalogues' weights are not read).  One execute
 * enqueues, on one stream, the cell build of every catalogue and persistent
 * pair launches that drain a shared queue of tiles ordered by decreasing
 * cost: one for xi and one for wp, or, in binary32 when every xi pair lies
 * inside the wp search (xi R_max at most r_p,max and pi_max), one launch that
 * counts both.  Execute allocates nothing and is safe to capture in a
 * hipGraph; the plan owns all scratch memory.
 *
 *   cp_plan_create   mocks: nmocks point sets (device pointers read at every
 *                    execute, so the caller may refill them in place);
 *                    xi_edges / wp_edges may be NULL to skip that statistic;
 *                    o: precision, refine, periodic (must be 1) and boxsize.
 *                    refine 0: the settings are tuned (and cached) by timing
 *                    single calls of the requested statistics on the median
 *                    catalogue, or, for the single binary32 launch, trial
 *                    plans of up to four catalogues picked at even quantiles
 *                    of the pair work (n^2).
 *   cp_plan_execute  enqueue one evaluation on stream (asynchronous).
 *   cp_plan_results  synchronise the stream of the last execute and copy counts:
 *                    xi_npairs nmocks*(xi_nedges-1), wp_npairs
 *                    nmocks*(wp_nedges-1)*npibins (either may be NULL);
 *                    auto-counts follow o->count_mode.  CP_ERR_INTERNAL when a
 *                    work queue was not drained (the counts would be short).
 *   cp_plan_destroy  free everything (NULL is fine).
 */
typedef struct cp_plan cp_plan;

int cp_plan_create(const cp_points *mocks, int nmocks, const double *xi_edges,
                   int xi_nedges, const double *wp_edges, int wp_nedges,
                   double pimax, int npibins, const cp_options *o,
                   cp_plan **out);
int cp_plan_execute(cp_plan *plan, void *stream);
int cp_plan_results(cp_plan *plan, uint64_t *xi_npairs, uint64_t *wp_npairs);
int cp_plan_stats(cp_plan *plan, cp_stats *xi_stats, cp_stats *wp_stats);
int cp_plan_destroy(cp_plan *plan);

/*
 * Estimators on top of the counts (Section 1).  Host functions on host
 * arrays: they touch no device and need no stream.
 *
 *   cp_rr_periodic_xi  expected pair counts of n uniformly random points in a
 *       periodic cube of side boxsize (Section 1: the random-pair term is
 *       analytic for a periodic cube), per bin [e_k, e_k+1):
 *       n (n - 1) * (4 pi / 3) (e_k+1^3 - e_k^3) / L^3 ordered pairs, half of
 *       that for CP_UNIQUE.  rr: nedges - 1 doubles.  The largest edge must
 *       not exceed boxsize / 2 (minimum-image shells beyond are cut by the
 *       cube): CP_ERR_INVALID_ARG.
 *   cp_rr_periodic_wp  the same for the 2-D (r_p, pi) bins of countpairs_wp:
 *       n (n - 1) * pi (e_k+1^2 - e_k^2) * 2 dpi / L^3 (both signs of the
 *       line-of-sight separation), dpi = pimax / npibins, rr rp-major
 *       (nedges - 1) * npibins doubles; needs pimax <= boxsize / 2 too.
 *   cp_xi_natural  xi_k = (dd_k / dd_norm) / (rr_k / rr_norm) - 1 (Section 1,
 *       eqn:xi), for nbins bins; with rr from cp_rr_periodic_* on the same
 *       count convention both norms are 1; with pair-counted randoms they are
 *       the pair totals, e.g. n_D (n_D - 1) and n_R (n_R - 1).  A bin with
 *       rr_k = 0 gives NaN.
 *   cp_wp_integrate  w_p(r_p,k) = 2 * sum_l xi(r_p,k, pi_l) * dpi, the
 *       line-of-sight integral of Section 1 as a sum over the npibins bins of
 *       width pimax / npibins; xi2d rp-major, wp nrpbins doubles.
 *
 * Errors: CP_ERR_INVALID_ARG (NULL arrays, bad edges, sizes, enums, norms).
 */
int cp_rr_periodic_xi(int64_t n, double boxsize, const double *edges, int nedges,
                      int count_mode, double *rr);
int cp_rr_periodic_wp(int64_t n, double boxsize, const double *rp_edges, int nedges,
                      double pimax, int npibins, int count_mode, double *rr);
int cp_xi_natural(const uint64_t *dd, double dd_norm, const double *rr, double rr_norm,
                  int nbins, double *xi);
int cp_wp_integrate(const double *xi2d, int nrpbins, int npibins, double pimax, double *wp);

#ifdef __cplusplus
}
#endif

#endif /* COUNTPAIRS_H */
