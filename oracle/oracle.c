/*
 * CPU FP64 oracle for gridded pair counting (Sinha & Garrison, "Corrfunc:
 * Blazing fast correlation functions with AVX512F SIMD intrinsics").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * What it computes (all in IEEE binary64, built with -ffp-contract=off so no
 * multiply-add is ever fused):
 *
 *   The naive pair-count definition (Section 1.1, Code 1): for every i in set
 *   1 and every j in set 2 (j != i for an auto-count), compute the separation,
 *   drop it when it falls outside [R_min, R_max), find its histogram bin, add
 *   one to the count and the pair weight to the weight sum.
 *
 *   Separations follow the two metrics of Section 1.1 (eqn:separations):
 *     xi(r):   r^2   = dx^2 + dy^2 + dz^2, accept r < R_max
 *     wp(rp):  rp^2  = dx^2 + dy^2,  pi = |dz|, accept rp < R_max, pi < pi_max
 *   Comparisons are made on squared separations (Section 2.2, "Vector
 *   intrinsics in existing SIMD kernels", and Code 4), against squared edges.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - d_a = fl(p2_a - p1_a); in a periodic box of side L, if d_a > L/2 then
 *     d_a = fl(d_a - L), else if d_a < -L/2 then d_a = fl(d_a + L)
 *     (minimum image, the periodic cube of Section 1.1).
 *   - s = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)), left to right, unfused
 *     (the operation order of Code 3: rp^2 first, then + dz^2).
 *   - squared edges E_k = fl(e_k * e_k); bin k iff E_k <= s < E_{k+1}
 *     (half-open: Code 1 skips a separation below the smallest edge or at or
 *     above the largest one).
 *   - wp is kept as the 2-D histogram xi(rp, pi) of Section 1.1: pi bin l
 *     iff q_l <= pi < q_{l+1} with q_l = fl(l * fl(pi_max / npibins)) for
 *     0 < l < npibins, q_0 = 0 and q_npibins = pi_max.  Summing over l gives
 *     the paper's 1-D rp histogram with the pi < pi_max filter.
 *   - the pair weight is w_i * w_j; the weighted separation sum adds
 *     w_i * w_j * sqrt(s) (xi) or w_i * w_j * sqrt(rp^2) (wp).  Sums are
 *     Neumaier-compensated so the oracle's own rounding stays far below the
 *     1e-12 relative tolerance used against the GPU.
 *   - auto-counts are returned as ORDERED pairs (each unordered pair twice),
 *     which is what counting unique pairs and doubling the total afterwards
 *     (Section 2.1, "Reducing the number of cell pairs") gives.  The oracle
 *     visits ordered pairs directly and never doubles.
 *
 * Two enumerations of the same definition:
 *   oracle_count(..., use_grid = 0): the plain double loop of Code 1.
 *   oracle_count(..., use_grid = 1): the chaining mesh of Section 1.2 -
 *     cells of side at least R_max (pi_max along z for wp); every pair inside
 *     R_max lies in the 27 neighbouring cells (fewer when an axis has fewer
 *     than 3 cells, neighbours de-duplicated).  No refinement, no bounding
 *     box pruning, no sorting: only the neighbourhood rule of Section 1.2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_XI = 0, ORACLE_WP = 1 };

enum {
  ORACLE_OK = 0,
  ORACLE_ERR_ARG = -1,
  ORACLE_ERR_OUT_OF_BOX = -2,
  ORACLE_ERR_NONFINITE = -3,
  ORACLE_ERR_NOMEM = -4
};

/* Neumaier compensated accumulator. */
typedef struct {
  double sum, comp;
} nsum;

static void nsum_add(nsum *a, double v) {
  double t = a->sum + v;
  if (fabs(a->sum) >= fabs(v))
    a->comp += (a->sum - t) + v;
  else
    a->comp += (v - t) + a->sum;
  a->sum = t;
}

/* Minimum-image separation along one axis (periodic cube, Section 1.1). */
static double sep_axis(double a, double b, int periodic, double L, double halfL) {
  double d = b - a;
  if (periodic) {
    if (d > halfL)
      d = d - L;
    else if (d < -halfL)
      d = d + L;
  }
  return d;
}

typedef struct {
  int mode;
  int periodic;
  double L, halfL;
  int nbins;          /* separation bins */
  const double *E;    /* squared edges, nbins + 1 */
  double pimax;
  int npibins;
  const double *q;    /* pi edges, npibins + 1 (q[0] = 0, q[npibins] = pimax) */
  int nout;           /* nbins * (mode == wp ? npibins : 1) */
} pair_rule;

/* Bin of a squared separation: k with E[k] <= s < E[k+1], or -1. */
static int sep_bin(const pair_rule *R, double s) {
  if (s < R->E[0] || s >= R->E[R->nbins]) return -1;
  int k = 0;
  while (k + 1 < R->nbins && s >= R->E[k + 1]) k++;
  return k;
}

/* Pi bin: l with q[l] <= pi < q[l+1], or -1 when pi >= pi_max. */
static int pi_bin(const pair_rule *R, double pi) {
  if (pi >= R->pimax) return -1;
  int l = 0;
  while (l + 1 < R->npibins && pi >= R->q[l + 1]) l++;
  return l;
}

/* Evaluate one ordered pair; returns the output slot or -1, and the
 * separation whose square root is averaged (s for xi, rp^2 for wp). */
static int eval_pair(const pair_rule *R, double x1, double y1, double z1,
                     double x2, double y2, double z2, double *sq_out) {
  double dx = sep_axis(x1, x2, R->periodic, R->L, R->halfL);
  double dy = sep_axis(y1, y2, R->periodic, R->L, R->halfL);
  double dz = sep_axis(z1, z2, R->periodic, R->L, R->halfL);
  double xx = dx * dx;
  double yy = dy * dy;
  double rp2 = xx + yy;
  if (R->mode == ORACLE_XI) {
    double zz = dz * dz;
    double s = rp2 + zz;
    int k = sep_bin(R, s);
    *sq_out = s;
    return k;
  } else {
    int k = sep_bin(R, rp2);
    if (k < 0) return -1;
    int l = pi_bin(R, fabs(dz));
    if (l < 0) return -1;
    *sq_out = rp2;
    return k * R->npibins + l;
  }
}

typedef struct {
  uint64_t *cnt;
  nsum *w, *wr;
} accum;

static void accum_pair(accum *A, int slot, double weight, double sq) {
  A->cnt[slot] += 1;
  nsum_add(&A->w[slot], weight);
  nsum_add(&A->wr[slot], weight * sqrt(sq));
}

/* ------------------------------------------------------------------ grid */

typedef struct {
  int n[3];
  double lo[3], cs[3];
  int64_t *start; /* ncell + 1 */
  int64_t *idx;   /* point indices grouped by cell */
} cellgrid;

static int cell_of(const cellgrid *G, int a, double v) {
  double t = (v - G->lo[a]) / G->cs[a];
  int c = (int)floor(t);
  if (c < 0) c = 0;
  if (c >= G->n[a]) c = G->n[a] - 1;
  return c;
}

/* Cells of side >= reach along each axis (Section 1.2). */
static int grid_build(cellgrid *G, int64_t n, const double *x, const double *y,
                      const double *z, const double lo[3], const double ext[3],
                      const double reach[3]) {
  const double *p[3] = {x, y, z};
  int64_t ncell = 1;
  for (int a = 0; a < 3; a++) {
    int na = 1;
    if (ext[a] > 0 && reach[a] > 0) {
      /* the 1e-9 margin keeps computed cell indices of two points closer
       * than `reach` at most one apart despite rounding */
      double f = floor(ext[a] / (reach[a] * (1.0 + 1e-9)));
      if (f > 1) na = f > 1024 ? 1024 : (int)f;
    }
    G->n[a] = na;
    G->lo[a] = lo[a];
    G->cs[a] = ext[a] > 0 ? ext[a] / na : 1.0;
    ncell *= na;
  }
  G->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  G->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int *cid = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  if (!G->start || !G->idx || !cid) {
    free(G->start); free(G->idx); free(cid);
    return ORACLE_ERR_NOMEM;
  }
  for (int64_t i = 0; i < n; i++) {
    int c[3];
    for (int a = 0; a < 3; a++) c[a] = cell_of(G, a, p[a][i]);
    cid[i] = (c[0] * G->n[1] + c[1]) * G->n[2] + c[2];
    G->start[cid[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; c++) G->start[c + 1] += G->start[c];
  int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  if (!fill) { free(G->start); free(G->idx); free(cid); return ORACLE_ERR_NOMEM; }
  memcpy(fill, G->start, (size_t)ncell * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) G->idx[fill[cid[i]]++] = i;
  free(fill);
  free(cid);
  return ORACLE_OK;
}

static void grid_free(cellgrid *G) {
  free(G->start);
  free(G->idx);
}

/* Distinct neighbour cell coordinates along one axis (offsets -1, 0, +1,
 * wrapped when periodic, clipped otherwise, duplicates removed). */
static int axis_neighbours(int c, int n, int periodic, int out[3]) {
  int m = 0;
  for (int o = -1; o <= 1; o++) {
    int t = c + o;
    if (periodic) {
      t = ((t % n) + n) % n;
    } else if (t < 0 || t >= n) {
      continue;
    }
    int dup = 0;
    for (int k = 0; k < m; k++) dup |= (out[k] == t);
    if (!dup) out[m++] = t;
  }
  return m;
}

/* ------------------------------------------------------------- validation */

static int check_points(int64_t n, const double *x, const double *y,
                        const double *z, const double *w, int periodic, double L) {
  const double *p[3] = {x, y, z};
  for (int64_t i = 0; i < n; i++) {
    for (int a = 0; a < 3; a++) {
      double v = p[a][i];
      if (!isfinite(v)) return ORACLE_ERR_NONFINITE;
      if (periodic && (v < 0.0 || v >= L)) return ORACLE_ERR_OUT_OF_BOX;
    }
    if (w && !isfinite(w[i])) return ORACLE_ERR_NONFINITE;
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------------ entry */

/*
 * oracle_count: ordered pair counts of set 1 against set 2.
 *   mode      ORACLE_XI or ORACLE_WP
 *   autocorr  1: set 2 is set 1 and the pair (i, i) is skipped
 *   x1..w1    set 1 (host arrays of n1 doubles; w1 may be NULL: weight 1)
 *   x2..w2    set 2 (ignored when autocorr)
 *   periodic  1: cube [0, L)^3 with minimum-image separations
 *   edges     nedges >= 2 strictly increasing separation edges, edges[0] >= 0
 *   pimax, npibins   pi binning (wp only)
 *   use_grid  0: all pairs (Code 1), 1: chaining mesh (Section 1.2)
 *   nthreads  OpenMP threads (<= 0: runtime default)
 * Outputs (nout = (nedges-1) * (wp ? npibins : 1) entries, separation-major):
 *   npairs    counts; wsum = sum of w_i w_j; wrsum = sum of w_i w_j sqrt(sep^2)
 *             (wsum / wrsum may be NULL)
 */
int oracle_count(int mode, int autocorr,
                 int64_t n1, const double *x1, const double *y1, const double *z1,
                 const double *w1,
                 int64_t n2, const double *x2, const double *y2, const double *z2,
                 const double *w2,
                 int periodic, double L,
                 const double *edges, int nedges, double pimax, int npibins,
                 int use_grid, int nthreads,
                 uint64_t *npairs, double *wsum, double *wrsum) {
  if (mode != ORACLE_XI && mode != ORACLE_WP) return ORACLE_ERR_ARG;
  if (nedges < 2 || !edges || !npairs || n1 < 0) return ORACLE_ERR_ARG;
  for (int k = 0; k < nedges; k++)
    if (!isfinite(edges[k]) || (k > 0 && !(edges[k] > edges[k - 1])))
      return ORACLE_ERR_ARG;
  if (edges[0] < 0) return ORACLE_ERR_ARG;
  if (mode == ORACLE_WP && (!(pimax > 0) || !isfinite(pimax) || npibins < 1))
    return ORACLE_ERR_ARG;
  if (periodic && (!(L > 0) || !isfinite(L))) return ORACLE_ERR_ARG;
  if (autocorr) {
    n2 = n1; x2 = x1; y2 = y1; z2 = z1; w2 = w1;
  } else if (n2 < 0) {
    return ORACLE_ERR_ARG;
  }
  int rc = check_points(n1, x1, y1, z1, w1, periodic, L);
  if (rc == ORACLE_OK && !autocorr) rc = check_points(n2, x2, y2, z2, w2, periodic, L);
  if (rc != ORACLE_OK) return rc;

  pair_rule R;
  R.mode = mode;
  R.periodic = periodic;
  R.L = L;
  R.halfL = 0.5 * L;
  R.nbins = nedges - 1;
  double *E = (double *)malloc(sizeof(double) * (size_t)nedges);
  int npi = mode == ORACLE_WP ? npibins : 1;
  double *q = (double *)malloc(sizeof(double) * (size_t)(npi + 1));
  if (!E || !q) { free(E); free(q); return ORACLE_ERR_NOMEM; }
  for (int k = 0; k < nedges; k++) E[k] = edges[k] * edges[k];
  R.E = E;
  R.pimax = pimax;
  R.npibins = npi;
  if (mode == ORACLE_WP) {
    double dpi = pimax / npibins;
    q[0] = 0.0;
    for (int l = 1; l < npibins; l++) q[l] = (double)l * dpi;
    q[npibins] = pimax;
  } else {
    q[0] = 0.0;
    q[1] = 0.0;
  }
  R.q = q;
  R.nout = R.nbins * npi;

  int nt = 1;
#ifdef _OPENMP
  nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  size_t nout = (size_t)R.nout;
  uint64_t *cnt = (uint64_t *)calloc(nout * (size_t)nt, sizeof(uint64_t));
  nsum *sw = (nsum *)calloc(nout * (size_t)nt, sizeof(nsum));
  nsum *swr = (nsum *)calloc(nout * (size_t)nt, sizeof(nsum));
  if (!cnt || !sw || !swr) {
    free(E); free(q); free(cnt); free(sw); free(swr);
    return ORACLE_ERR_NOMEM;
  }

  cellgrid G;
  memset(&G, 0, sizeof(G));
  if (use_grid) {
    double lo[3], ext[3], reach[3];
    const double *pa1[3] = {x1, y1, z1}, *pa2[3] = {x2, y2, z2};
    for (int a = 0; a < 3; a++) {
      if (periodic) {
        lo[a] = 0.0;
        ext[a] = L;
      } else {
        double mn = INFINITY, mx = -INFINITY;
        for (int64_t i = 0; i < n1; i++) { mn = fmin(mn, pa1[a][i]); mx = fmax(mx, pa1[a][i]); }
        for (int64_t i = 0; i < n2; i++) { mn = fmin(mn, pa2[a][i]); mx = fmax(mx, pa2[a][i]); }
        if (!(mx >= mn)) { mn = 0; mx = 0; }
        lo[a] = mn;
        ext[a] = mx - mn;
      }
      reach[a] = edges[nedges - 1];
    }
    if (mode == ORACLE_WP) reach[2] = pimax;
    rc = grid_build(&G, n2, x2, y2, z2, lo, ext, reach);
    if (rc != ORACLE_OK) {
      free(E); free(q); free(cnt); free(sw); free(swr);
      return rc;
    }
  }

#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    accum A;
    A.cnt = cnt + nout * (size_t)t;
    A.w = sw + nout * (size_t)t;
    A.wr = swr + nout * (size_t)t;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n1; i++) {
      double xi = x1[i], yi = y1[i], zi = z1[i];
      double wi = w1 ? w1[i] : 1.0;
      if (!use_grid) {
        for (int64_t j = 0; j < n2; j++) {
          if (autocorr && j == i) continue;
          double sq;
          int slot = eval_pair(&R, xi, yi, zi, x2[j], y2[j], z2[j], &sq);
          if (slot < 0) continue;
          accum_pair(&A, slot, wi * (w2 ? w2[j] : 1.0), sq);
        }
      } else {
        int cx[3], cy[3], cz[3];
        int mx = axis_neighbours(cell_of(&G, 0, xi), G.n[0], periodic, cx);
        int my = axis_neighbours(cell_of(&G, 1, yi), G.n[1], periodic, cy);
        int mz = axis_neighbours(cell_of(&G, 2, zi), G.n[2], periodic, cz);
        for (int a = 0; a < mx; a++)
          for (int b = 0; b < my; b++)
            for (int c = 0; c < mz; c++) {
              int64_t cell = ((int64_t)cx[a] * G.n[1] + cy[b]) * G.n[2] + cz[c];
              for (int64_t m = G.start[cell]; m < G.start[cell + 1]; m++) {
                int64_t j = G.idx[m];
                if (autocorr && j == i) continue;
                double sq;
                int slot = eval_pair(&R, xi, yi, zi, x2[j], y2[j], z2[j], &sq);
                if (slot < 0) continue;
                accum_pair(&A, slot, wi * (w2 ? w2[j] : 1.0), sq);
              }
            }
      }
    }
  }

  for (size_t s = 0; s < nout; s++) {
    uint64_t c = 0;
    nsum tw = {0, 0}, twr = {0, 0};
    for (int t = 0; t < nt; t++) {
      size_t o = nout * (size_t)t + s;
      c += cnt[o];
      nsum_add(&tw, sw[o].sum);
      nsum_add(&tw, sw[o].comp);
      nsum_add(&twr, swr[o].sum);
      nsum_add(&twr, swr[o].comp);
    }
    npairs[s] = c;
    if (wsum) wsum[s] = tw.sum + tw.comp;
    if (wrsum) wrsum[s] = twr.sum + twr.comp;
  }
  if (use_grid) grid_free(&G);
  free(E); free(q); free(cnt); free(sw); free(swr);
  return ORACLE_OK;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
