// Host side of libcountpairs: argument checks, grid geometry, the binary32
// error bound and decision tables, device scratch, kernel launches and the
// C ABI declared in include/countpairs.h.
#include "cp_internal.h"
#include "../../include/countpairs.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace cp {

// kernels (grid_kernels.hip, pair_kernels.hip)
__global__ void k_bbox_partial(PointsDev a, PointsDev b, double *out, int *err);
__global__ void k_bbox_final(const double *part, int nblk, double *out);
__global__ void k_fill_i32(int *p, int64_t n, int v);
__global__ void k_fill2_i32(int *a, int64_t na, int *b, int64_t nb);
__global__ void k_colcount(const PointsDev *pts, const GridGeom *geom, int *mat, int *err);
__global__ void k_colscatter(const PointsDev *pts, const GridGeom *geom, const int *off,
                             double4 *out);
__global__ void k_colcells(const GridGeom *geom, const int *off, const double4 *colgrp,
                           double4 *grp, int *cstart, const int *maxspan,
                           const int64_t *col_prefix, int *colcnt);
__global__ void k_fill_u64(unsigned long long *p, int64_t n);
__global__ void k_fill_f64(double *p, int64_t n);
__global__ void k_scan_sums(const int *in, const ScanSeg *segs, int nseg, int *tsum);
__global__ void k_scan_apply(const int *in, int *out, const ScanSeg *segs, int nseg,
                             const int *tsum);
__global__ void k_assign(const PointsDev *pts, const GridGeom *geom, int *cell_count, int *cid,
                         int *rank, int *err);
__global__ void k_group(const PointsDev *pts, const GridGeom *geom, const int *cstart,
                        const int *cid, const int *rank, double4 *grp);
__global__ void k_cellsort(const GridGeom *geom, int nmock, const int *cstart, const double4 *grp,
                           double4 *pos, float4 *strm, CellBox *cbox, const int64_t *win_prefix,
                           int mode);
__global__ void k_tiles(const GridGeom *geom, int nmock, const int *cstart, const int *maxspan,
                        const int64_t *col_prefix, int *colcnt, const int *coloff, Tile *tiles,
                        int emit);
template <int MODE, int PREC, int W> __global__ void k_pairs(PairParams P);


// ------------------------------------------------------------ error state

constexpr int kMaxDevices = 64;   // devices whose per-device state the library keeps

static thread_local std::string g_err;
static thread_local cp_stats g_stats;
static thread_local bool g_stats_valid = false;

static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

// error reporting for the host-only entry points in other files
int report_error(int code, const char *msg) { return fail(code, msg); }

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(CP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// --------------------------------------------------------- rounding helpers

static float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -INFINITY);
  return f;
}
static float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}
static uint32_t fbits(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}
static float bitsf(uint32_t b) {
  float f;
  memcpy(&f, &b, 4);
  return f;
}

// ----------------------------------------------------------- decision table
//
// Each edge E_k has an uncertain band [C_k, A_k) of binary32 estimates v:
// v < C_k proves s < E_k and v >= A_k proves s >= E_k.  The table is indexed
// by (bits(v) >> shift) clamped to [lo, hi]; entry = (t_lo, t_hi | kup):
//   slot = kup - 1 + (v >= t_hi),  uncertain = (v >= t_lo) && !(v >= t_hi),
// where slot counts the edges certainly below v (0 = below E_0, nb + 1 =
// at or above E_nb).  A cell holding more than one band boundary is marked
// uncertain as a whole, which is always safe.

// A fixed-capacity array: the binning set-up of a call runs without heap
// allocation (the entry point without allocation relies on it).
template <class T, int N> struct Fixed {
  T v[N];
  int n = 0;
  void assign(int m, const T &x) {
    n = m;
    for (int i = 0; i < m; i++) v[i] = x;
  }
  void resize(int m) { n = m; }
  int size() const { return n; }
  bool empty() const { return n == 0; }
  T *data() { return v; }
  const T *data() const { return v; }
  T &operator[](int i) { return v[i]; }
  const T &operator[](int i) const { return v[i]; }
};

constexpr int kTabMax = 4096;   // decision-table cells

struct Table {
  Fixed<uint2, kTabMax> e;
  int lo = 0, hi = 0;
};
using EdgeF = Fixed<float, kMaxBins + 1>;
using EdgeD = Fixed<double, kMaxBins + 1>;

static const uint32_t kBig = 0x7E000000u;     // ~4.25e37, finite
static const float kNegBig = -3.0e38f;

static uint32_t hi_with_k(float z, int k) {
  uint32_t b = fbits(z);
  uint32_t b2 = (b & ~63u) | (uint32_t)k;
  if (b2 < b) b2 += 64;
  return b2;
}

static bool build_table(const EdgeF &C, const EdgeF &Av, int shift, Table &T) {
  const int nt = C.size();  // nb + 1 thresholds
  // merged uncertain zones
  struct Z {
    float lo, hi;
  };
  Fixed<Z, kMaxBins + 1> zones;
  for (int k = 0; k < nt; k++) {
    if (!(Av[k] > C[k])) continue;
    if (!zones.empty() && C[k] <= zones[zones.n - 1].hi)
      zones[zones.n - 1].hi = std::max(zones[zones.n - 1].hi, Av[k]);
    else
      zones[zones.n++] = {C[k], Av[k]};
  }
  auto sigma = [&](float v) {
    int s = 0;
    for (int k = 0; k < nt; k++) s += (Av[k] <= v);
    return s;
  };
  auto cell_of = [&](float v) { return (int)((int32_t)fbits(v) >> shift); };
  float minpos = INFINITY;
  for (int k = 0; k < nt; k++) {
    if (C[k] > 0) minpos = std::min(minpos, C[k]);
    if (Av[k] > 0) minpos = std::min(minpos, Av[k]);
  }
  if (!std::isfinite(minpos)) minpos = Av[nt - 1];
  T.lo = cell_of(minpos);
  T.hi = std::max(T.lo, cell_of(Av[nt - 1]));
  if (T.hi - T.lo + 1 > kTabMax) return false;
  T.e.assign(T.hi - T.lo + 1, make_uint2(0, 0));
  for (int m = T.lo; m <= T.hi; m++) {
    const float vlo = m == T.lo ? -INFINITY : bitsf((uint32_t)m << shift);
    const float vhi = m == T.hi ? INFINITY : bitsf((uint32_t)(m + 1) << shift);
    int nin = 0;          // zones meeting this cell, and the first of them
    Z first{0.f, 0.f};
    for (int q = 0; q < zones.size(); q++)
      if (zones[q].hi > vlo && zones[q].lo < vhi) {
        if (!nin) first = zones[q];
        nin++;
      }
    uint2 ent;
    const uint2 all_unc = make_uint2(fbits(kNegBig), kBig | 1u);
    if (nin == 0) {
      const float rep = m == T.lo ? bitsf((uint32_t)m << shift) : vlo;
      const int s = sigma(rep);
      ent = make_uint2(kBig, kBig | (uint32_t)(s + 1));
    } else if (nin > 1) {
      ent = all_unc;
    } else {
      const Z z = first;
      const bool sin = z.lo > vlo, ein = z.hi < vhi;
      if (!sin && !ein) {
        ent = all_unc;
      } else if (!sin && ein) {
        const int sh = sigma(z.hi);
        ent = make_uint2(fbits(kNegBig), hi_with_k(z.hi, sh));
      } else if (sin && !ein) {
        const int sl = sigma(std::nextafter(z.lo, -INFINITY));
        ent = make_uint2(fbits(z.lo), kBig | (uint32_t)(sl + 1));
      } else {
        const int sl = sigma(std::nextafter(z.lo, -INFINITY));
        const int sh = sigma(z.hi);
        if (sh == sl + 1)
          ent = make_uint2(fbits(z.lo), hi_with_k(z.hi, sh));
        else
          ent = all_unc;
      }
    }
    T.e[m - T.lo] = ent;
  }
  return true;
}

// ---------------------------------------------------------------- geometry

struct Geometry {
  int n[3], r[3], wrap[3];
  double lo[3], cs[3], ext[3];
  int maxspan;
  bool ok;
};

static Geometry choose_geometry(int mode, bool periodic, double box, const double lo[3],
                                const double ext[3], double rmax, double pimax,
                                const int refine_in[3], int64_t npts_total) {
  Geometry g;
  const double reach[3] = {rmax, rmax, mode == XI ? rmax : pimax};
  int refine[3];
  for (int a = 0; a < 3; a++) {
    // default: cells of R_max/2 on every axis (the paper's CPU default keeps
    // z at R_max because its z-sorted late entry prunes along z; here finer
    // z cells and the cell-level bounding-box test do that job)
    int dflt = 2;
    refine[a] = refine_in && refine_in[a] > 0 ? refine_in[a] : dflt;
    if (refine[a] > 8) refine[a] = 8;
  }
  for (int a = 0; a < 3; a++) {
    g.lo[a] = periodic ? 0.0 : lo[a];
    g.ext[a] = periodic ? box : ext[a];
    g.wrap[a] = 0;
    int ref = refine[a];
    int n = 1;
    if (g.ext[a] > 0) {
      for (;;) {
        double f = std::floor(g.ext[a] / (reach[a] / ref * (1.0 + 1e-9)));
        n = f < 1 ? 1 : (f > kMaxAxisCells ? kMaxAxisCells : (int)f);
        if (!periodic || ref <= 1 || n >= 2 * ref + 1) break;
        ref--;
      }
    }
    if (periodic && n < 2 * ref + 1) {
      // fewer than three cells per reach: one cell, per-pair minimum image
      n = 1;
      ref = 0;
      g.wrap[a] = 1;
    }
    if (!periodic && n == 1) ref = 0;
    g.n[a] = n;
    g.r[a] = ref;
  }
  // bound the cell count by the points (sparse data): coarsen the finest axis
  const int64_t cap = std::max<int64_t>(4096, 4 * npts_total);
  while ((int64_t)g.n[0] * g.n[1] * g.n[2] > cap) {
    int a = 0;
    for (int b = 1; b < 3; b++)
      if (g.n[b] > g.n[a]) a = b;
    int nn = std::max(1, (int)(g.n[a] * 0.8));
    if (periodic && nn < 2 * g.r[a] + 1) {
      // keep the no-aliasing condition: drop to one wrapped cell
      nn = 1;
      g.r[a] = 0;
      g.wrap[a] = 1;
    }
    if (!periodic && nn == 1) g.r[a] = 0;
    g.n[a] = nn;
  }
  for (int a = 0; a < 3; a++) g.cs[a] = g.ext[a] > 0 ? g.ext[a] / g.n[a] : 1.0;
  int span = std::max(2, 2 * g.r[2]);
  if (periodic && !g.wrap[2]) span = std::min(span, g.n[2] - 2 * g.r[2]);
  g.maxspan = std::max(1, span);
  g.ok = true;
  return g;
}

// Queue items of a tile.  The tile's neighbour columns are listed in a fixed
// order (the kernel decodes the same order): for an auto-count the half-shell
// of Section 2.1 taken geometrically -- the tile's own column first (searched
// forward in z only), then the columns at x offset 0 and y offset 1..r_y, then
// x offsets 1..r_x with every y offset; for a cross-count the whole
// (2 r_x + 1) x (2 r_y + 1) block.  Each cell pair of the box is met once
// because every periodic axis has at least 2 r + 1 cells or is a single
// wrapped cell.  The list is cut into consecutive chunks of about equal
// estimated cost, one queue item each, so that no item is much heavier than
// the rest: a column whose x-y gap to the tile's column is g costs about
// (1 - g^2 / R^2)^2 of an adjacent one (fitted to measured per-column times)
// and the own column 0.9.  A chunk aims at 4.5 sqrt(137 / c) adjacent columns,
// kept within [2.2, 12], where c is the expected number of searched points in
// one adjacent column's reach (density npts2 / box volume) times the cost
// factor (2 for binary64, 2 for weights, 2.5 for w_p): light items are
// dominated by the per-item set-up and want more columns, heavy ones want the
// finer split for the end of the queue (fitted to timings from R_max = 5 to
// 100).
static void split_columns(const Geometry &g, bool autoc, double reach, double reach_z,
                          double npts2, double cost, int chunk_pct, PairParams &P) {
  const int rx = g.r[0], ry = g.r[1], ncy = 2 * ry + 1;
  const int ncols = autoc ? 1 + ry + rx * ncy : (2 * rx + 1) * ncy;
  Fixed<double, (2 * 8 + 1) * (2 * 8 + 1) + 1> cum;   // columns + 1 at refine 8 per axis
  cum.assign(ncols + 1, 0.0);
  for (int c = 0; c < ncols; c++) {
    int ox, oy;
    if (autoc) {
      if (c <= ry) {
        ox = 0;
        oy = c;
      } else {
        ox = 1 + (c - 1 - ry) / ncy;
        oy = (c - 1 - ry) % ncy - ry;
      }
    } else {
      ox = c / ncy - rx;
      oy = c % ncy - ry;
    }
    double w;
    if (autoc && c == 0) {
      w = 0.9;
    } else {
      const double gx = std::max(std::abs(ox) - 1, 0) * g.cs[0];
      const double gy = std::max(std::abs(oy) - 1, 0) * g.cs[1];
      const double t = reach > 0 ? 1.0 - (gx * gx + gy * gy) / (reach * reach) : 1.0;
      w = std::max(t > 0 ? t * t : 0.0, 0.02);
    }
    cum[c + 1] = cum[c] + w;
  }
  const double tot = cum[ncols];
  const double vol = g.ext[0] * g.ext[1] * g.ext[2];
  double per = 2.2;
  if (vol > 0 && npts2 > 0) {
    const double c = npts2 / vol * g.cs[0] * g.cs[1] * (2.0 * reach_z + g.cs[2]) * cost;
    per = std::min(12.0, std::max(2.2, 4.5 * std::sqrt(137.0 / std::max(c, 1e-9))));
  }
  per *= chunk_pct * 0.01;   // the autotuner's scale of the target
  int m = (int)std::lround(tot / per);
  m = std::max(1, std::min(m, std::min(kMaxChunks, ncols)));
  P.nsplit = m;
  P.chunk[0] = 0;
  for (int k = 1; k < m; k++) {
    const double target = tot * k / m;
    int best = P.chunk[k - 1] + 1;
    for (int b = best; b <= ncols - (m - k); b++)
      if (std::fabs(cum[b] - target) < std::fabs(cum[best] - target)) best = b;
    P.chunk[k] = best;
  }
  P.chunk[m] = ncols;
}

static GridGeom to_dev_geom(const Geometry &g, bool periodic, double box, int64_t pbase,
                            int64_t cbase, int64_t sbase, int64_t npts, int64_t colbase) {
  GridGeom G;
  memset(&G, 0, sizeof(G));
  for (int a = 0; a < 3; a++) {
    G.n[a] = g.n[a];
    G.r[a] = g.r[a];
    G.wrap[a] = g.wrap[a];
    G.lo[a] = g.lo[a];
    G.cs[a] = g.cs[a];
    G.inv[a] = 1.0 / g.cs[a];
  }
  G.periodic = periodic ? 1 : 0;
  G.box = periodic ? box : 0.0;
  G.halfbox = 0.5 * G.box;
  G.pbase = pbase;
  G.cbase = cbase;
  G.sbase = sbase;
  G.npts = npts;
  G.ncell = g.n[0] * g.n[1] * g.n[2];
  G.ncol = g.n[0] * g.n[1];
  G.colbase = colbase;
  G.mbase = 0;
  G.nblk = col_blocks(npts);
  return G;
}

// ------------------------------------------------------ binary32 error bound

struct Bounds {
  double eps;        // |s~ - s| bound for the squared (projected) separation
  double eta_pi;     // |pi~ - pi| bound (wp)
};

static Bounds error_bounds(int mode, const Geometry &g, double EB, double pimax, double M) {
  const double u = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
  const double eB = std::sqrt(EB);
  Bounds b;
  if (mode == XI) {
    const double P =
        0.5 * std::sqrt(g.cs[0] * g.cs[0] + g.cs[1] * g.cs[1] + g.cs[2] * g.cs[2]) * (1 + 1e-6);
    const double G = 2 * P + eB;
    const double eta = u * G * 1.01 + 4 * std::sqrt(3.0) * u64 * M;
    b.eps = 2.0 * (7.5 * u * G * G + 2 * eB * eta + eta * eta + 8 * u64 * (EB + 2 * eB * M));
    b.eta_pi = 0;
  } else {
    const double P = 0.5 * std::sqrt(g.cs[0] * g.cs[0] + g.cs[1] * g.cs[1]) * (1 + 1e-6);
    const double G = 2 * P + eB;
    const double eta = u * G * 1.01 + 4 * std::sqrt(2.0) * u64 * M;
    b.eps = 2.0 * (5.5 * u * G * G + 2 * eB * eta + eta * eta + 8 * u64 * (EB + 2 * eB * M));
    const double Pz = 0.5 * g.cs[2] * (1 + 1e-6);
    b.eta_pi = 2.0 * (u * (2 * Pz + 2 * pimax) * 1.01 + 4 * u64 * M);
  }
  return b;
}

// ----------------------------------------------------------- device arena

struct Arena {
  void *base = nullptr;
  size_t cap = 0;
};
static thread_local Arena g_arena;

// Pinned host staging of the per-call upload and download, one buffer per
// thread, grown on demand and kept until the process ends (each call has
// synchronised its stream before it returns, so the next call may reuse it).
struct Pinned {
  char *p = nullptr;
  size_t cap = 0;
};
static thread_local Pinned g_pin;

static char *pinned_staging(size_t bytes) {
  if (g_pin.cap < bytes) {
    if (g_pin.p) (void)hipHostFree(g_pin.p);
    g_pin = Pinned();
    const size_t want = std::max<size_t>(bytes, (size_t)1 << 19);
    void *q = nullptr;
    if (hipHostMalloc(&q, want, hipHostMallocDefault) != hipSuccess) return nullptr;
    g_pin.p = (char *)q;
    g_pin.cap = want;
  }
  return g_pin.p;
}

struct Carver {
  char *p;
  size_t off = 0;
  bool dry;
  explicit Carver(void *b, bool d) : p((char *)b), dry(d) {}
  template <class T> T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *r = dry ? nullptr : (T *)(p + off);
    off += n * sizeof(T);
    return r;
  }
};

// Device buffers of one gridded point set.
struct SetBufs {
  int *ccount, *cstart, *cid, *rank, *colcnt, *coloff;
  int *tsum;            // tile totals of the segmented scans
  int *colmat;          // column x block counts of the LDS column grouping
  double4 *pos, *grp;   // grp: points grouped by cell before the z order
  float4 *strm;
  CellBox *cbox;
  Tile *tiles;
};

static void carve_set(Carver &cv, SetBufs &S, int64_t n, int64_t ncell, int64_t ncol,
                      bool want_tiles, int64_t maxtiles) {
  S.ccount = cv.take<int>(ncell * kCountStride);
  S.cstart = cv.take<int>(ncell + 1);
  const int64_t nmat = ncol <= kColLds ? ncol * kColBlocks : 0;
  S.tsum = cv.take<int>(std::max({scan_tiles(ncell), scan_tiles(ncol), scan_tiles(nmat)}));
  S.colmat = cv.take<int>(nmat + 1);
  S.cid = cv.take<int>(n > 0 ? n : 1);
  S.rank = cv.take<int>(n > 0 ? n : 1);
  // +8 records: the pair kernels prefetch scalar loads past a cell's end
  S.pos = cv.take<double4>(n + 8);
  S.grp = cv.take<double4>(n > 0 ? n : 1);
  S.strm = cv.take<float4>(n + 8);
  S.cbox = cv.take<CellBox>(ncell);
  // column counts and offsets: the column grouping of every set, the tile
  // queue of the tiled set
  S.colcnt = cv.take<int>(ncol + 1);
  S.coloff = cv.take<int>(ncol + 1);
  S.tiles = want_tiles ? cv.take<Tile>(maxtiles) : nullptr;
}

// Small per-call records uploaded in one copy.
struct Smalls {
  GridGeom geom[2];
  PointsDev pts[2];
  ScanSeg seg[4];   // cells, columns, column x block matrix of set 1 and of set 2
  int64_t win_prefix[2][2];   // z-order windows of set 1 and set 2
  int64_t col_prefix[2];
  int maxspan[2];
  int ntiles_dummy;
};

// Host staging sizes of one call: the small records and decision tables
// (tables of at most kTabMax cells each, 256-byte aligned pieces), and the
// histogram, weight sums, statistics and error flag.
constexpr size_t kUpMax = sizeof(Smalls) + 2 * 8 * kTabMax + 16 * (kMaxBins + 1) + 8 * 256;
constexpr size_t kDownMax = 3 * 8 * (size_t)kMaxBins * kMaxPiBins + 8 * kStatWords + 4 + 8 * 256;

struct Call {
  int mode;          // XI / WP
  bool cross;
  const cp_points *d1, *d2;
  const double *edges;
  int nedges;
  double pimax;
  int npi;
  const cp_options *o;
  // the entry point without allocation: its device scratch (the library's
  // static array) in place of the workspace or the thread's arena; such a
  // call creates no events and copies results straight into the outputs
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  // launch settings that refine = 0 leaves to the library (0: defaults)
  int chunk_pct = 0;
  int waves = 0;
};

static int check_points(const cp_points *p, const char *name) {
  if (!p) return fail(CP_ERR_INVALID_ARG, std::string(name) + " is NULL");
  if (p->n < 0) return fail(CP_ERR_INVALID_ARG, std::string(name) + "->n < 0");
  if (p->n > ((int64_t)1 << 31) - 1)
    return fail(CP_ERR_INVALID_ARG, std::string(name) + "->n above 2^31 - 1");
  if (p->dtype != CP_F64 && p->dtype != CP_F32)
    return fail(CP_ERR_INVALID_ARG, std::string(name) + "->dtype must be CP_F64 or CP_F32");
  if (p->n > 0 && (!p->x || !p->y || !p->z))
    return fail(CP_ERR_INVALID_ARG, std::string(name) + " has NULL coordinates");
  return CP_OK;
}

static int check_common(const Call &c) {
  if (!c.o) return fail(CP_ERR_INVALID_ARG, "options is NULL");
  const cp_options &o = *c.o;
  if (!c.edges || c.nedges < 2) return fail(CP_ERR_INVALID_ARG, "need nedges >= 2 edges");
  if (c.nedges - 1 > kMaxBins)
    return fail(CP_ERR_INVALID_ARG, "at most " + std::to_string(kMaxBins) + " bins");
  for (int k = 0; k < c.nedges; k++) {
    if (!std::isfinite(c.edges[k])) return fail(CP_ERR_INVALID_ARG, "non-finite edge");
    if (k > 0 && !(c.edges[k] > c.edges[k - 1]))
      return fail(CP_ERR_INVALID_ARG, "edges must increase strictly");
  }
  if (c.edges[0] < 0) return fail(CP_ERR_INVALID_ARG, "edges[0] < 0");
  if (c.mode == WP) {
    if (!(c.pimax > 0) || !std::isfinite(c.pimax))
      return fail(CP_ERR_INVALID_ARG, "pimax must be positive and finite");
    if (c.npi < 1 || c.npi > kMaxPiBins)
      return fail(CP_ERR_INVALID_ARG, "npibins must be in [1, " + std::to_string(kMaxPiBins) + "]");
  }
  if (o.precision != CP_PREC_FP64 && o.precision != CP_PREC_FP32_RECHECK)
    return fail(CP_ERR_INVALID_ARG, "bad precision");
  if (o.count_mode != CP_ORDERED && o.count_mode != CP_UNIQUE)
    return fail(CP_ERR_INVALID_ARG, "bad count_mode");
  if (o.no_prune != 0 && o.no_prune != 1) return fail(CP_ERR_INVALID_ARG, "no_prune must be 0 or 1");
  if (o.periodic && (!(o.boxsize > 0) || !std::isfinite(o.boxsize)))
    return fail(CP_ERR_INVALID_ARG, "periodic needs a positive finite boxsize");
  for (int a = 0; a < 3; a++)
    if (o.refine[a] < 0) return fail(CP_ERR_INVALID_ARG, "refine must be >= 0");
  if (o.workspace && !o.workspace_bytes)
    return fail(CP_ERR_INVALID_ARG, "workspace given with zero size");
  return CP_OK;
}

static int64_t max_tiles_bound(int64_t n, int64_t ncell, int64_t ncol) {
  return ncell + n / kTileMax + ncol + 1;
}

// Launch the cell build of one point set (cell counts .. tiles).
static int launch_build(hipStream_t st, const PointsDev *d_pts, const GridGeom *d_geom,
                        const SetBufs &S, int64_t n, int64_t ncell, int64_t ncol, int mode,
                        const ScanSeg *d_seg_cells, const ScanSeg *d_seg_cols,
                        const ScanSeg *d_seg_mat,
                        const int64_t *d_win_prefix, const int64_t *d_col_prefix,
                        const int *d_maxspan, int *d_err, bool tiles, int *zero = nullptr,
                        int64_t zero_words = 0) {
  (void)hipGetLastError();
  const char *ce = getenv("CP_BUILD_COLUMNS");
  bool counted = false;   // the columns' tile counts are in colcnt already
  if (n > 0 && ncol <= kColLds && !(ce && ce[0] == '0')) {
    // grouping through LDS column histograms: the column x block counts in
    // colmat (scanned in place), column order in pos before the z pass
    // overwrites it; the per-column pass also counts the column's tiles
    if (zero_words)
      hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((zero_words + 255) / 256, 64)),
                         dim3(256), 0, st, zero, zero_words, 0);
    const int nb1 = col_blocks(n);
    hipLaunchKernelGGL(k_colcount, dim3(nb1), dim3(1024), 0, st, d_pts, d_geom, S.colmat, d_err);
    const unsigned tm = (unsigned)scan_tiles(ncol * nb1);
    if (tm > 1)
      hipLaunchKernelGGL(k_scan_sums, dim3(tm), dim3(256), 0, st, S.colmat, d_seg_mat, 1, S.tsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(tm), dim3(256), 0, st, S.colmat, S.colmat, d_seg_mat, 1,
                       S.tsum);
    hipLaunchKernelGGL(k_colscatter, dim3(nb1), dim3(1024), 0, st, d_pts, d_geom, S.colmat, S.pos);
    hipLaunchKernelGGL(k_colcells, dim3((unsigned)std::min<int64_t>(ncol, 8192)), dim3(256), 0, st,
                       d_geom, S.colmat, S.pos, S.grp, S.cstart, d_maxspan, d_col_prefix,
                       tiles ? S.colcnt : nullptr);
    counted = tiles;
  } else {
    // the cell counters (and the caller's extra range) cleared by one launch
    const int64_t nfill = ncell * kCountStride;
    const int fb =
        (int)std::min<int64_t>(std::max<int64_t>((nfill + zero_words + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(k_fill2_i32, dim3(fb), dim3(256), 0, st, S.ccount, nfill, zero, zero_words);
    const int ab = (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 8192);
    if (n > 0)
      hipLaunchKernelGGL(k_assign, dim3(ab, 1), dim3(256), 0, st, d_pts, d_geom, S.ccount, S.cid,
                         S.rank, d_err);
    const unsigned sc = (unsigned)scan_tiles(ncell);
    if (sc > 1)   // a single tile needs no tile totals
      hipLaunchKernelGGL(k_scan_sums, dim3(sc), dim3(256), 0, st, S.ccount, d_seg_cells, 1, S.tsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(sc), dim3(256), 0, st, S.ccount, S.cstart, d_seg_cells, 1,
                       S.tsum);
    if (n > 0)
      hipLaunchKernelGGL(k_group, dim3(ab, 1), dim3(256), 0, st, d_pts, d_geom, S.cstart, S.cid,
                         S.rank, S.grp);
  }
  const int64_t nwin = (n + kSortWin - 1) / kSortWin;
  const int cb = (int)std::min<int64_t>(std::max<int64_t>((nwin + 3) / 4, 1), 16384);
  if (n > 0)
    hipLaunchKernelGGL(k_cellsort, dim3(cb), dim3(256), 0, st, d_geom, 1, S.cstart, S.grp, S.pos,
                       S.strm, S.cbox, d_win_prefix, mode);
  if (tiles) {
    const int tb = (int)std::min<int64_t>(std::max<int64_t>((ncol + 3) / 4, 1), 16384);
    if (!counted)
      hipLaunchKernelGGL(k_tiles, dim3(tb), dim3(256), 0, st, d_geom, 1, S.cstart, d_maxspan,
                         d_col_prefix, S.colcnt, S.coloff, S.tiles, 0);
    const unsigned tc = (unsigned)scan_tiles(ncol);
    if (tc > 1)
      hipLaunchKernelGGL(k_scan_sums, dim3(tc), dim3(256), 0, st, S.colcnt, d_seg_cols, 1, S.tsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(tc), dim3(256), 0, st, S.colcnt, S.coloff, d_seg_cols,
                       1, S.tsum);
    hipLaunchKernelGGL(k_tiles, dim3(tb), dim3(256), 0, st, d_geom, 1, S.cstart, d_maxspan,
                       d_col_prefix, S.colcnt, S.coloff, S.tiles, 1);
  }
  return hipGetLastError() == hipSuccess ? CP_OK : fail(CP_ERR_DEVICE, "cell build launch failed");
}

static int g_num_cus = 0;
static int num_cus() {
  if (!g_num_cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) g_num_cus = p.multiProcessorCount;
    if (g_num_cus <= 0) g_num_cus = 256;
  }
  return g_num_cus;
}

// Waves per pair-kernel workgroup: four, or fewer when the per-wave
// histograms (w_p with many bins, weighted) would not fit the 160 KB of LDS;
// 0 when not even one wave's fits.
// Copies of the w_p wave histogram: the tile's points are z-neighbours of
// one column, so for one streamed point most lanes add to the same few
// (r_p, pi) counters and their LDS atomics serialise; lane l adds to copy
// l mod wpc, the copies of a counter in adjacent words.  The most copies
// (up to 8) that still leave room for five 4-wave workgroups per CU (the
// pair kernel's register-bound occupancy); CP_WP_COPIES (1, 2, 4 or 8)
// overrides the choice.
static int wp_copies(int mode, int prec, int weighted, int n32, int n64, int nb, int npi,
                     int nx = 0, int nbx = 0) {
  if (mode != WP && mode != WPXI) return 1;
  if (const char *e = getenv("CP_WP_COPIES")) {
    const int c = atoi(e);
    if (c == 1 || c == 2 || c == 4 || c == 8) return c;
  }
  for (int c = 8; c > 1; c >>= 1) {
    const LdsLayout L = lds_layout(mode, prec, weighted, n32, n64, nb, npi, c, nx, nbx);
    if (L.common + 4 * L.wave_bytes + kStaticLds <= (size_t)160 * 1024 / 5) return c;
  }
  return 1;
}

static int pick_waves(const LdsLayout &LY, size_t *lds, int most = 4) {
  for (int nw = std::min(4, std::max(1, most)); nw >= 1; nw--) {
    const size_t l = LY.common + (size_t)nw * LY.wave_bytes;
    if (l + kStaticLds <= 160 * 1024) {
      *lds = l;
      return nw;
    }
  }
  return 0;
}

template <int MODE, int PREC, int W>
static int launch_pairs_t(hipStream_t st, const PairParams &P, size_t lds, int nwaves) {
  auto kern = k_pairs<MODE, PREC, W>;
  static thread_local size_t set_lds = 0;
  if (lds > 65536 && lds > set_lds) {
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return fail(CP_ERR_DEVICE, "cannot raise the LDS limit of the pair kernel");
    set_lds = lds;
  }
  // exactly the workgroups the CUs hold at once (registers, LDS and waves, as
  // the runtime computes them for this kernel): a surplus would only start
  // once the queues were drained and then probe every queue head, adding
  // device-scope atomics to the end of the launch
  static thread_local size_t occ_lds = ~(size_t)0;
  static thread_local int occ_nw = 0, occ_per_cu = 0;
  if (occ_lds != lds || occ_nw != nwaves) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 64 * nwaves, lds) != hipSuccess ||
        n < 1)
      n = std::max(1, std::min(8, (int)(160 * 1024 / std::max<size_t>(lds, 1))));
    occ_lds = lds;
    occ_nw = nwaves;
    occ_per_cu = n;
  }
  const int grid = num_cus() * occ_per_cu;
  (void)hipGetLastError();  // drop any stale error so the check below is about this launch
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * nwaves), lds, st, P);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CP_OK
                         : fail(CP_ERR_DEVICE, std::string("pair launch failed: ") +
                                                   hipGetErrorString(e));
}

static int launch_pairs(hipStream_t st, int mode, int prec, int w, const PairParams &P,
                        size_t lds, int nwaves) {
  if (mode == WPXI) {
    if (prec != F32R || w) return fail(CP_ERR_INTERNAL, "fused w_p + xi is binary32, unweighted");
    return launch_pairs_t<WPXI, F32R, 0>(st, P, lds, nwaves);
  }
  if (mode == XI) {
    if (prec == F32R)
      return w ? launch_pairs_t<XI, F32R, 1>(st, P, lds, nwaves)
               : launch_pairs_t<XI, F32R, 0>(st, P, lds, nwaves);
    return w ? launch_pairs_t<XI, F64, 1>(st, P, lds, nwaves)
             : launch_pairs_t<XI, F64, 0>(st, P, lds, nwaves);
  }
  if (prec == F32R) return w ? launch_pairs_t<WP, F32R, 1>(st, P, lds, nwaves)
                             : launch_pairs_t<WP, F32R, 0>(st, P, lds, nwaves);
  return w ? launch_pairs_t<WP, F64, 1>(st, P, lds, nwaves)
           : launch_pairs_t<WP, F64, 0>(st, P, lds, nwaves);
}

// Binning setup shared by single calls and plans.
struct Binning {
  EdgeD E;
  EdgeF C32, A32;
  Table t32, t64;
  int shift;
  float AB32;
  float eps32, eps32_3;
  Bounds bnd;
  float inv_dpi32, pi_delta, pi_hi32, pi_delta64;
  double dpi;
};

static int make_binning(int mode, int prec, const double *edges, int nedges, double pimax,
                        int npi, const Geometry &g, double M, Binning &B) {
  const int nb = nedges - 1;
  B.E.resize(nedges);
  for (int k = 0; k < nedges; k++) B.E[k] = edges[k] * edges[k];
  const double EB = B.E[nb];
  B.bnd = error_bounds(mode, g, EB, pimax, M);
  EdgeF C32, A32, C64, A64;
  C32.resize(nedges);
  A32.resize(nedges);
  C64.resize(nedges);
  A64.resize(nedges);
  for (int k = 0; k < nedges; k++) {
    const double e = B.E[k];
    if (e == 0.0) {
      C32[k] = A32[k] = C64[k] = A64[k] = -FLT_MAX;   // s >= 0 = E_0 always
      continue;
    }
    C32[k] = f32_down(e - B.bnd.eps);
    A32[k] = f32_up(e + B.bnd.eps);
    C64[k] = f32_down(e * (1.0 - std::ldexp(1.0, -22)));
    A64[k] = f32_up(e * (1.0 + std::ldexp(1.0, -22)));
  }
  for (int shift = 18; shift <= 23; shift++) {
    bool ok = build_table(C64, A64, shift, B.t64);
    if (ok && prec == F32R) ok = build_table(C32, A32, shift, B.t32);
    if (ok) {
      B.shift = shift;
      break;
    }
    if (shift == 23) return fail(CP_ERR_INVALID_ARG, "edges span too many octaves");
  }
  if (prec != F32R) B.t32 = B.t64;
  B.AB32 = A32[nb];
  B.eps32 = f32_up(B.bnd.eps);
  B.eps32_3 = f32_up(B.bnd.eps + 2.0 * std::ldexp(1.0, -24) * EB * 1.01);
  B.C32 = C32;
  B.A32 = A32;
  B.dpi = mode == WP ? pimax / npi : 1.0;
  if (mode == WP) {
    const double u = std::ldexp(1.0, -24);
    B.inv_dpi32 = (float)(1.0 / B.dpi);
    // pi band, in units of dpi: the estimate's error eta_pi, the roundings of
    // fl32(1 / dpi) and of the product (2u of at most npi + 1), the rounding
    // of the pre-filter pi_hi32 and of fl32(1 - pi_delta), and the binary64
    // edges; it also covers pi_max itself, whose edge is the integer npi, so
    // a pair away from every integer is surely below pi_max
    B.pi_delta = (float)(B.bnd.eta_pi / B.dpi + 8 * u * npi + 1e-12 * npi);
    // the binary64 loops bin fl32(|dz|) of the binary64 |dz| < pi_max the
    // same way: its error is at most u |dz| < u pi_max (1.01 for margin)
    B.pi_delta64 = (float)(1.01 * u * pimax / B.dpi + 8 * u * npi + 1e-12 * npi);
    B.pi_hi32 = f32_up(pimax + B.bnd.eta_pi);
  } else {
    B.inv_dpi32 = 1.0f;
    B.pi_delta = B.pi_delta64 = 0.f;
    B.pi_hi32 = 0.f;
  }
  return CP_OK;
}

// Binning of xi inside a fused w_p + xi launch.  The kernel forms the xi
// estimate s~ = fl32(pi~ * pi~ + v~) from the w_p estimates: v~ of r_p^2
// (error at most eps of the w_p bound) and pi~ of |dz| (error at most
// eta_pi).  Against the binary64 reference s = fl(fl(dx^2 + dy^2) + fl(dz^2)):
//   |s~ - s| <= u32 (pi~^2 + v~) + (pi~ + |dz|) eta_pi + eps + 2 u64 s.
// A decision is only taken for s~ < AB32x = up(E_B + bound), where pi~ and
// |dz| are at most Z = sqrt(E_B + bound + eps) + eta_pi; the bound and Z are
// iterated to a fixed point, and twice the bound makes the bands.  Returns
// false (no fusion) when the bound is not small against E_B.
static bool make_binning_wpxi(const double *edges, int nedges, const Binning &Bw, Binning &Bx) {
  const int nb = nedges - 1;
  Bx.E.resize(nedges);
  for (int k = 0; k < nedges; k++) Bx.E[k] = edges[k] * edges[k];
  const double EB = Bx.E[nb];
  const double u = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
  const double eta = Bw.bnd.eta_pi, epsw = Bw.bnd.eps;
  double bound = 0.0;
  for (int it = 0; it < 4; it++) {
    const double Z = std::sqrt(EB + bound + epsw) * (1.0 + 1e-6) + eta;
    bound = 2.0 * (u * 1.01 * (Z * Z + EB + bound + epsw) + 2.0 * Z * eta + epsw +
                   2.0 * u64 * 1.01 * (EB + bound));
  }
  if (!(bound < 0.25 * EB)) return false;
  Bx.bnd = Bw.bnd;
  Bx.bnd.eps = bound;
  EdgeF C, A;
  C.resize(nedges);
  A.resize(nedges);
  for (int k = 0; k < nedges; k++) {
    const double e = Bx.E[k];
    if (e == 0.0) {
      C[k] = A[k] = -FLT_MAX;
      continue;
    }
    C[k] = f32_down(e - bound);
    A[k] = f32_up(e + bound);
  }
  bool ok = false;
  for (int shift = 18; shift <= 23 && !ok; shift++) {
    ok = build_table(C, A, shift, Bx.t32);
    if (ok) Bx.shift = shift;
  }
  if (!ok) return false;
  Bx.AB32 = A[nb];
  Bx.C32 = C;
  Bx.A32 = A;
  return true;
}

// The binning of the last call on this thread, reused while its inputs are
// unchanged (the tables cost ~10 us to build; repeated calls on one
// configuration are the common case).  run() takes the reference after any
// tuning runs, so no nested call replaces it while it is in use.
struct BinningKey {
  int mode = -1, prec = -1, nedges = 0, npi = 0;
  double pimax = 0, M = 0, cs[3] = {0, 0, 0};
  Fixed<double, kMaxBins + 1> edges;
  bool operator==(const BinningKey &k) const {
    if (mode != k.mode || prec != k.prec || nedges != k.nedges || npi != k.npi ||
        pimax != k.pimax || M != k.M || cs[0] != k.cs[0] || cs[1] != k.cs[1] || cs[2] != k.cs[2])
      return false;
    for (int i = 0; i < nedges; i++)
      if (edges[i] != k.edges[i]) return false;
    return true;
  }
};
static thread_local BinningKey g_bin_key;
static thread_local Binning g_bin;

static int cached_binning(int mode, int prec, const double *edges, int nedges, double pimax,
                          int npi, const Geometry &g, double M, const Binning *&out) {
  BinningKey k;
  k.mode = mode;
  k.prec = prec;
  k.nedges = nedges;
  k.npi = npi;
  k.pimax = pimax;
  k.M = M;
  for (int a = 0; a < 3; a++) k.cs[a] = g.cs[a];
  k.edges.assign(nedges, 0.0);
  for (int i = 0; i < nedges; i++) k.edges[i] = edges[i];
  if (!(k == g_bin_key)) {
    g_bin_key = BinningKey();   // invalid until the tables are built
    const int rc = make_binning(mode, prec, edges, nedges, pimax, npi, g, M, g_bin);
    if (rc) return rc;
    g_bin_key = k;
  }
  out = &g_bin;
  return CP_OK;
}

static int map_err_flags(int flags) {
  if (flags & 1) return fail(CP_ERR_NONFINITE, "non-finite coordinate or weight");
  if (flags & 2) return fail(CP_ERR_OUT_OF_BOX, "periodic coordinate outside [0, boxsize)");
  return CP_OK;
}

// ------------------------------------------------------------- autotuning
//
// refine = 0 on every axis leaves the launch settings to the library
// (Section 3.1: the run time varies by up to 50 % with the refine factors,
// whose automatic choice the paper names as future work).  Candidates are
// timed on the call's own data -- device time of whole calls, best of three --
// by coordinate descent: the refine factors first, then the work-chunk
// target of the queue items, then the waves per workgroup; the winner is
// cached per workload signature (tune_cache.cpp).  CP_AUTOTUNE=0 switches
// tuning off (library defaults).

static const int kRefineCands[][3] = {{2, 2, 2}, {2, 2, 1}, {2, 2, 3}, {3, 3, 2},
                                      {3, 3, 3}, {1, 1, 1}, {4, 4, 3}};
static const int kChunkCands[] = {70, 140};
static const int kWaveCands[] = {2};

static bool autotune_on() {
  const char *e = getenv("CP_AUTOTUNE");
  return !(e && e[0] == '0');
}

// statistic, precision, weights, periodic, log2 of the point counts and of
// the expected neighbours per point within reach, pi_max / R_max for wp
static std::string tune_key(const Call &c, double volume) {
  const cp_options &o = *c.o;
  const int64_t n1 = c.d1 ? c.d1->n : 0;
  const int64_t n2 = c.cross && c.d2 ? c.d2->n : n1;
  const double R = c.edges[c.nedges - 1];
  const double reach = c.mode == XI ? 4.0 / 3.0 * M_PI * R * R * R : M_PI * R * R * 2.0 * c.pimax;
  const double neigh = std::max(1.0, (double)n2) * reach / std::max(volume, 1e-300);
  auto l2 = [](double v) { return (int)std::lround(std::log2(std::max(v, 1e-3))); };
  std::string k = std::string(c.mode == XI ? "xi" : "wp") + (c.cross ? "-cross" : "") +
                  (o.precision == CP_PREC_FP64 ? "/fp64" : "/fp32") + (o.need_ravg ? "/w" : "/u") +
                  (o.periodic ? "/p" : "/n") + "/n" + std::to_string(l2((double)std::max<int64_t>(n1, 1)));
  if (c.cross) k += "/m" + std::to_string(l2((double)std::max<int64_t>(n2, 1)));
  k += "/k" + std::to_string(l2(neigh));
  if (c.mode == WP) k += "/z" + std::to_string((int)std::lround(2.0 * std::log2(c.pimax / R)));
  return k;
}

static int run(const Call &c, uint64_t *npairs, double *wsum, double *ravg);

// Device time of one candidate's settings (refine, chunk target, waves).
using TuneTimer = std::function<int(const int ref[3], int chunk, int waves, double &ms)>;

// Coordinate descent over the candidates with `time_of` as the objective;
// stores the best settings under key.
static int tune_with(const TuneTimer &time_of, const std::string &key, TuneChoice &best) {
  best = TuneChoice();
  best.ms = INFINITY;
  // a candidate that does not fit a caller's workspace is skipped
  auto consider = [&](const int ref[3], int chunk, int waves) -> int {
    double ms;
    const int rc = time_of(ref, chunk, waves, ms);
    if (rc == CP_ERR_NOMEM) return CP_OK;
    if (rc) return rc;
    if (ms < best.ms) {
      for (int a = 0; a < 3; a++) best.refine[a] = ref[a];
      best.chunk_pct = chunk;
      best.waves = waves;
      best.ms = ms;
    }
    return CP_OK;
  };
  int rc;
  for (const auto &ref : kRefineCands)
    if ((rc = consider(ref, 100, 4))) return rc;
  if (!std::isfinite(best.ms)) return fail(CP_ERR_NOMEM, "no tuning candidate fits the workspace");
  const int bref[3] = {best.refine[0], best.refine[1], best.refine[2]};
  for (int ch : kChunkCands)
    if ((rc = consider(bref, ch, 4))) return rc;
  const int bch = best.chunk_pct;
  for (int wv : kWaveCands)
    if ((rc = consider(bref, bch, wv))) return rc;
  tune_store(key, best);
  return CP_OK;
}

// Times the candidates on every call of `calls` (the objective is their sum).
static int tune(const std::vector<Call> &calls, const std::string &key, TuneChoice &best) {
  std::vector<cp_options> opts;
  for (const Call &c : calls) opts.push_back(*c.o);
  std::vector<uint64_t> n;
  std::vector<double> w, r;
  auto time_of = [&](const int ref[3], int chunk, int waves, double &ms) -> int {
    ms = 0.0;
    for (size_t i = 0; i < calls.size(); i++) {
      Call c = calls[i];
      cp_options &o = opts[i];
      for (int a = 0; a < 3; a++) o.refine[a] = ref[a];
      c.o = &o;
      c.chunk_pct = chunk;
      c.waves = waves;
      const size_t nout = (size_t)(c.nedges - 1) * (c.mode == WP ? c.npi : 1);
      n.assign(nout, 0);
      w.assign(nout, 0.0);
      r.assign(nout, 0.0);
      double t = INFINITY;
      for (int rep = 0; rep < 3; rep++) {
        const int rc = run(c, n.data(), o.need_ravg ? w.data() : nullptr,
                           o.need_ravg ? r.data() : nullptr);
        if (rc) return rc;
        t = std::min(t, (double)g_stats.ms_total);
      }
      ms += t;
    }
    return CP_OK;
  };
  return tune_with(time_of, key, best);
}

// ------------------------------------------------------------- single call

static int run(const Call &c, uint64_t *npairs, double *wsum, double *ravg) {
  int rc = check_common(c);
  if (rc) return rc;
  if ((rc = check_points(c.d1, c.cross ? "d1" : "d"))) return rc;
  if (c.cross && (rc = check_points(c.d2, "d2"))) return rc;
  if (!npairs) return fail(CP_ERR_INVALID_ARG, "npairs is NULL");
  const cp_options &o = *c.o;
  if (o.need_ravg && (!wsum || !ravg))
    return fail(CP_ERR_INVALID_ARG, "need_ravg with NULL wsum or ravg");
  const int nb = c.nedges - 1;
  const int npi = c.mode == WP ? c.npi : 1;
  const int nout = nb * npi;
  const bool autoc = !c.cross;
  const cp_points &p1 = *c.d1;
  const cp_points &p2 = autoc ? *c.d1 : *c.d2;
  hipStream_t st = (hipStream_t)o.stream;
  g_stats_valid = false;
  memset(npairs, 0, sizeof(uint64_t) * nout);
  if (o.need_ravg) {
    memset(wsum, 0, sizeof(double) * nout);
    memset(ravg, 0, sizeof(double) * nout);
  }
  if (p1.n + (autoc ? 0 : p2.n) == 0) {
    memset(&g_stats, 0, sizeof(g_stats));
    g_stats.precision = o.precision;
    g_stats_valid = true;
    return CP_OK;
  }
  const bool weighted = o.need_ravg != 0;
  const double rmax = c.edges[nb];

  const bool noalloc = c.scratch != nullptr;
  // timing events: created once per thread and device, reused by every call
  // (the call without allocation creates and records none)
  static thread_local hipEvent_t tl_ev[kMaxDevices][4];
  hipEvent_t *ev = nullptr;
  if (!noalloc) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CP_ERR_DEVICE, "device index out of range");
    ev = tl_ev[dev];
    for (int i = 0; i < 4; i++)
      if (!ev[i]) HIPCHK(hipEventCreate(&ev[i]));
    HIPCHK(hipEventRecord(ev[0], st));
  }

  PointsDev pd[2];
  auto fillpd = [](const cp_points &p, PointsDev &d) {
    d.x = p.x;
    d.y = p.y;
    d.z = p.z;
    d.w = p.w;
    d.n = p.n;
    d.dtype = p.dtype;
    d.pad = 0;
  };
  fillpd(p1, pd[0]);
  fillpd(p2, pd[1]);

  // ---- domain
  double lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
  int *d_err0 = nullptr;
  if (!o.periodic) {
    // joint bounding box (Section 2.1: computed first) - needs a round trip
    // scratch for the reduction: the head of the caller's workspace, or of
    // the thread's cached arena (grown here if needed)
    const int nblk = 256;
    const size_t pre = sizeof(double) * (6 * nblk + 6) + 64;
    double *d_part = nullptr;
    if (noalloc) {
      if (c.scratch_bytes < pre) return fail(CP_ERR_NOMEM, "static scratch too small");
      d_part = (double *)c.scratch;
    } else if (o.workspace) {
      if (o.workspace_bytes < pre) return fail(CP_ERR_NOMEM, "workspace too small");
      d_part = (double *)o.workspace;
    } else {
      if (g_arena.cap < pre) {
        if (g_arena.base) {
          HIPCHK(hipDeviceSynchronize());
          (void)hipFree(g_arena.base);
          g_arena.base = nullptr;
          g_arena.cap = 0;
        }
        if (hipMalloc(&g_arena.base, 1 << 20) != hipSuccess) {
          g_arena.base = nullptr;
          return fail(CP_ERR_NOMEM, "hipMalloc of the scratch arena failed");
        }
        g_arena.cap = 1 << 20;
      }
      d_part = (double *)g_arena.base;
    }
    d_err0 = (int *)(d_part + 6 * nblk + 6);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, d_err0, (int64_t)1, 0);
    PointsDev b = pd[1];
    if (autoc) b.n = 0;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nblk), dim3(256), 0, st, pd[0], b, d_part, d_err0);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, d_part, nblk, d_part + 6 * nblk);
    double bb[6];
    int eflag = 0;
    HIPCHK(hipMemcpyAsync(bb, d_part + 6 * nblk, sizeof(bb), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&eflag, d_err0, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if ((rc = map_err_flags(eflag))) return rc;
    for (int a = 0; a < 3; a++) {
      lo[a] = bb[a];
      ext[a] = bb[a + 3] - bb[a];
      if (!(ext[a] >= 0)) {
        lo[a] = 0;
        ext[a] = 0;
      }
    }
  }
  const int64_t ntot = p1.n + (autoc ? 0 : p2.n);
  // launch settings: the caller's refine, or tuned / cached (refine 0)
  int refine_eff[3] = {o.refine[0], o.refine[1], o.refine[2]};
  int chunk_pct = c.chunk_pct > 0 ? c.chunk_pct : 100;
  int waves_most = c.waves > 0 ? c.waves : 4;
  int tuned = 0;
  if (!refine_eff[0] && !refine_eff[1] && !refine_eff[2]) {
    TuneChoice tc;
    tuned = 3;
    if (autotune_on()) {
      const double vol = o.periodic ? o.boxsize * o.boxsize * o.boxsize : ext[0] * ext[1] * ext[2];
      const std::string key = tune_key(c, vol);
      if (tune_lookup(key, tc)) {
        tuned = 2;
      } else if (!noalloc) {
        if ((rc = tune({c}, key, tc))) return rc;
        tuned = 1;
        // the call's own timing starts after the tuning runs
        if (!noalloc) HIPCHK(hipEventRecord(ev[0], st));
      }
    }
    for (int a = 0; a < 3; a++) refine_eff[a] = tc.refine[a];
    chunk_pct = tc.chunk_pct;
    waves_most = tc.waves;
  }
  Geometry g = choose_geometry(c.mode, o.periodic != 0, o.boxsize, lo, ext, rmax, c.pimax,
                               refine_eff, ntot);
  int prec = o.precision == CP_PREC_FP32_RECHECK ? F32R : F64;
  if (g.wrap[0] || g.wrap[1] || g.wrap[2]) prec = F64;   // per-pair minimum image: binary64
  // Weighted xi: every counted pair needs its binary64 separation, and on
  // gfx950 the binary64 loops (which skip the square root on records with no
  // lane in range) are faster than the binary32 screen with a list of the
  // in-range pairs evaluated in binary64 (measured on 10^6 clustered points:
  // 1.55 against 1.79 ms), so binary32 mode runs them unless
  // CP_XI_WEIGHTED_BINARY32=1 asks for the screen.
  if (c.mode == XI && o.need_ravg && prec == F32R) {
    const char *env = getenv("CP_XI_WEIGHTED_BINARY32");
    if (!(env && env[0] == '1')) prec = F64;
  }
  double M = 0;
  for (int a = 0; a < 3; a++) M = std::max(M, std::fabs(g.lo[a]) + g.ext[a]);
  if (o.periodic) M = std::max(M, o.boxsize);
  const Binning *Bp = nullptr;
  if ((rc = cached_binning(c.mode, prec, c.edges, c.nedges, c.pimax, npi, g, M, Bp))) return rc;
  const Binning &B = *Bp;

  const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int64_t ncol = (int64_t)g.n[0] * g.n[1];
  const int64_t maxt = max_tiles_bound(p1.n, ncell, ncol);
  const int n32 = (int)B.t32.e.size(), n64 = (int)B.t64.e.size();

  // ---- scratch layout
  float *d_c32 = nullptr, *d_a32 = nullptr;
  auto layout = [&](Carver &cv, SetBufs &S1, SetBufs &S2, Smalls *&sm, uint2 *&t32, uint2 *&t64,
                    double *&E, unsigned long long *&hist, double *&hw, double *&hwr,
                    unsigned long long *&stats, int *&err) {
    float *&c32 = d_c32, *&a32 = d_a32;
    carve_set(cv, S1, p1.n, ncell, ncol, true, maxt);
    if (!autoc) carve_set(cv, S2, p2.n, ncell, ncol, false, 0);
    sm = cv.take<Smalls>(1);
    t32 = cv.take<uint2>(n32);
    t64 = cv.take<uint2>(n64);
    E = cv.take<double>(c.nedges);
    c32 = cv.take<float>(c.nedges);
    a32 = cv.take<float>(c.nedges);
    hist = cv.take<unsigned long long>(nout);
    hw = cv.take<double>(nout);
    hwr = cv.take<double>(nout);
    stats = cv.take<unsigned long long>(kStatWords);
    err = cv.take<int>(1);
  };
  SetBufs S1, S2;
  Smalls *d_sm;
  uint2 *d_t32, *d_t64;
  double *d_E, *d_hw, *d_hwr;
  unsigned long long *d_hist, *d_stats;
  int *d_err;
  {
    Carver dry(nullptr, true);
    layout(dry, S1, S2, d_sm, d_t32, d_t64, d_E, d_hist, d_hw, d_hwr, d_stats, d_err);
    const size_t need = dry.off + 256;
    void *base;
    if (noalloc) {
      if (need > c.scratch_bytes)
        return fail(CP_ERR_NOMEM, "this call needs " + std::to_string(need) +
                                      " bytes of device scratch; the static scratch of "
                                      "countpairs_xi_noalloc holds " +
                                      std::to_string(c.scratch_bytes));
      base = c.scratch;
    } else if (o.workspace) {
      if (o.workspace_bytes < need)
        return fail(CP_ERR_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
      base = o.workspace;
    } else {
      if (g_arena.cap < need) {
        if (g_arena.base) {
          HIPCHK(hipDeviceSynchronize());
          (void)hipFree(g_arena.base);
          g_arena.base = nullptr;
          g_arena.cap = 0;
        }
        size_t want = need + need / 4;
        if (hipMalloc(&g_arena.base, want) != hipSuccess) {
          g_arena.base = nullptr;
          return fail(CP_ERR_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
        }
        g_arena.cap = want;
      }
      base = g_arena.base;
    }
    Carver cv(base, false);
    layout(cv, S1, S2, d_sm, d_t32, d_t64, d_E, d_hist, d_hw, d_hwr, d_stats, d_err);
  }
  if (autoc) S2 = S1;

  // ---- small records
  Smalls hs;
  memset(&hs, 0, sizeof(hs));
  hs.geom[0] = to_dev_geom(g, o.periodic != 0, o.boxsize, 0, 0, 0, p1.n, 0);
  hs.geom[1] = to_dev_geom(g, o.periodic != 0, o.boxsize, 0, 0, 0, p2.n, 0);
  hs.pts[0] = pd[0];
  hs.pts[1] = pd[1];
  hs.seg[0] = {0, 0, ncell, 0, kCountStride};
  hs.seg[1] = {0, 0, ncol, 0, 1};
  hs.seg[2] = {0, 0, ncol * col_blocks(p1.n), 0, 1};
  hs.seg[3] = {0, 0, ncol * col_blocks(p2.n), 0, 1};
  hs.win_prefix[0][0] = 0;
  hs.win_prefix[0][1] = (p1.n + kSortWin - 1) / kSortWin;
  hs.win_prefix[1][0] = 0;
  hs.win_prefix[1][1] = (p2.n + kSortWin - 1) / kSortWin;
  hs.col_prefix[0] = 0;
  hs.col_prefix[1] = ncol;
  hs.maxspan[0] = g.maxspan;
  {
    // the small records and tables are carved consecutively: one upload
    char *up0 = (char *)d_sm;
    const size_t upn = (size_t)((char *)(d_a32 + c.nedges) - up0);
    if (upn > kUpMax) return fail(CP_ERR_INTERNAL, "upload block larger than expected");
    // staging: pinned (the copy is a plain DMA); on the stack for the call
    // without allocation, or if pinned memory cannot be had
    alignas(16) char hstack[kUpMax];
    char *hup = noalloc ? nullptr : pinned_staging(kUpMax + kDownMax);
    if (!hup) hup = hstack;
    memset(hup, 0, upn);
    auto put = [&](const void *dev, const void *src, size_t bytes) {
      if (bytes) memcpy(hup + ((const char *)dev - up0), src, bytes);
    };
    put(d_sm, &hs, sizeof(hs));
    put(d_t32, B.t32.e.data(), (size_t)n32 * 8);
    put(d_t64, B.t64.e.data(), (size_t)n64 * 8);
    put(d_E, B.E.data(), (size_t)c.nedges * 8);
    put(d_c32, B.C32.data(), (size_t)c.nedges * 4);
    put(d_a32, B.A32.data(), (size_t)c.nedges * 4);
    HIPCHK(hipMemcpyAsync(up0, hup, upn, hipMemcpyHostToDevice, st));
  }
  // ---- cell build
  // histogram, weight sums, statistics and error flag are carved
  // consecutively: the build's first fill clears them too (zero bits are 0
  // and 0.0)
  const int64_t words = (int64_t)(((char *)(d_err + 1) - (char *)d_hist) / 4);
  rc = launch_build(st, &d_sm->pts[0], &d_sm->geom[0], S1, p1.n, ncell, ncol, c.mode,
                    &d_sm->seg[0], &d_sm->seg[1], &d_sm->seg[2], d_sm->win_prefix[0], d_sm->col_prefix,
                    d_sm->maxspan, d_err, true, (int *)d_hist, words);
  if (rc) return rc;
  if (!autoc) {
    rc = launch_build(st, &d_sm->pts[1], &d_sm->geom[1], S2, p2.n, ncell, ncol, c.mode,
                      &d_sm->seg[0], &d_sm->seg[1], &d_sm->seg[3], d_sm->win_prefix[1],
                      d_sm->col_prefix,
                      d_sm->maxspan, d_err, false);
    if (rc) return rc;
  }
  if (!noalloc) HIPCHK(hipEventRecord(ev[1], st));

  // ---- pairs
  PairParams P;
  memset(&P, 0, sizeof(P));
  P.tiles = S1.tiles;
  P.ntiles = S1.coloff + ncol;
  split_columns(g, autoc, rmax, c.mode == XI ? rmax : c.pimax, (double)p2.n,
                (prec == F64 ? 2.0 : 1.0) * (weighted ? 2.0 : 1.0) * (c.mode == WP ? 2.5 : 1.0),
                chunk_pct, P);
  P.geom1 = &d_sm->geom[0];
  P.geom2 = &d_sm->geom[1];
  P.pos1 = S1.pos;
  P.pos2 = S2.pos;
  P.strm2 = S2.strm;
  P.cstart2 = S2.cstart;
  P.cbox2 = S2.cbox;
  P.tab32 = d_t32 ? d_t32 : d_t64;
  P.tab64 = d_t64;
  P.tab32_lo = B.t32.lo;
  P.tab32_hi = B.t32.hi;
  P.tab64_lo = B.t64.lo;
  P.tab64_hi = B.t64.hi;
  P.tab_shift = B.shift;
  P.E = d_E;
  P.C32 = d_c32;
  P.A32 = d_a32;
  P.nb = nb;
  P.nslots = nb + 2;
  P.AB32 = B.AB32;
  P.eps32 = B.eps32;
  P.eps32_3 = B.eps32_3;
  P.EB = B.E[nb];
  P.pimax = c.pimax;
  P.dpi = B.dpi;
  P.inv_dpi = 1.0 / B.dpi;
  P.npi = npi;
  P.inv_dpi32 = B.inv_dpi32;
  P.pi_delta = B.pi_delta;
  P.pi_delta64 = B.pi_delta64;
  P.pi_hi32 = B.pi_hi32;
  P.autocorr = autoc ? 1 : 0;
  P.weighted = weighted ? 1 : 0;
  P.noprune = o.no_prune;
  P.hist = d_hist;
  P.hw = d_hw;
  P.hwr = d_hwr;
  P.stats = d_stats;
  P.hist_stride = nout;
  P.wpc = wp_copies(c.mode, prec, weighted, n32, n64, nb, npi);
  const LdsLayout LY = lds_layout(c.mode, prec, weighted, n32, n64, nb, npi, P.wpc);
  size_t lds = 0;
  const int nwaves = pick_waves(LY, &lds, waves_most);
  if (!nwaves) return fail(CP_ERR_INVALID_ARG, "too many bins for the LDS budget");
  if ((rc = launch_pairs(st, c.mode, prec, weighted, P, lds, nwaves))) return rc;
  if (!noalloc) HIPCHK(hipEventRecord(ev[2], st));

  // ---- results
  unsigned long long hst[kStatWords];
  int eflag = 0;
  std::vector<unsigned long long> h;
  std::vector<double> hwv, hwrv;
  if (noalloc) {
    // straight into the caller's outputs (raw counts and sums, finished
    // in place below), statistics and error flag on the stack
    HIPCHK(hipMemcpyAsync(npairs, d_hist, 8 * (size_t)nout, hipMemcpyDeviceToHost, st));
    if (weighted) {
      HIPCHK(hipMemcpyAsync(wsum, d_hw, 8 * (size_t)nout, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(ravg, d_hwr, 8 * (size_t)nout, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(hst, d_stats, sizeof(hst), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&eflag, d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    // histogram, weight sums, statistics and the error flag are carved
    // consecutively, so one download brings them all
    h.resize(nout);
    hwv.resize(nout);
    hwrv.resize(nout);
    char *dn0 = (char *)d_hist;
    const size_t dnn = (size_t)((char *)(d_err + 1) - dn0);
    if (dnn > kDownMax) return fail(CP_ERR_INTERNAL, "download block larger than expected");
    std::vector<char> hvec;
    char *hdn = pinned_staging(kUpMax + kDownMax);
    if (hdn) {
      hdn += kUpMax;
    } else {
      hvec.resize(dnn);
      hdn = hvec.data();
    }
    HIPCHK(hipMemcpyAsync(hdn, dn0, dnn, hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(ev[3], st));
    HIPCHK(hipStreamSynchronize(st));
    auto get = [&](void *dst, const void *dev, size_t bytes) {
      memcpy(dst, hdn + ((const char *)dev - dn0), bytes);
    };
    get(h.data(), d_hist, 8 * (size_t)nout);
    if (weighted) {
      get(hwv.data(), d_hw, 8 * (size_t)nout);
      get(hwrv.data(), d_hwr, 8 * (size_t)nout);
    }
    get(hst, d_stats, sizeof(hst));
    get(&eflag, d_err, sizeof(int));
  }
  const int ntiles = (int)hst[4];
  rc = map_err_flags(eflag);
  if (!rc) {
    const int64_t nitems = (int64_t)ntiles * P.nsplit;
    for (int k = 0; k < kQueues; k++) {
      const int64_t len = nitems * (k + 1) / kQueues - nitems * k / kQueues;
      if (hst[5 + k * kQStride] < (unsigned long long)len)
        rc = fail(CP_ERR_INTERNAL, "work queue not drained");
    }
  }
  if (rc) {
    // failed calls leave zero outputs (the raw sums were copied into them)
    memset(npairs, 0, sizeof(uint64_t) * nout);
    if (o.need_ravg) {
      memset(wsum, 0, sizeof(double) * nout);
      memset(ravg, 0, sizeof(double) * nout);
    }
    return rc;
  }

  const double mult = (autoc && o.count_mode == CP_ORDERED) ? 2.0 : 1.0;
  for (int k = 0; k < nout; k++) {
    // noalloc: npairs, wsum and ravg hold the raw count and sums
    const unsigned long long hk = noalloc ? npairs[k] : h[k];
    const double w = noalloc ? (weighted ? wsum[k] : 0.0) : hwv[k];
    const double wr = noalloc ? (weighted ? ravg[k] : 0.0) : hwrv[k];
    npairs[k] = (uint64_t)hk * (uint64_t)mult;
    if (weighted) {
      wsum[k] = w * mult;
      ravg[k] = hk ? wr / w : 0.0;
    }
  }
  memset(&g_stats, 0, sizeof(g_stats));
  g_stats.candidates = hst[0];
  g_stats.rechecks = hst[1];
  g_stats.cell_pairs = hst[2];
  g_stats.cell_pairs_pruned = hst[3];
  g_stats.tiles = (uint64_t)ntiles;
  for (int a = 0; a < 3; a++) {
    g_stats.grid[a] = g.n[a];
    g_stats.refine[a] = g.r[a];
  }
  if (!noalloc) {
    (void)hipEventElapsedTime(&g_stats.ms_grid, ev[0], ev[1]);
    (void)hipEventElapsedTime(&g_stats.ms_pairs, ev[1], ev[2]);
    (void)hipEventElapsedTime(&g_stats.ms_total, ev[0], ev[3]);
  }
  g_stats.precision = prec == F32R ? CP_PREC_FP32_RECHECK : CP_PREC_FP64;
  g_stats.tuned = tuned;
  g_stats.chunk_pct = chunk_pct;
  g_stats.waves = nwaves;
  g_stats_valid = true;
  return CP_OK;
}

// ------------------------------------------------- static device scratch
//
// Device scratch of countpairs_xi_noalloc: a file-scope array that every
// device the library runs on holds from module load until the process ends.
// Host code never uses the array's name as an address: its device address
// comes from hipGetSymbolAddress, once per device with that device current
// (on the device's first such call), and is kept per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int static_scratch(void **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CP_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CP_OK;
}

} // namespace cp

// =================================================================== C ABI

using namespace cp;

extern "C" {

void cp_default_options(cp_options *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = CP_PREC_FP32_RECHECK;
  o->count_mode = CP_ORDERED;
}

int countpairs_xi(const cp_points *d, const double *edges, int nedges, const cp_options *o,
                  uint64_t *npairs, double *wsum, double *ravg) {
  try {
    Call c{XI, false, d, nullptr, edges, nedges, 0.0, 1, o};
    return run(c, npairs, wsum, ravg);
  } catch (...) {
    return fail(CP_ERR_INTERNAL, "unexpected exception");
  }
}

int countpairs_wp(const cp_points *d, const double *rp_edges, int nedges, double pimax,
                  int npibins, const cp_options *o, uint64_t *npairs, double *wsum,
                  double *rpavg) {
  try {
    Call c{WP, false, d, nullptr, rp_edges, nedges, pimax, npibins, o};
    return run(c, npairs, wsum, rpavg);
  } catch (...) {
    return fail(CP_ERR_INTERNAL, "unexpected exception");
  }
}

int countpairs_xi_noalloc(const cp_points *d, const double *edges, int nedges,
                          const cp_options *o, uint64_t *npairs, double *wsum, double *ravg) {
  try {
    if (o && o->workspace)
      return fail(CP_ERR_INVALID_ARG,
                  "countpairs_xi_noalloc takes no workspace: it uses the library's static scratch");
    void *sp = nullptr;
    int rc = static_scratch(&sp);
    if (rc) return rc;
    Call c{XI, false, d, nullptr, edges, nedges, 0.0, 1, o, sp, kScratchBytes};
    return run(c, npairs, wsum, ravg);
  } catch (...) {
    return fail(CP_ERR_INTERNAL, "unexpected exception");
  }
}

int countpairs_cross(const cp_points *d1, const cp_points *d2, const double *edges, int nedges,
                     const cp_options *o, uint64_t *npairs, double *wsum, double *ravg) {
  try {
    Call c{XI, true, d1, d2, edges, nedges, 0.0, 1, o};
    return run(c, npairs, wsum, ravg);
  } catch (...) {
    return fail(CP_ERR_INTERNAL, "unexpected exception");
  }
}

int countpairs_cross_wp(const cp_points *d1, const cp_points *d2, const double *rp_edges,
                        int nedges, double pimax, int npibins, const cp_options *o,
                        uint64_t *npairs, double *wsum, double *rpavg) {
  try {
    Call c{WP, true, d1, d2, rp_edges, nedges, pimax, npibins, o};
    return run(c, npairs, wsum, rpavg);
  } catch (...) {
    return fail(CP_ERR_INTERNAL, "unexpected exception");
  }
}

const char *countpairs_strerror(int code) {
  switch (code) {
  case CP_OK: return "ok";
  case CP_ERR_INVALID_ARG: return "invalid argument";
  case CP_ERR_OUT_OF_BOX: return "coordinate outside the periodic box";
  case CP_ERR_NONFINITE: return "non-finite coordinate or weight";
  case CP_ERR_NOMEM: return "out of device memory or workspace too small";
  case CP_ERR_DEVICE: return "HIP runtime error";
  case CP_ERR_INTERNAL: return "internal consistency check failed";
  default: return "unknown error";
  }
}

const char *countpairs_last_error(void) { return g_err.c_str(); }

int countpairs_last_stats(cp_stats *out) {
  if (!out) return CP_ERR_INVALID_ARG;
  if (!g_stats_valid) return fail(CP_ERR_INVALID_ARG, "no successful call on this thread");
  *out = g_stats;
  return CP_OK;
}

} // extern "C"

extern "C" size_t countpairs_workspace_size(int kind, int64_t n1, int64_t n2, const double *edges,
                                            int nedges, double pimax, int npibins,
                                            const cp_options *o) {
  (void)edges;
  (void)pimax;
  (void)o;
  if (n1 < 0 || n2 < 0 || nedges < 2) return 0;
  const bool cross = kind >= 2;
  const int npi = (kind == 1 || kind == 3) ? std::max(1, npibins) : 1;
  const int64_t ntot = n1 + (cross ? n2 : 0);
  const int64_t ncell = std::max<int64_t>(4096, 4 * ntot);   // the cell-count cap
  const int64_t ncol = std::min<int64_t>(ncell, (int64_t)kMaxAxisCells * kMaxAxisCells);
  Carver cv(nullptr, true);
  SetBufs S1, S2;
  carve_set(cv, S1, n1, ncell, ncol, true, max_tiles_bound(n1, ncell, ncol));
  if (cross) carve_set(cv, S2, n2, ncell, ncol, false, 0);
  const int nout = (nedges - 1) * npi;
  cv.take<Smalls>(1);
  cv.take<uint2>(4096);
  cv.take<uint2>(4096);
  cv.take<double>(nedges);
  cv.take<float>(nedges);
  cv.take<float>(nedges);
  cv.take<unsigned long long>(nout);
  cv.take<double>(nout);
  cv.take<double>(nout);
  cv.take<unsigned long long>(kStatWords);
  cv.take<int>(1);
  return cv.off + 256;
}

// ================================================================== plans

namespace cp {

struct Batch {
  bool on = false;
  int mode = XI, prec = F32R;
  Geometry g;
  Binning B;
  int nb = 0, npi = 1, nout = 0;
  int64_t ncell = 0, ncol = 0, ncell_tot = 0, ncol_tot = 0, npts_tot = 0, maxtiles = 0;
  std::vector<GridGeom> geoms;
  std::vector<ScanSeg> segs;      // nmock cell segments, then 1 column segment
  std::vector<int64_t> win_prefix, col_prefix;
  std::vector<int> maxspan;
  // column build (grids of up to kColLds columns): one column x block matrix
  // per catalogue, nmock scan segments over them
  bool colpath = false;
  std::vector<ScanSeg> msegs;
  int64_t nmat_tot = 0, mtiles = 0;
  int maxnb = 1;
  // device
  GridGeom *d_geom = nullptr;
  PointsDev *d_pts = nullptr;
  ScanSeg *d_segs = nullptr, *d_msegs = nullptr;
  int64_t *d_win_prefix = nullptr, *d_col_prefix = nullptr;
  int *d_maxspan = nullptr;
  SetBufs S{};
  uint2 *d_t32 = nullptr, *d_t64 = nullptr;
  double *d_E = nullptr;
  float *d_c32 = nullptr, *d_a32 = nullptr;
  unsigned long long *d_hist = nullptr, *d_stats = nullptr;
  double *d_hw = nullptr, *d_hwr = nullptr;
  int *d_err = nullptr;
  size_t lds = 0;
  int nwaves = 4;
  int waves_most = 4;      // launch settings from the caller or the tuner
  int wpc = 1;             // copies of the w_p wave histogram
  int chunk_pct = 100;
  double pimax = 0.0;
  PairParams P{};
};

} // namespace cp

struct cp_plan {
  int nmock = 0;
  std::vector<int> order;        // queue position -> caller's index
  std::vector<int64_t> n;        // points per catalogue (queue order)
  int64_t maxn = 0;
  std::vector<cp::PointsDev> pts;
  cp::Batch xi, wp;
  int count_mode = CP_ORDERED;
  int noprune = 0;
  int tuned = 0;                 // as cp_stats.tuned
  // xi and w_p in one launch (binary32): the w_p batch's build and pair
  // launch serve both statistics; xi keeps only its histogram
  bool fused = false;
  cp::Binning xbin;              // xi decision table of the fused estimate
  uint2 *d_tabx = nullptr;
  double *d_Ex = nullptr;
  void *mem = nullptr;
  hipStream_t cap = nullptr;
  hipStream_t last = nullptr;    // stream of the last execute (results and stats sync it)
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  int timed = 0;                 // 1: eager events, 2: graph events
  hipEvent_t ev[5] = {};
};

namespace cp {

static int batch_prepare(cp_plan &pl, Batch &b, int mode, int prec, const double *edges,
                         int nedges, double pimax, int npi, const cp_options &o) {
  b.on = true;
  b.mode = mode;
  b.nb = nedges - 1;
  b.npi = mode == WP ? npi : 1;
  b.pimax = mode == WP ? pimax : 0.0;
  b.nout = b.nb * b.npi;
  const double lo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
  b.g = choose_geometry(mode, true, o.boxsize, lo, ext, edges[nedges - 1], pimax, o.refine,
                        pl.maxn);
  b.prec = (b.g.wrap[0] || b.g.wrap[1] || b.g.wrap[2]) ? F64 : prec;
  int rc = make_binning(mode, b.prec, edges, nedges, pimax, b.npi, b.g, o.boxsize, b.B);
  if (rc) return rc;
  b.ncell = (int64_t)b.g.n[0] * b.g.n[1] * b.g.n[2];
  b.ncol = (int64_t)b.g.n[0] * b.g.n[1];
  b.geoms.clear();
  b.segs.clear();
  b.win_prefix.assign(1, 0);
  b.col_prefix.assign(1, 0);
  b.maxspan.clear();
  int64_t pb = 0;
  for (int m = 0; m < pl.nmock; m++) {
    const int64_t cbase = b.ncell * m, sbase = (b.ncell + 1) * m, colbase = b.ncol * m;
    b.geoms.push_back(to_dev_geom(b.g, true, o.boxsize, pb, cbase, sbase, pl.n[m], colbase));
    b.segs.push_back({cbase, sbase, b.ncell, scan_tiles(b.ncell) * m, kCountStride});
    b.win_prefix.push_back(b.win_prefix.back() + (pl.n[m] + kSortWin - 1) / kSortWin);
    b.col_prefix.push_back(b.ncol * (m + 1));
    b.maxspan.push_back(b.g.maxspan);
    pb += pl.n[m];
  }
  b.npts_tot = pb;
  b.ncell_tot = b.ncell * pl.nmock;
  b.ncol_tot = b.ncol * pl.nmock;
  b.segs.push_back({0, 0, b.ncol_tot, 0, 1});
  // the column build, as for single calls: each catalogue's matrix holds
  // ncol * nblk counts and, after its scan, the total (one more word)
  const char *ce = getenv("CP_BUILD_COLUMNS");
  b.colpath = b.ncol <= kColLds && !(ce && ce[0] == '0');
  b.msegs.clear();
  b.nmat_tot = 0;
  b.mtiles = 0;
  b.maxnb = 1;
  if (b.colpath) {
    for (GridGeom &G : b.geoms) {
      G.mbase = b.nmat_tot;
      const int64_t len = b.ncol * G.nblk;
      b.msegs.push_back({G.mbase, G.mbase, len, b.mtiles, 1});
      b.mtiles += scan_tiles(len);
      b.nmat_tot += len + 1;
      b.maxnb = std::max(b.maxnb, G.nblk);
    }
  }
  b.maxtiles = max_tiles_bound(b.npts_tot, b.ncell_tot, b.ncol_tot);
  b.wpc = wp_copies(mode, b.prec, 0, (int)b.B.t32.e.size(), (int)b.B.t64.e.size(), b.nb, b.npi);
  const LdsLayout LY = lds_layout(mode, b.prec, 0, (int)b.B.t32.e.size(),
                                  (int)b.B.t64.e.size(), b.nb, b.npi, b.wpc);
  b.nwaves = pick_waves(LY, &b.lds, b.waves_most);
  if (!b.nwaves) return fail(CP_ERR_INVALID_ARG, "too many bins for the LDS budget");
  return CP_OK;
}

static void batch_carve(Carver &cv, cp_plan &pl, Batch &b) {
  if (!b.on) return;
  const int nm = pl.nmock;
  b.d_geom = cv.take<GridGeom>(nm);
  b.d_pts = cv.take<PointsDev>(nm);
  b.d_segs = cv.take<ScanSeg>(nm + 1);
  b.d_msegs = cv.take<ScanSeg>(b.colpath ? nm : 1);
  b.d_win_prefix = cv.take<int64_t>(nm + 1);
  b.d_col_prefix = cv.take<int64_t>(nm + 1);
  b.d_maxspan = cv.take<int>(nm);
  // cell_start needs ncell + 1 per catalogue
  b.S.ccount = cv.take<int>(b.ncell_tot * kCountStride);
  b.S.tsum = cv.take<int>(
      std::max({scan_tiles(b.ncell) * nm, scan_tiles(b.ncol_tot), b.colpath ? b.mtiles : 1}));
  b.S.colmat = cv.take<int>(b.colpath ? b.nmat_tot : 1);
  b.S.cstart = cv.take<int>(b.ncell_tot + nm);
  b.S.cid = cv.take<int>(std::max<int64_t>(b.npts_tot, 1));
  b.S.rank = cv.take<int>(std::max<int64_t>(b.npts_tot, 1));
  b.S.pos = cv.take<double4>(b.npts_tot + 8);
  b.S.grp = cv.take<double4>(std::max<int64_t>(b.npts_tot, 1));
  b.S.strm = cv.take<float4>(b.npts_tot + 8);
  b.S.cbox = cv.take<CellBox>(b.ncell_tot);
  b.S.colcnt = cv.take<int>(b.ncol_tot + 1);
  b.S.coloff = cv.take<int>(b.ncol_tot + 1);
  b.S.tiles = cv.take<Tile>(b.maxtiles);
  b.d_t32 = cv.take<uint2>(b.B.t32.e.size());
  b.d_t64 = cv.take<uint2>(b.B.t64.e.size());
  b.d_E = cv.take<double>(b.nb + 1);
  b.d_c32 = cv.take<float>(b.nb + 1);
  b.d_a32 = cv.take<float>(b.nb + 1);
  b.d_hist = cv.take<unsigned long long>((int64_t)b.nout * nm);
  b.d_hw = cv.take<double>(1);
  b.d_hwr = cv.take<double>(1);
  b.d_stats = cv.take<unsigned long long>(kStatWords);
  b.d_err = cv.take<int>(1);
}

static int batch_upload(cp_plan &pl, Batch &b) {
  if (!b.on) return CP_OK;
  const int nm = pl.nmock;
  HIPCHK(hipMemcpy(b.d_geom, b.geoms.data(), sizeof(GridGeom) * nm, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_pts, pl.pts.data(), sizeof(PointsDev) * nm, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_segs, b.segs.data(), sizeof(ScanSeg) * (nm + 1), hipMemcpyHostToDevice));
  if (b.colpath)
    HIPCHK(hipMemcpy(b.d_msegs, b.msegs.data(), sizeof(ScanSeg) * nm, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_win_prefix, b.win_prefix.data(), 8 * (nm + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_col_prefix, b.col_prefix.data(), 8 * (nm + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_maxspan, b.maxspan.data(), 4 * nm, hipMemcpyHostToDevice));
  if (!b.B.t32.e.empty())
    HIPCHK(hipMemcpy(b.d_t32, b.B.t32.e.data(), 8 * b.B.t32.e.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_t64, b.B.t64.e.data(), 8 * b.B.t64.e.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_E, b.B.E.data(), 8 * (b.nb + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_c32, b.B.C32.data(), 4 * (b.nb + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b.d_a32, b.B.A32.data(), 4 * (b.nb + 1), hipMemcpyHostToDevice));
  PairParams &P = b.P;
  memset(&P, 0, sizeof(P));
  P.tiles = b.S.tiles;
  P.ntiles = b.S.coloff + b.ncol_tot;
  split_columns(b.g, true, std::sqrt(b.B.E[b.nb]), b.mode == XI ? std::sqrt(b.B.E[b.nb]) : b.pimax,
                (double)b.npts_tot / std::max(1, pl.nmock),
                (b.prec == F64 ? 2.0 : 1.0) * (b.mode == WP ? 2.5 : 1.0), b.chunk_pct, P);
  P.geom1 = b.d_geom;
  P.geom2 = b.d_geom;
  P.pos1 = b.S.pos;
  P.pos2 = b.S.pos;
  P.strm2 = b.S.strm;
  P.cstart2 = b.S.cstart;
  P.cbox2 = b.S.cbox;
  P.tab32 = b.B.t32.e.empty() ? b.d_t64 : b.d_t32;
  P.tab64 = b.d_t64;
  P.tab32_lo = b.B.t32.lo;
  P.tab32_hi = b.B.t32.hi;
  P.tab64_lo = b.B.t64.lo;
  P.tab64_hi = b.B.t64.hi;
  P.tab_shift = b.B.shift;
  P.E = b.d_E;
  P.C32 = b.d_c32;
  P.A32 = b.d_a32;
  P.nb = b.nb;
  P.nslots = b.nb + 2;
  P.AB32 = b.B.AB32;
  P.eps32 = b.B.eps32;
  P.eps32_3 = b.B.eps32_3;
  P.EB = b.B.E[b.nb];
  P.pimax = b.pimax;
  P.dpi = b.B.dpi;
  P.inv_dpi = 1.0 / b.B.dpi;
  P.npi = b.npi;
  P.wpc = b.wpc;
  P.inv_dpi32 = b.B.inv_dpi32;
  P.pi_delta = b.B.pi_delta;
  P.pi_delta64 = b.B.pi_delta64;
  P.pi_hi32 = b.B.pi_hi32;
  P.autocorr = 1;
  P.weighted = 0;
  P.noprune = pl.noprune;
  P.hist = b.d_hist;
  P.hw = b.d_hw;
  P.hwr = b.d_hwr;
  P.stats = b.d_stats;
  P.hist_stride = b.nout;
  return CP_OK;
}

static int batch_enqueue(cp_plan &pl, Batch &b, hipStream_t st) {
  if (!b.on) return CP_OK;
  const int nm = pl.nmock;
  auto blocks = [](int64_t n, int per, int cap) {
    return (int)std::min<int64_t>(std::max<int64_t>((n + per - 1) / per, 1), cap);
  };
  if (pl.fused && &b == &pl.xi) {
    // the fused w_p launch fills xi's histogram: clear it and xi's flag
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks((int64_t)b.nout * nm, 256, 1024)), dim3(256), 0,
                       st, b.d_hist, (int64_t)b.nout * nm);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, b.d_err, (int64_t)1, 0);
    return hipGetLastError() == hipSuccess ? CP_OK : fail(CP_ERR_DEVICE, "launch failed");
  }
  if (!b.colpath)
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(b.ncell_tot * kCountStride, 256, 8192)), dim3(256),
                       0, st, b.S.ccount, b.ncell_tot * kCountStride, 0);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks((int64_t)b.nout * nm, 256, 1024)), dim3(256), 0, st,
                     b.d_hist, (int64_t)b.nout * nm);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, b.d_stats, (int64_t)kStatWords);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, b.d_err, (int64_t)1, 0);
  if (b.colpath) {
    // every catalogue's column build at once (blockIdx.y = catalogue); the
    // per-column pass also counts the columns' tiles
    hipLaunchKernelGGL(k_colcount, dim3(b.maxnb, nm), dim3(1024), 0, st, b.d_pts, b.d_geom,
                       b.S.colmat, b.d_err);
    const unsigned tm = (unsigned)b.mtiles;
    hipLaunchKernelGGL(k_scan_sums, dim3(tm), dim3(256), 0, st, b.S.colmat, b.d_msegs, nm,
                       b.S.tsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(tm), dim3(256), 0, st, b.S.colmat, b.S.colmat,
                       b.d_msegs, nm, b.S.tsum);
    hipLaunchKernelGGL(k_colscatter, dim3(b.maxnb, nm), dim3(1024), 0, st, b.d_pts, b.d_geom,
                       b.S.colmat, b.S.pos);
    hipLaunchKernelGGL(k_colcells, dim3((unsigned)std::min<int64_t>(b.ncol, 8192), nm), dim3(256),
                       0, st, b.d_geom, b.S.colmat, b.S.pos, b.S.grp, b.S.cstart, b.d_maxspan,
                       b.d_col_prefix, b.S.colcnt);
  } else {
    hipLaunchKernelGGL(k_assign, dim3(blocks(pl.maxn, 256, 4096), nm), dim3(256), 0, st, b.d_pts,
                       b.d_geom, b.S.ccount, b.S.cid, b.S.rank, b.d_err);
    const unsigned sc = (unsigned)(scan_tiles(b.ncell) * nm);
    hipLaunchKernelGGL(k_scan_sums, dim3(sc), dim3(256), 0, st, b.S.ccount, b.d_segs, nm,
                       b.S.tsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(sc), dim3(256), 0, st, b.S.ccount, b.S.cstart,
                       b.d_segs, nm, b.S.tsum);
    hipLaunchKernelGGL(k_group, dim3(blocks(pl.maxn, 256, 4096), nm), dim3(256), 0, st, b.d_pts,
                       b.d_geom, b.S.cstart, b.S.cid, b.S.rank, b.S.grp);
  }
  hipLaunchKernelGGL(k_cellsort, dim3(blocks(b.win_prefix[nm], 4, 65536)), dim3(256), 0, st,
                     b.d_geom, nm, b.S.cstart, b.S.grp, b.S.pos, b.S.strm, b.S.cbox, b.d_win_prefix,
                     b.mode);
  const int tb = blocks(b.ncol_tot, 4, 65536);
  if (!b.colpath)
    hipLaunchKernelGGL(k_tiles, dim3(tb), dim3(256), 0, st, b.d_geom, nm, b.S.cstart, b.d_maxspan,
                       b.d_col_prefix, b.S.colcnt, b.S.coloff, b.S.tiles, 0);
  const unsigned tcol = (unsigned)scan_tiles(b.ncol_tot);
  hipLaunchKernelGGL(k_scan_sums, dim3(tcol), dim3(256), 0, st, b.S.colcnt, b.d_segs + nm, 1,
                     b.S.tsum);
  hipLaunchKernelGGL(k_scan_apply, dim3(tcol), dim3(256), 0, st, b.S.colcnt, b.S.coloff,
                     b.d_segs + nm, 1, b.S.tsum);
  hipLaunchKernelGGL(k_tiles, dim3(tb), dim3(256), 0, st, b.d_geom, nm, b.S.cstart, b.d_maxspan,
                     b.d_col_prefix, b.S.colcnt, b.S.coloff, b.S.tiles, 1);
  return launch_pairs(st, (pl.fused && &b == &pl.wp) ? WPXI : b.mode, b.prec, 0, b.P, b.lds,
                      b.nwaves);
}

// Enqueue one evaluation.  With timing events (eager mode only) the xi and
// wp halves are timed separately; a captured graph is timed as a whole.
static int plan_enqueue(cp_plan &pl, hipStream_t st, bool events) {
  int rc;
  (void)hipGetLastError();
  if (events) HIPCHK(hipEventRecord(pl.ev[0], st));
  if ((rc = batch_enqueue(pl, pl.xi, st))) return rc;
  if (events) HIPCHK(hipEventRecord(pl.ev[1], st));
  if ((rc = batch_enqueue(pl, pl.wp, st))) return rc;
  if (events) HIPCHK(hipEventRecord(pl.ev[2], st));
  return CP_OK;
}

} // namespace cp

extern "C" {

int cp_plan_destroy(cp_plan *pl) {
  if (!pl) return CP_OK;
  if (pl->gexec) (void)hipGraphExecDestroy(pl->gexec);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  for (auto &e : pl->ev)
    if (e) (void)hipEventDestroy(e);
  if (pl->mem) (void)hipFree(pl->mem);
  delete pl;
  return CP_OK;
}

// forced: launch settings to use as given (the tuner's trial plans), else
// the caller's refine or the tuned settings.
static int plan_create(const cp_points *mocks, int nmocks, const double *xi_edges, int xi_nedges,
                       const double *wp_edges, int wp_nedges, double pimax, int npibins,
                       const cp_options *o, const TuneChoice *forced, cp_plan **out) {
  try {
    if (!out) return fail(CP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!mocks || nmocks < 1 || nmocks > 65535)
      return fail(CP_ERR_INVALID_ARG, "need 1..65535 catalogues");
    if (!o) return fail(CP_ERR_INVALID_ARG, "options is NULL");
    if (!o->periodic) return fail(CP_ERR_INVALID_ARG, "plans need a periodic box");
    if (!xi_edges && !wp_edges) return fail(CP_ERR_INVALID_ARG, "no statistic requested");
    int rc;
    for (int m = 0; m < nmocks; m++) {
      std::string nm = "mocks[" + std::to_string(m) + "]";
      if ((rc = check_points(&mocks[m], nm.c_str()))) return rc;
    }
    if (xi_edges) {
      Call c{XI, false, &mocks[0], nullptr, xi_edges, xi_nedges, 0.0, 1, o};
      if ((rc = check_common(c))) return rc;
    }
    if (wp_edges) {
      Call c{WP, false, &mocks[0], nullptr, wp_edges, wp_nedges, pimax, npibins, o};
      if ((rc = check_common(c))) return rc;
    }
    cp_plan *pl = new cp_plan();
    pl->nmock = nmocks;
    pl->count_mode = o->count_mode;
    pl->noprune = o->no_prune;
    pl->order.resize(nmocks);
    for (int m = 0; m < nmocks; m++) pl->order[m] = m;
    // longest first: the queue hands out the biggest catalogues' tiles first
    std::stable_sort(pl->order.begin(), pl->order.end(),
                     [&](int a, int b) { return mocks[a].n > mocks[b].n; });
    for (int q = 0; q < nmocks; q++) {
      const cp_points &p = mocks[pl->order[q]];
      pl->n.push_back(p.n);
      pl->maxn = std::max(pl->maxn, p.n);
      PointsDev d;
      d.x = p.x;
      d.y = p.y;
      d.z = p.z;
      d.w = nullptr;   // plans count pairs only
      d.n = p.n;
      d.dtype = p.dtype;
      d.pad = 0;
      pl->pts.push_back(d);
    }
    const int prec = o->precision == CP_PREC_FP32_RECHECK ? F32R : F64;
    // xi and w_p in one launch (binary32): every xi pair must lie in the w_p
    // search (xi R_max at most r_p,max and pi_max); CP_PLAN_FUSED=0 keeps two
    const char *fe = getenv("CP_PLAN_FUSED");
    const bool want_fused = xi_edges && wp_edges && prec == F32R && !(fe && fe[0] == '0') &&
                            xi_edges[xi_nedges - 1] <= wp_edges[wp_nedges - 1] &&
                            xi_edges[xi_nedges - 1] <= pimax;
    // launch settings: the caller's refine, or tuned (cached): by timing
    // single calls of the requested statistics on the median catalogue, or,
    // for a fused launch, plans of up to four catalogues picked at even
    // quantiles of the pair work (taken as n^2), which the largest dominate
    cp_options po = *o;
    po.need_ravg = 0;
    po.count_mode = CP_ORDERED;
    TuneChoice tc;
    if (forced) {
      tc = *forced;
      for (int a = 0; a < 3; a++) po.refine[a] = tc.refine[a];
      pl->tuned = 0;
    } else if (!po.refine[0] && !po.refine[1] && !po.refine[2]) {
      pl->tuned = 3;
      if (autotune_on()) {
        const int med = pl->order[nmocks / 2];   // order: decreasing size
        std::vector<Call> calls;
        if (xi_edges && !want_fused)
          calls.push_back(Call{XI, false, &mocks[med], nullptr, xi_edges, xi_nedges, 0.0, 1, &po});
        if (wp_edges)
          calls.push_back(Call{WP, false, &mocks[med], nullptr, wp_edges, wp_nedges, pimax, npibins, &po});
        const double vol = po.boxsize * po.boxsize * po.boxsize;
        const std::string key = "plan:" + tune_key(calls[0], vol) +
                                (want_fused ? "+fused" : calls.size() > 1 ? "+wp" : "");
        if (tune_lookup(key, tc)) {
          pl->tuned = 2;
        } else {
          if (want_fused) {
            std::vector<cp_points> trial;
            double tot = 0.0, acc = 0.0;
            for (int q = 0; q < nmocks; q++) tot += (double)pl->n[q] * (double)pl->n[q];
            const int K = std::min(nmocks, 4);
            for (int q = 0, k = 0; q < nmocks && k < K; q++) {
              acc += (double)pl->n[q] * (double)pl->n[q];
              // catalogue q (in decreasing size) holds quantile (k + 1/2) / K
              for (; k < K && acc >= tot * (k + 0.5) / K; k++) trial.push_back(mocks[pl->order[q]]);
            }
            const TuneTimer ptime = [&](const int ref[3], int chunk, int waves, double &ms) -> int {
              TuneChoice f;
              for (int a = 0; a < 3; a++) f.refine[a] = ref[a];
              f.chunk_pct = chunk;
              f.waves = waves;
              cp_plan *sp = nullptr;
              int r = plan_create(trial.data(), (int)trial.size(), xi_edges, xi_nedges, wp_edges,
                                  wp_nedges, pimax, npibins, o, &f, &sp);
              if (r) return r;
              ms = INFINITY;
              for (int rep = 0; rep < 3 && !r; rep++) {
                cp_stats xs;
                if (!(r = cp_plan_execute(sp, o->stream)) && !(r = cp_plan_stats(sp, &xs, nullptr)) &&
                    rep > 0)
                  ms = std::min(ms, (double)xs.ms_total);
              }
              cp_plan_destroy(sp);
              return r;
            };
            rc = tune_with(ptime, key, tc);
          } else {
            rc = tune(calls, key, tc);
          }
          if (rc) {
            cp_plan_destroy(pl);
            return rc;
          }
          pl->tuned = 1;
        }
      }
      for (int a = 0; a < 3; a++) po.refine[a] = tc.refine[a];
    }
    for (Batch *b : {&pl->xi, &pl->wp}) {
      b->chunk_pct = tc.chunk_pct;
      b->waves_most = tc.waves;
    }
    if (xi_edges && (rc = batch_prepare(*pl, pl->xi, XI, prec, xi_edges, xi_nedges, 0.0, 1, po))) {
      cp_plan_destroy(pl);
      return rc;
    }
    if (wp_edges &&
        (rc = batch_prepare(*pl, pl->wp, WP, prec, wp_edges, wp_nedges, pimax, npibins, po))) {
      cp_plan_destroy(pl);
      return rc;
    }
    if (want_fused && pl->xi.prec == F32R && pl->wp.prec == F32R &&
        make_binning_wpxi(xi_edges, xi_nedges, pl->wp.B, pl->xbin)) {
      Batch &b = pl->wp;
      const int n32 = (int)b.B.t32.e.size(), n64 = (int)b.B.t64.e.size();
      const int nx = (int)pl->xbin.t32.e.size(), nbx = xi_nedges - 1;
      b.wpc = wp_copies(WPXI, F32R, 0, n32, n64, b.nb, b.npi, nx, nbx);
      const LdsLayout LY = lds_layout(WPXI, F32R, 0, n32, n64, b.nb, b.npi, b.wpc, nx, nbx);
      b.nwaves = pick_waves(LY, &b.lds, b.waves_most);
      if (b.nwaves) pl->fused = true;
      else {   // back to two launches
        const LdsLayout L2 = lds_layout(WP, F32R, 0, n32, n64, b.nb, b.npi, 1);
        b.wpc = 1;
        b.nwaves = pick_waves(L2, &b.lds, b.waves_most);
      }
    }
    auto carve_fused = [&](Carver &cv) {
      if (!pl->fused) return;
      pl->d_tabx = cv.take<uint2>(pl->xbin.t32.e.size());
      pl->d_Ex = cv.take<double>(xi_nedges);
    };
    Carver dry(nullptr, true);
    batch_carve(dry, *pl, pl->xi);
    batch_carve(dry, *pl, pl->wp);
    carve_fused(dry);
    if (hipMalloc(&pl->mem, dry.off + 256) != hipSuccess) {
      pl->mem = nullptr;
      cp_plan_destroy(pl);
      return fail(CP_ERR_NOMEM, "plan allocation of " + std::to_string(dry.off) + " bytes failed");
    }
    Carver cv(pl->mem, false);
    batch_carve(cv, *pl, pl->xi);
    batch_carve(cv, *pl, pl->wp);
    carve_fused(cv);
    if ((rc = batch_upload(*pl, pl->xi)) || (rc = batch_upload(*pl, pl->wp))) {
      cp_plan_destroy(pl);
      return rc;
    }
    if (pl->fused) {
      const Binning &X = pl->xbin;
      if (hipMemcpy(pl->d_tabx, X.t32.e.data(), 8 * X.t32.e.size(), hipMemcpyHostToDevice) !=
              hipSuccess ||
          hipMemcpy(pl->d_Ex, X.E.data(), 8 * (size_t)xi_nedges, hipMemcpyHostToDevice) !=
              hipSuccess) {
        cp_plan_destroy(pl);
        return fail(CP_ERR_DEVICE, "plan upload failed");
      }
      PairParams &P = pl->wp.P;
      P.wpc = pl->wp.wpc;
      P.tabx = pl->d_tabx;
      P.tabx_lo = X.t32.lo;
      P.tabx_hi = X.t32.hi;
      P.tabx_shift = X.shift;
      P.Ex = pl->d_Ex;
      P.nbx = xi_nedges - 1;
      P.AB32x = X.AB32;
      P.histx = pl->xi.d_hist;
      P.histx_stride = pl->xi.nout;
    }
    for (auto &e : pl->ev) {
      if (hipEventCreate(&e) != hipSuccess) {
        cp_plan_destroy(pl);
        return fail(CP_ERR_DEVICE, "hipEventCreate failed");
      }
    }
    if (hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking) != hipSuccess) {
      cp_plan_destroy(pl);
      return fail(CP_ERR_DEVICE, "hipStreamCreate failed");
    }
    const char *env = getenv("CP_PLAN_NO_GRAPH");
    pl->use_graph = !(env && env[0] == '1');
    *out = pl;
    return CP_OK;
  } catch (...) {
    return fail(CP_ERR_INTERNAL, "unexpected exception");
  }
}

int cp_plan_create(const cp_points *mocks, int nmocks, const double *xi_edges, int xi_nedges,
                   const double *wp_edges, int wp_nedges, double pimax, int npibins,
                   const cp_options *o, cp_plan **out) {
  return plan_create(mocks, nmocks, xi_edges, xi_nedges, wp_edges, wp_nedges, pimax, npibins, o,
                     nullptr, out);
}

int cp_plan_execute(cp_plan *pl, void *stream) {
  if (!pl) return fail(CP_ERR_INVALID_ARG, "plan is NULL");
  hipStream_t st = (hipStream_t)stream;
  pl->last = st;
  if (!pl->use_graph) {
    pl->timed = 1;
    return plan_enqueue(*pl, st, true);
  }
  if (!pl->gexec) {
    // capture the whole pipeline once on the plan's own stream
    (void)hipGetLastError();
    HIPCHK(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
    int rc = plan_enqueue(*pl, pl->cap, false);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(pl->cap, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(CP_ERR_DEVICE, "graph capture failed");
    e = hipGraphInstantiate(&pl->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      pl->gexec = nullptr;
      return fail(CP_ERR_DEVICE, "graph instantiation failed");
    }
  }
  HIPCHK(hipEventRecord(pl->ev[3], st));
  HIPCHK(hipGraphLaunch(pl->gexec, st));
  HIPCHK(hipEventRecord(pl->ev[4], st));
  pl->timed = 2;
  return CP_OK;
}

int cp_plan_results(cp_plan *pl, uint64_t *xi_npairs, uint64_t *wp_npairs) {
  if (!pl) return fail(CP_ERR_INVALID_ARG, "plan is NULL");
  HIPCHK(hipStreamSynchronize(pl->last));
  int flags = 0;
  const double mult = pl->count_mode == CP_ORDERED ? 2 : 1;
  for (int s = 0; s < 2; s++) {
    Batch &b = s ? pl->wp : pl->xi;
    uint64_t *out = s ? wp_npairs : xi_npairs;
    if (!b.on) continue;
    int f = 0;
    HIPCHK(hipMemcpy(&f, b.d_err, sizeof(int), hipMemcpyDeviceToHost));
    flags |= f;
    if (f) continue;
    // every queue item must have been taken (as for single calls; a fused
    // plan's xi shares the w_p launch, checked with w_p)
    if (!(pl->fused && s == 0)) {
      std::vector<unsigned long long> st(kStatWords);
      HIPCHK(hipMemcpy(st.data(), b.d_stats, sizeof(unsigned long long) * kStatWords,
                       hipMemcpyDeviceToHost));
      const int64_t nitems = (int64_t)st[4] * b.P.nsplit;
      for (int k = 0; k < kQueues; k++) {
        const int64_t len = nitems * (k + 1) / kQueues - nitems * k / kQueues;
        if (st[5 + (size_t)k * kQStride] < (unsigned long long)len)
          return fail(CP_ERR_INTERNAL, "work queue not drained");
      }
    }
    if (!out) continue;
    std::vector<unsigned long long> h((size_t)b.nout * pl->nmock);
    HIPCHK(hipMemcpy(h.data(), b.d_hist, 8 * h.size(), hipMemcpyDeviceToHost));
    for (int q = 0; q < pl->nmock; q++) {
      const int m = pl->order[q];
      for (int k = 0; k < b.nout; k++)
        out[(size_t)m * b.nout + k] = (uint64_t)h[(size_t)q * b.nout + k] * (uint64_t)mult;
    }
  }
  return map_err_flags(flags);
}

int cp_plan_stats(cp_plan *pl, cp_stats *xs, cp_stats *ws) {
  if (!pl) return fail(CP_ERR_INVALID_ARG, "plan is NULL");
  HIPCHK(hipStreamSynchronize(pl->last));
  for (int s = 0; s < 2; s++) {
    // a fused plan's xi reports the shared w_p launch (grid, work, timing)
    Batch &b = (s || pl->fused) ? pl->wp : pl->xi;
    cp_stats *o = s ? ws : xs;
    if (!o) continue;
    memset(o, 0, sizeof(*o));
    if (!(s ? pl->wp : pl->xi).on) continue;
    unsigned long long st[kStatWords];
    int nt = 0;
    HIPCHK(hipMemcpy(st, b.d_stats, sizeof(st), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&nt, b.S.coloff + b.ncol_tot, sizeof(int), hipMemcpyDeviceToHost));
    o->candidates = st[0];
    o->rechecks = st[1];
    o->cell_pairs = st[2];
    o->cell_pairs_pruned = st[3];
    o->tiles = nt;
    o->precision = b.prec == F32R ? CP_PREC_FP32_RECHECK : CP_PREC_FP64;
    o->tuned = pl->tuned;
    o->chunk_pct = b.chunk_pct;
    o->waves = b.nwaves;
    for (int a = 0; a < 3; a++) {
      o->grid[a] = b.g.n[a];
      o->refine[a] = b.g.r[a];
    }
    float ms = 0;
    if (pl->timed == 1) {
      const int si = pl->fused ? 1 : s;
      if (hipEventElapsedTime(&ms, pl->ev[si], pl->ev[si + 1]) == hipSuccess) o->ms_pairs = ms;
      if (hipEventElapsedTime(&ms, pl->ev[0], pl->ev[2]) == hipSuccess) o->ms_total = ms;
    } else if (pl->timed == 2) {
      if (hipEventElapsedTime(&ms, pl->ev[3], pl->ev[4]) == hipSuccess) o->ms_total = ms;
    }
    (void)hipGetLastError();
  }
  return CP_OK;
}

} // extern "C"
