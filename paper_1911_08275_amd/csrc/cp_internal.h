// Internal types shared by the host side and the kernels of libcountpairs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace cp {

constexpr int kWave = 64;
constexpr int kTileMax = 64;        // points per primary tile (one per lane)
constexpr int kMaxAxisCells = 1023; // cells per axis (packed in 10 bits)
constexpr int kMaxBins = 60;        // separation bins; slots 0 and nb+1 are trash and
                                    // slot + 1 must fit the 6-bit table code
constexpr int kMaxPiBins = 256;
constexpr int kZSortMax = 4096;   // cells up to this many points are z-sorted
constexpr int kSortWin = 128;     // grouped positions per wave of the z-order pass
constexpr int kColLds = 8192;     // columns up to which the build groups points through LDS
constexpr int kColBlocks = 256;   // most blocks of that grouping (matrix of kColBlocks x columns)
// Blocks of the LDS column grouping for n points: chunks of at least 2048.
__host__ __device__ inline int col_blocks(int64_t n) {
  const int64_t b = (n + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > kColBlocks ? kColBlocks : b));
}
// Work queues of the pair kernel: one per XCD (workgroups are dealt to the
// MI355X's 8 XCDs round-robin, so blockIdx.x % 8 names the XCD), each
// holding a contiguous, hence spatially compact, share of the items; a wave
// drains its own queue first, so a cell's records are reused from its XCD's
// L2, then helps the others.
constexpr int kQueues = 8;
// Statistics words: candidates, rechecks, cell pairs, pruned, tile count,
// then the kQueues queue heads, kQStride words (4 KB) apart so that their
// device-scope atomics land in different memory channels.  Packed into one
// 64-byte line the heads handed out at most ~86 items per microsecond in all,
// which bounded launches of many light items (measured: xi at R_max = 10 took
// 1.25 ms with packed heads, 0.71 ms with spread ones).
constexpr int kQStride = 512;
constexpr int kStatWords = 5 + kQueues * kQStride;
// Most queue items per tile (chunks of the tile's neighbour-column list).
constexpr int kMaxChunks = 32;
constexpr int kStaticLds = 256;  // LDS the pair kernel declares statically (queue mask)
constexpr int kWStripe = 8;       // copies of each weight sum per wave (lane & 7)

// Cell counters of the build: one per cell, kCountStride ints apart.
constexpr int kCountStride = 1;

// Segmented exclusive scans (cell counts -> cell starts, tile counts -> tile
// offsets): out[out_off + k] = sum of the first k of the segment's len values
// in[(in_off + j) * stride], and out[out_off + len] = their total.  Tiles of
// kScanTile values, numbered across the segments of one launch from tile0.
constexpr int kScanTile = 4096;
struct ScanSeg {
  int64_t in_off;
  int64_t out_off;
  int64_t len;
  int64_t tile0;
  int64_t stride;
};
__host__ __device__ inline int64_t scan_tiles(int64_t len) {
  return len > 0 ? (len + kScanTile - 1) / kScanTile : 1;
}

// Sets the calling thread's countpairs_last_error text and returns code.
int report_error(int code, const char *msg);

// Autotuned launch settings of one workload signature (tune_cache.cpp).
struct TuneChoice {
  int refine[3] = {2, 2, 2};
  int chunk_pct = 100;   // scale of the queue items' work-chunk target, percent
  int waves = 4;         // most waves per pair-kernel workgroup
  double ms = 0.0;       // device time of the tuned call
};
bool tune_lookup(const std::string &key, TuneChoice &out);
void tune_store(const std::string &key, const TuneChoice &t);
std::string tune_cache_file();

// WPXI: w_p and xi of the same catalogues in one pass over the w_p search
// (binary32 mode; every xi pair lies inside the w_p cylinder when the xi
// R_max is at most both r_p,max and pi_max).  Where the kernel tests
// MODE == XI, WPXI takes the w_p side.
enum Mode { XI = 0, WP = 1, WPXI = 2 };
enum Prec { F64 = 0, F32R = 1 };

// Geometry of one catalogue's cell grid.  Cells are ordered x-major, z
// fastest: cell = (cx * ny + cy) * nz + cz, so a run of z-cells in one
// (x, y) column is contiguous in the sorted point arrays.
struct GridGeom {
  int n[3];        // cells per axis
  int r[3];        // neighbour reach in cells per axis
  int wrap[3];     // 1: single periodic cell on this axis, per-pair minimum image
  int periodic;
  double lo[3];    // domain origin
  double cs[3];    // cell side
  double inv[3];   // 1 / cell side
  double box;      // periodic side
  double halfbox;
  int64_t pbase;   // first sorted point of this catalogue
  int64_t cbase;   // first entry of this catalogue in cell arrays
  int64_t sbase;   // first entry of this catalogue in cell_start (ncell + 1 per catalogue)
  int64_t npts;
  int ncell;
  int ncol;
  int64_t colbase; // first entry of this catalogue in per-column arrays
  int64_t mbase;   // first entry of this catalogue's column x block matrix (column build)
  int nblk;        // blocks of the column build for this catalogue
};

// Input point set on the device (one catalogue).
struct PointsDev {
  const void *x, *y, *z;
  const double *w;
  int64_t n;
  int dtype;       // 0 f64, 1 f32
  int pad;
};

struct CellBox {
  double lo[3];
  double hi[3];
};

// A primary tile: <= 64 consecutive sorted points of one column whose cells
// span z-cells [cz0, cz1].
struct Tile {
  int64_t p0;      // first sorted point (absolute)
  int n;           // points in the tile
  int mock;        // catalogue index
  int col;         // column cx * ny + cy
  int cz0, cz1;
  int pad;
};

struct PairParams {
  // work queue
  const Tile *tiles;
  const int *ntiles;         // device: number of tiles in the queue
  int nsplit;                // queue items per tile: chunks of its neighbour-column list
  int chunk[kMaxChunks + 1]; // chunk k covers list columns [chunk[k], chunk[k + 1])
  // geometry (indexed by tile.mock); set 2 is the searched (streamed) set
  const GridGeom *geom1;
  const GridGeom *geom2;
  const double4 *pos1;       // sorted (x, y, z, w) of set 1 (tiles)
  const double4 *pos2;       // sorted (x, y, z, w) of set 2
  const float4 *strm2;       // sorted cell-local binary32 stream of set 2
  const int *cstart2;        // cell starts of set 2 (relative to pbase)
  const CellBox *cbox2;      // cell bounding boxes of set 2
  // binning
  const uint2 *tab32;        // binary32 decision table (FP32 mode)
  const uint2 *tab64;        // decision table for fl32(s64) (FP64 values)
  int tab32_lo, tab32_hi, tab64_lo, tab64_hi;
  int tab_shift;
  const double *E;           // squared edges, nb + 1
  const float *C32, *A32;    // binary32 band of each edge: v < C proves s < E,
                             // v >= A proves s >= E (nb + 1 each)
  int nb;                    // separation bins
  int nslots;                // nb + 2
  float AB32;                // binary32 s~ >= AB32 -> certainly >= E_B
  float eps32;               // binary32 bound on |(s~ - E_t) - (s - E_t)| of the
                             // folded two-slot evaluation (rounded up)
  float eps32_3;             // the same for the three-slot evaluation, whose second
                             // difference is formed from the first (adds 2 u E_B)
  double EB;                 // E_B
  // wp
  double pimax, dpi, inv_dpi;   // inv_dpi = fl(1 / dpi)
  int npi;
  int wpc;                   // copies of the wave's histogram (power of two)
  float inv_dpi32, pi_delta, pi_hi32;
  float pi_delta64;          // pi band of the binary64 loops' binary32 pi bin
  // flags
  int autocorr;
  int weighted;
  int noprune;               // 1: no unit is skipped or narrowed by its bounding box
  // outputs (per catalogue)
  unsigned long long *hist;  // [nmock][nb * npi]
  double *hw;                // [nmock][nb * npi] sum of weights
  double *hwr;               // [nmock][nb * npi] sum of weight * separation
  unsigned long long *stats; // kStatWords: candidates, rechecks, cell pairs, pruned,
                             // tile count (written by the pair kernel), queue heads
  int hist_stride;           // nb * npi
  // xi of a WPXI launch: decision table of s~ = fl32(pi~^2 + rp~^2) (bands
  // of its own error bound), squared edges, histogram
  const uint2 *tabx;
  int tabx_lo, tabx_hi, tabx_shift;
  const double *Ex;          // nbx + 1
  int nbx;
  float AB32x;               // s~ >= AB32x -> certainly >= the last xi edge
  unsigned long long *histx; // [nmock][nbx]
  int histx_stride;
};

} // namespace cp

namespace cp {

// Frame origin of a cell along axis a: the cell centre in binary64.  The
// cell build and the pair kernels must evaluate this identically (same
// expression, no contraction) so binary32 offsets from it are consistent.
__host__ __device__ inline double frame_origin(const GridGeom &g, int a, int c) {
  double t = ((double)c + 0.5) * g.cs[a];
  return g.lo[a] + t;
}

__host__ __device__ inline int cell_coord(const GridGeom &g, int a, double v) {
  double t = (v - g.lo[a]) * g.inv[a];
  if (!(t >= 0.0)) return 0;              // also NaN (rejected elsewhere)
  if (t >= (double)g.n[a]) return g.n[a] - 1;
  return (int)t;                          // t >= 0: truncation is floor
}

// LDS layout of the pair kernel, shared by the host (launch size) and the
// device: decision tables and squared edges, then per wave the lane-private
// counters and the weight sums.
__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

struct LdsLayout {
  size_t tab32, tab64, E, tabx, Ex, common, wave_hist, wave_w, wave_list, wave_histx, wave_bytes;
};

// Weighted xi with the binary32 filter: the filter needs no decision table
// (it only tests s~ against the band above E_B), and every pair it passes
// goes to a per-wave list of (tile lane, record) pairs that is evaluated in
// binary64, 64 pairs at a time.
__host__ __device__ constexpr bool xi_f32_weighted(int mode, int prec, int weighted) {
  return mode == XI && prec == F32R && weighted;
}
// List entries per wave: fewer than 64 are left over after a drain, and a
// group of four records adds at most 4 x 64.
constexpr int kListCap = 64 + 4 * 64;

// wpc: copies of the w_p histogram (and weight sums) per wave, interleaved
// counter by counter; lane l adds to copy l mod wpc.  nx, nbx: the xi table
// entries and bins of a WPXI launch (xi rows, one per lane pair, follow the
// w_p histogram).
__host__ __device__ inline LdsLayout lds_layout(int mode, int prec, int weighted, int n32, int n64,
                                               int nb, int npi, int wpc = 1, int nx = 0,
                                               int nbx = 0) {
  LdsLayout L;
  size_t off = 0;
  L.tab32 = off;
  if (xi_f32_weighted(mode, prec, weighted)) n32 = 0;
  off += (size_t)(prec == F32R ? n32 : 0) * 8;
  L.tab64 = off;
  off += (size_t)n64 * 8;
  L.E = off;
  off += (size_t)(nb + 1) * 8;
  L.tabx = off;
  L.Ex = off;
  if (mode == WPXI) {
    off += (size_t)nx * 8;
    L.Ex = off;
    off += (size_t)(nbx + 1) * 8;
  }
  L.common = align16(off);
  const int NS = nb + 2;
  const size_t words = mode == XI ? (size_t)NS * 64 : (size_t)NS * npi * wpc;
  L.wave_hist = align16(words * 4);
  // weight sums are shared by the wave (one row of slots), not lane-private
  L.wave_w = weighted ? (mode == XI ? (size_t)NS * kWStripe : words) * 8 : 0;
  L.wave_list = L.wave_hist + 2 * L.wave_w;
  L.wave_histx = L.wave_list + (xi_f32_weighted(mode, prec, weighted) ? (size_t)kListCap * 4 : 0);
  L.wave_bytes = L.wave_histx + (mode == WPXI ? (size_t)(nbx + 2) * 32 * 4 : 0);
  return L;
}

} // namespace cp
