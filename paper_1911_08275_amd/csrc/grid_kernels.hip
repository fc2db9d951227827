// Cell-list build on the device: bounding box, cell assignment, counting
// sort into cell-ordered SoA, per-cell bounding boxes and primary tiles.
//
// Section 2.1 ("Creating 3D cells", "Improving cache utilization"): the
// library computes the bounding box of the data, divides it into cells whose
// side is a fraction of R_max (of pi_max along z for wp) and copies each
// cell's points into contiguous per-cell storage.  Section 2.2: each cell
// also keeps the bounding box of its members for the minimum-separation test.
#include "cp_internal.h"

#include <float.h>

namespace cp {

// Error bits raised by the cell build; the host maps them to status codes.
enum { ERRF_NONFINITE = 1, ERRF_OUT_OF_BOX = 2 };

__device__ inline double load_coord(const void *p, int dtype, int64_t i) {
  return dtype == 0 ? ((const double *)p)[i] : (double)((const float *)p)[i];
}

// ------------------------------------------------------------ bounding box

// Partial min/max of up to two point sets; out[blk * 6 + {0..5}] =
// (min x, min y, min z, max x, max y, max z).  Non-finite values set
// ERRF_NONFINITE and are left out.
__global__ __launch_bounds__(256) void k_bbox_partial(PointsDev a, PointsDev b,
                                                      double *out, int *err) {
  double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX};
  double mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int s = 0; s < 2; s++) {
    const PointsDev &P = s ? b : a;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += stride) {
      double v[3] = {load_coord(P.x, P.dtype, i), load_coord(P.y, P.dtype, i),
                     load_coord(P.z, P.dtype, i)};
      bool fin = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
      if (P.w) fin = fin && isfinite(P.w[i]);
      if (!fin) {
        bad = 1;
        continue;
      }
      for (int k = 0; k < 3; k++) {
        mn[k] = fmin(mn[k], v[k]);
        mx[k] = fmax(mx[k], v[k]);
      }
    }
  }
  if (bad) atomicOr(err, ERRF_NONFINITE);
  __shared__ double red[6][256];
  for (int k = 0; k < 3; k++) {
    red[k][threadIdx.x] = mn[k];
    red[k + 3][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int k = 0; k < 3; k++) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[k + 3][threadIdx.x] = fmax(red[k + 3][threadIdx.x], red[k + 3][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) out[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_bbox_final(const double *part, int nblk, double *out) {
  int k = threadIdx.x;
  if (k >= 6) return;
  double v = k < 3 ? DBL_MAX : -DBL_MAX;
  for (int b = 0; b < nblk; b++) v = k < 3 ? fmin(v, part[b * 6 + k]) : fmax(v, part[b * 6 + k]);
  out[k] = v;
}

// --------------------------------------------------------- fills and scans

__global__ void k_fill_i32(int *p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_fill_f64(double *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

struct ScanSeg {
  int64_t in_off;
  int64_t out_off;
  int64_t len;
};

// Exclusive scan of one segment per block: out[0..len] with out[len] = total.
// Each of the 1024 threads sums a contiguous chunk, the block scans the
// chunk sums, then each thread writes its chunk.
__global__ __launch_bounds__(1024) void k_scan_segments(const int *in, int *out,
                                                        const ScanSeg *segs) {
  // Tiles of 4096 values: 4 consecutive values per thread, a shuffle scan
  // inside each wave, the 16 wave totals scanned by wave 0, and a running
  // carry from tile to tile.
  const ScanSeg S = segs[blockIdx.x];
  const int *src = in + S.in_off;
  int *dst = out + S.out_off;
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int carry = 0;
  // the next tile's values are loaded before this tile's barriers, so the
  // memory latency overlaps the scan
  int nv[4];
#pragma unroll
  for (int k = 0; k < 4; k++) nv[k] = 4 * (int64_t)tid + k < S.len ? src[4 * tid + k] : 0;
  for (int64_t t0 = 0; t0 < S.len; t0 += 4096) {
    const int64_t i0 = t0 + 4 * (int64_t)tid;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = nv[k];
    const int64_t n0 = i0 + 4096;
#pragma unroll
    for (int k = 0; k < 4; k++) nv[k] = n0 + k < S.len ? src[n0 + k] : 0;
    const int loc = (v[0] + v[1]) + (v[2] + v[3]);
    int x = loc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
      int t = lane < 16 ? wsum[lane] : 0;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const int y = __shfl_up(t, off);
        if (lane >= off) t += y;
      }
      if (lane < 16) wsum[lane] = t;
    }
    __syncthreads();
    int run = carry + (w > 0 ? wsum[w - 1] : 0) + (x - loc);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (i0 + k < S.len) dst[i0 + k] = run;
      run += v[k];
    }
    carry += wsum[15];
    __syncthreads();
  }
  if (tid == 0) dst[S.len] = carry;
}

// --------------------------------------------------------- cell assignment

// One catalogue per blockIdx.y.  Validates the points (finite; inside
// [0, box) when periodic), computes their cell and takes a rank inside the
// cell with an atomic counter (the order inside a cell is arbitrary; counts
// do not depend on it).
__global__ __launch_bounds__(256) void k_assign(const PointsDev *pts, const GridGeom *geom,
                                                int *cell_count, int *cid, int *rank,
                                                int *err) {
  const PointsDev P = pts[blockIdx.y];
  const GridGeom &G = geom[blockIdx.y];
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v[3] = {load_coord(P.x, P.dtype, i), load_coord(P.y, P.dtype, i),
                   load_coord(P.z, P.dtype, i)};
    int c[3];
    for (int a = 0; a < 3; a++) {
      if (!isfinite(v[a])) bad |= ERRF_NONFINITE;
      else if (G.periodic && (v[a] < 0.0 || v[a] >= G.box)) bad |= ERRF_OUT_OF_BOX;
      c[a] = cell_coord(G, a, v[a]);
    }
    if (P.w && !isfinite(P.w[i])) bad |= ERRF_NONFINITE;
    int cell = (c[0] * G.n[1] + c[1]) * G.n[2] + c[2];
    cid[G.pbase + i] = cell;
    rank[G.pbase + i] = atomicAdd(&cell_count[G.cbase + cell], 1);
  }
  if (bad) atomicOr(err, bad);
}

// Cell order, z ascending inside each cell (Section 2.1 contiguous per-cell
// storage and z-sorted cells, used by the late entry / early exit of Section 2.2).  k_group
// copies every point's (x, y, z, w) to its cell's range in the atomic order;
// k_cellfin, one wave per cell, ranks the cell's points by z (ties by grouped
// position, so the ranks form a permutation), writes them in that order
// together with their binary32 stream records, and takes the cell's bounding
// box.  Cells above kZSortMax points keep the grouped order.
__global__ __launch_bounds__(256) void k_group(const PointsDev *pts, const GridGeom *geom,
                                               const int *cstart, const int *cid,
                                               const int *rank, double4 *grp) {
  const PointsDev P = pts[blockIdx.y];
  const GridGeom &G = geom[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int cell = cid[G.pbase + i];
    const int64_t k = G.pbase + cstart[G.sbase + cell] + rank[G.pbase + i];
    grp[k] = make_double4(load_coord(P.x, P.dtype, i), load_coord(P.y, P.dtype, i),
                          load_coord(P.z, P.dtype, i), P.w ? P.w[i] : 1.0);
  }
}

// Stream record of a point in the frame of its own cell (centre O):
//   xi: (-2 px, -2 py, -2 pz, |p|^2)      wp: (-2 px, -2 py, pz, px^2 + py^2)
// with p = fl32(x - O).
__device__ inline float4 stream_record(const GridGeom &G, int cell, const double4 &v, int mode) {
  const int cz = cell % G.n[2];
  const int cy = (cell / G.n[2]) % G.n[1];
  const int cx = cell / (G.n[2] * G.n[1]);
  const float px = (float)(v.x - frame_origin(G, 0, cx));
  const float py = (float)(v.y - frame_origin(G, 1, cy));
  const float pz = (float)(v.z - frame_origin(G, 2, cz));
  float4 s;
  s.x = -2.0f * px;
  s.y = -2.0f * py;
  if (mode == XI) {
    s.z = -2.0f * pz;
    s.w = __builtin_fmaf(pz, pz, __builtin_fmaf(py, py, px * px));
  } else {
    s.z = pz;
    s.w = __builtin_fmaf(py, py, px * px);
  }
  return s;
}

constexpr int kZChunk = 256;    // z values staged in LDS per step, per wave

// NP points per lane: rank by a broadcast scan over the staged z values,
// then write them (and their stream records) at b + rank; min/max update.
template <int NP>
__device__ inline void cellfin_pass(const GridGeom &G, int cell, const double4 *grp,
                                    int64_t base, int n, int q0, int lane, double *zw,
                                    double4 *pos, float4 *strm, int mode, double mn[3],
                                    double mx[3]) {
  double4 v[NP];
  int kq[NP], r[NP];
#pragma unroll
  for (int p = 0; p < NP; p++) {
    kq[p] = q0 + p * 64 + lane;
    v[p] = kq[p] < n ? grp[base + kq[p]] : make_double4(0.0, 0.0, 0.0, 0.0);
    r[p] = kq[p];
  }
  if (n <= kZSortMax) {
#pragma unroll
    for (int p = 0; p < NP; p++) r[p] = 0;
    for (int c0 = 0; c0 < n; c0 += kZChunk) {
      const int cnt = min(kZChunk, n - c0);
      if (q0 == 0 || n > kZChunk) {   // (re)stage this chunk
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int t = lane; t < cnt; t += 64) zw[t] = grp[base + c0 + t].z;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll 4
      for (int t = 0; t < cnt; t++) {
        const double zj = zw[t];
#pragma unroll
        for (int p = 0; p < NP; p++)
          r[p] += (zj < v[p].z || (zj == v[p].z && c0 + t < kq[p])) ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int p = 0; p < NP; p++) {
    if (kq[p] < n) {
      pos[base + r[p]] = v[p];
      strm[base + r[p]] = stream_record(G, cell, v[p], mode);
      mn[0] = fmin(mn[0], v[p].x); mx[0] = fmax(mx[0], v[p].x);
      mn[1] = fmin(mn[1], v[p].y); mx[1] = fmax(mx[1], v[p].y);
      mn[2] = fmin(mn[2], v[p].z); mx[2] = fmax(mx[2], v[p].z);
    }
  }
}

__global__ __launch_bounds__(256) void k_cellfin(const GridGeom *geom, int nmock,
                                                 const int *cstart, const double4 *grp,
                                                 double4 *pos, float4 *strm, CellBox *cbox,
                                                 const int64_t *cell_prefix, int mode) {
  __shared__ double zsh[4][kZChunk];
  const int w = threadIdx.x >> 6;
  const int wid = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  double *zw = zsh[w];
  const int64_t total = cell_prefix[nmock];
  for (int64_t gc = wid; gc < total; gc += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    int lo = 0, hi = nmock - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (cell_prefix[mid] <= gc) lo = mid; else hi = mid - 1;
    }
    const GridGeom &G = geom[lo];
    const int c = (int)(gc - cell_prefix[lo]);
    const int b = cstart[G.sbase + c], e = cstart[G.sbase + c + 1];
    const int n = e - b;
    const int64_t base = G.pbase + b;
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    if (n <= 64) {
      cellfin_pass<1>(G, c, grp, base, n, 0, lane, zw, pos, strm, mode, mn, mx);
    } else {
      for (int q0 = 0; q0 < n; q0 += 4 * 64)
        cellfin_pass<4>(G, c, grp, base, n, q0, lane, zw, pos, strm, mode, mn, mx);
    }
    for (int off = 32; off > 0; off >>= 1) {
      for (int a = 0; a < 3; a++) {
        mn[a] = fmin(mn[a], __shfl_xor(mn[a], off));
        mx[a] = fmax(mx[a], __shfl_xor(mx[a], off));
      }
    }
    if (lane == 0) {
      CellBox B;
      for (int a = 0; a < 3; a++) {
        B.lo[a] = mn[a];
        B.hi[a] = mx[a];
      }
      cbox[G.cbase + c] = B;
    }
  }
}

// ------------------------------------------------------------------ tiles

// Packing of each column's z-run of points into tiles: consecutive runs of
// at most 64 points (cells may be cut anywhere) whose cells span at most
// maxspan z-cells, so every lane holds a point whenever the column allows.
// emit = 0: count tiles per column; emit = 1: write them at the offsets of
// the scanned counts.
__device__ inline void walk_column(const GridGeom &G, const int *cs, int col, int maxspan,
                                   int mock, int emit, Tile *out, int64_t &ntile) {
  // cs[z] = start of z-cell z of the column (z = 0..nz), relative to the set
  const int nz = G.n[2];
  const int pend = cs[nz];
  int p = cs[0];
  int z = 0;   // cell of point p
  while (p < pend) {
    while (cs[z + 1] <= p) z++;
    // furthest cell allowed by the span limit, and its end
    const int zmax = min(nz - 1, z + maxspan - 1);
    const int lim = cs[zmax + 1];
    const int q = min(p + kTileMax, lim);
    int z1 = z;
    while (cs[z1 + 1] < q) z1++;
    if (emit) {
      Tile T;
      T.p0 = G.pbase + p;
      T.n = q - p;
      T.mock = mock;
      T.col = col;
      T.cz0 = z;
      T.cz1 = z1;
      T.pad = 0;
      out[ntile] = T;
    }
    ntile++;
    p = q;
  }
}

// Queue position of a column: blocks of 4 x 4 columns, block rows along x,
// so the tiles the waves of one XCD work on at the same time (a contiguous
// stretch of its share of the queue) sit in a compact patch of columns and
// share their neighbour cells in that XCD's L2.  A bijection on the columns.
__device__ inline int column_rank(int col, int nx, int ny) {
  constexpr int B = 4;
  const int cx = col / ny, cy = col % ny;
  const int bx = cx / B, by = cy / B;
  const int w = min(B, nx - bx * B), h = min(B, ny - by * B);
  return bx * B * ny + by * B * w + (cx - bx * B) * h + (cy - by * B);
}

// One wave per column: the column's cell starts are staged in the wave's LDS
// slice, then one lane walks them.  Counts and offsets are indexed by the
// column's queue position.
__global__ __launch_bounds__(256) void k_tiles(const GridGeom *geom, int nmock,
                                               const int *cstart, const int *maxspan,
                                               const int64_t *col_prefix, int *colcnt,
                                               const int *coloff, Tile *tiles, int emit) {
  __shared__ int csh[4][kMaxAxisCells + 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int *cs = csh[w];
  const int64_t total = col_prefix[nmock];
  for (int64_t gcol = wid; gcol < total; gcol += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    int lo = 0, hi = nmock - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (col_prefix[mid] <= gcol) lo = mid; else hi = mid - 1;
    }
    const GridGeom &G = geom[lo];
    const int col = (int)(gcol - col_prefix[lo]);
    const int nz = G.n[2];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int z = lane; z <= nz; z += 64) cs[z] = cstart[G.sbase + col * nz + z];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      const int64_t q = col_prefix[lo] + column_rank(col, G.n[0], G.n[1]);
      int64_t n = emit ? coloff[q] : 0;
      walk_column(G, cs, col, maxspan[lo], lo, emit, tiles, n);
      if (!emit) colcnt[q] = (int)n;
    }
  }
}

} // namespace cp
