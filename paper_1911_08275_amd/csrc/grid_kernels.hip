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
#include <limits.h>

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

// Zero two ranges in one launch.
__global__ void k_fill2_i32(int *a, int64_t na, int *b, int64_t nb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < na) a[i] = 0;
    else b[i - na] = 0;
  }
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

// Segment of launch tile b (segments ordered by tile0).
__device__ inline int scan_segment(const ScanSeg *segs, int nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].tile0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Values of one scan tile held by thread tid: four runs of four consecutive
// values, run g at tile offset g * 1024 + 4 tid (coalesced), zero past len.
// Loads use clamped indices so that all sixteen are in flight together.
__device__ inline void scan_load(const int *in, const ScanSeg &S, int64_t base, int tid,
                                 int (&v)[4][4]) {
#pragma unroll
  for (int g = 0; g < 4; g++)
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t j = base + g * 1024 + 4 * tid + k;
      v[g][k] = in[(S.in_off + min(j, S.len - 1)) * S.stride];
    }
#pragma unroll
  for (int g = 0; g < 4; g++)
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (base + g * 1024 + 4 * tid + k >= S.len) v[g][k] = 0;
}

__device__ inline int block_sum256(int x, int *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  const int t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Pass 1 of the segmented scans: the total of every tile (one block each).
__global__ __launch_bounds__(256) void k_scan_sums(const int *in, const ScanSeg *segs, int nseg,
                                                   int *tsum) {
  __shared__ int red[4];
  const int64_t b = blockIdx.x;
  const ScanSeg S = segs[scan_segment(segs, nseg, b)];
  if (S.len == 0) {
    if (threadIdx.x == 0) tsum[b] = 0;
    return;
  }
  int v[4][4];
  scan_load(in, S, (b - S.tile0) * kScanTile, threadIdx.x, v);
  int x = 0;
#pragma unroll
  for (int g = 0; g < 4; g++) x += (v[g][0] + v[g][1]) + (v[g][2] + v[g][3]);
  x = block_sum256(x, red);
  if (threadIdx.x == 0) tsum[b] = x;
}

// Pass 2: every tile scanned at once (one block each), starting from the sum
// of its segment's earlier tiles; the segment's last tile writes the total.
__global__ __launch_bounds__(256) void k_scan_apply(const int *in, int *out, const ScanSeg *segs,
                                                    int nseg, const int *tsum) {
  __shared__ int red[4];
  __shared__ int wsum[16];
  const int64_t b = blockIdx.x;
  const ScanSeg S = segs[scan_segment(segs, nseg, b)];
  int *dst = out + S.out_off;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (S.len == 0) {
    if (tid == 0) dst[0] = 0;
    return;
  }
  const int64_t base = (b - S.tile0) * kScanTile;
  int v[4][4];
  scan_load(in, S, base, tid, v);
  int c = 0;
  for (int64_t u = S.tile0 + tid; u < b; u += 256) c += tsum[u];
  const int carry = block_sum256(c, red);
  int loc[4], x[4];
#pragma unroll
  for (int g = 0; g < 4; g++) {
    loc[g] = (v[g][0] + v[g][1]) + (v[g][2] + v[g][3]);
    x[g] = loc[g];
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
    for (int g = 0; g < 4; g++) {
      const int y = __shfl_up(x[g], off);
      if (lane >= off) x[g] += y;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int g = 0; g < 4; g++) wsum[g * 4 + w] = x[g];
  }
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
#pragma unroll
  for (int g = 0; g < 4; g++) {
    const int q = g * 4 + w;
    int run = carry + (q > 0 ? wsum[q - 1] : 0) + (x[g] - loc[g]);
    const int64_t i0 = base + g * 1024 + 4 * (int64_t)tid;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (i0 + k < S.len) dst[i0 + k] = run;
      run += v[g][k];
    }
  }
  if (tid == 0 && base + kScanTile >= S.len) dst[S.len] = carry + wsum[15];
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
    rank[G.pbase + i] = atomicAdd(&cell_count[(G.cbase + cell) * kCountStride], 1);
  }
  if (bad) atomicOr(err, bad);
}

// ------------------------------------------------- column grouping (LDS)
//
// The same grouping without any device-scope atomic, when a block's LDS
// holds one counter per (x, y) column.  Each of nb blocks takes a contiguous
// chunk of its catalogue's points; pass 1 counts the chunk per column in LDS
// and writes the counts to a column-major matrix M[col * nb + block]; the
// exclusive scan of M gives, for every (column, block), where that block's
// points of that column start in column order (so M'[col * nb] is the
// column's start and the scan's total its end); pass 2 ranks each block's
// points inside their column with LDS atomics and writes them in column
// order; pass 3, one workgroup per column, counts the column's points per
// z-cell in LDS, writes the cell starts and moves the points to their cells.
// Order inside a cell is arbitrary, as with k_assign.

__device__ inline int column_of(const GridGeom &G, double x, double y) {
  return cell_coord(G, 0, x) * G.n[1] + cell_coord(G, 1, y);
}

// Chunk of a catalogue's points taken by block b of nb.
__device__ inline void block_chunk(int64_t n, int b, int nb, int64_t &i0, int64_t &i1) {
  const int64_t per = (n + nb - 1) / nb;
  i0 = min(n, (int64_t)b * per);
  i1 = min(n, i0 + per);
}

// One catalogue per blockIdx.y, its G.nblk blocks along x (blocks beyond
// them return), its matrix at mat + G.mbase.
// Pass 1 (validates the points as k_assign does).
__global__ __launch_bounds__(1024) void k_colcount(const PointsDev *pts, const GridGeom *geom,
                                                   int *mat, int *err) {
  __shared__ int h[kColLds];
  const PointsDev P = pts[blockIdx.y];
  const GridGeom &G = geom[blockIdx.y];
  const int ncol = G.n[0] * G.n[1], nb = G.nblk;
  if ((int)blockIdx.x >= nb) return;   // uniform over the block
  mat += G.mbase;
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) h[c] = 0;
  __syncthreads();
  int64_t i0, i1;
  block_chunk(P.n, blockIdx.x, nb, i0, i1);
  int bad = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double v[3] = {load_coord(P.x, P.dtype, i), load_coord(P.y, P.dtype, i),
                         load_coord(P.z, P.dtype, i)};
    for (int a = 0; a < 3; a++) {
      if (!isfinite(v[a])) bad |= ERRF_NONFINITE;
      else if (G.periodic && (v[a] < 0.0 || v[a] >= G.box)) bad |= ERRF_OUT_OF_BOX;
    }
    if (P.w && !isfinite(P.w[i])) bad |= ERRF_NONFINITE;
    atomicAdd(&h[column_of(G, v[0], v[1])], 1);
  }
  if (bad) atomicOr(err, bad);
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) mat[(int64_t)c * nb + blockIdx.x] = h[c];
}

// Pass 2: off = the scanned matrix; out: (x, y, z, w) in column order.
__global__ __launch_bounds__(1024) void k_colscatter(const PointsDev *pts, const GridGeom *geom,
                                                     const int *off, double4 *out) {
  __shared__ int base[kColLds];
  const PointsDev P = pts[blockIdx.y];
  const GridGeom &G = geom[blockIdx.y];
  const int ncol = G.n[0] * G.n[1], nb = G.nblk;
  if ((int)blockIdx.x >= nb) return;   // uniform over the block
  off += G.mbase;
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) base[c] = off[(int64_t)c * nb + blockIdx.x];
  __syncthreads();
  int64_t i0, i1;
  block_chunk(P.n, blockIdx.x, nb, i0, i1);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double x = load_coord(P.x, P.dtype, i), y = load_coord(P.y, P.dtype, i);
    const int k = atomicAdd(&base[column_of(G, x, y)], 1);
    out[G.pbase + k] = make_double4(x, y, load_coord(P.z, P.dtype, i), P.w ? P.w[i] : 1.0);
  }
}

// Cell order, z ascending inside each cell (Section 2.1 contiguous per-cell
// storage and z-sorted cells, used by the late entry / early exit of Section
// 2.2).  k_group copies every point's (x, y, z, w) to its cell's range in the
// atomic order; k_cellsort ranks each point by z inside its cell (ties by
// grouped position, so the ranks form a permutation), writes it in that order
// together with its binary32 stream record, and takes the cell's bounding
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
__device__ inline float4 stream_record(const GridGeom &G, int cx, int cy, int cz,
                                       const double4 &v, int mode) {
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

// Each wave takes a window of kSortWin consecutive grouped positions of one
// catalogue (kSortWin / 64 per lane).  A lane finds its point's cell from the
// coordinates (the cell k_assign computed, by the same function) and the
// cell's range [cb, ce) from the scanned counts; its z rank is the number of
// cell members that precede it in (z, grouped position) order: members at
// earlier positions with z <= its z, later ones with z < its z.  The wave
// stages the z of every cell its window touches in its LDS slice, kSortStage
// values at a time, and each lane scans its own cell's part of the stage.
//
// Bounding box: z from the ends of the z order (the lanes of rank 0 and
// n - 1), x and y from a segmented min/max over consecutive positions (the
// cells are contiguous runs) carried from block to block of the window; the
// window holding a cell's first position owns it and, when the cell runs past
// the window's end, reduces the rest of it too.  Every field of a box is
// written by exactly one lane.  Cells above kZSortMax points keep the grouped
// order, and their owner reduces all six extents over the whole cell.
// Every window's wave is independent (no workgroup barrier).
constexpr int kSortStage = 512;

// min/max of (x, y) in a/b folded over a segmented shuffle step
__device__ inline void fold_xy(double (&a)[2], double (&b)[2], int off, bool take) {
  double t[4];
  t[0] = __shfl_up(a[0], off);
  t[1] = __shfl_up(a[1], off);
  t[2] = __shfl_up(b[0], off);
  t[3] = __shfl_up(b[1], off);
  if (take) {
    a[0] = fmin(a[0], t[0]);
    a[1] = fmin(a[1], t[1]);
    b[0] = fmax(b[0], t[2]);
    b[1] = fmax(b[1], t[3]);
  }
}

__global__ __launch_bounds__(256) void k_cellsort(const GridGeom *geom, int nmock,
                                                  const int *cstart, const double4 *grp,
                                                  double4 *pos, float4 *strm, CellBox *cbox,
                                                  const int64_t *win_prefix, int mode) {
  constexpr int NP = kSortWin / 64;
  __shared__ double szz[4][kSortStage];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *zz = szz[w];
  const int64_t total = win_prefix[nmock];
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + w; gw < total; gw += stride) {
    int m = 0, hi = nmock - 1;
    while (m < hi) {
      const int mid = (m + hi + 1) >> 1;
      if (win_prefix[mid] <= gw) m = mid; else hi = mid - 1;
    }
    const GridGeom &G = geom[m];
    const int64_t pb = G.pbase;
    const int *cs = cstart + G.sbase;
    const int p0 = (int)(gw - win_prefix[m]) * kSortWin;
    const int p1 = (int)min((int64_t)p0 + kSortWin, G.npts);
    double4 v[NP];
    int cell[NP], cb[NP], ce[NP], r[NP];
    int rlo = INT_MAX, rhi = INT_MIN;
    // loads at clamped positions, issued together (no branch between them)
#pragma unroll
    for (int k = 0; k < NP; k++) v[k] = grp[pb + min(p0 + k * 64 + lane, p1 - 1)];
#pragma unroll
    for (int k = 0; k < NP; k++) {
      cell[k] = (cell_coord(G, 0, v[k].x) * G.n[1] + cell_coord(G, 1, v[k].y)) * G.n[2] +
                cell_coord(G, 2, v[k].z);
      cb[k] = cs[cell[k]];
      ce[k] = cs[cell[k] + 1];
    }
#pragma unroll
    for (int k = 0; k < NP; k++) {
      const int i = p0 + k * 64 + lane;
      r[k] = 0;
      if (i < p1) {
        if (ce[k] - cb[k] <= kZSortMax) {
          rlo = min(rlo, cb[k]);
          rhi = max(rhi, ce[k]);
        }
      } else {
        cb[k] = -1;
        ce[k] = 0;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      rlo = min(rlo, __shfl_xor(rlo, off));
      rhi = max(rhi, __shfl_xor(rhi, off));
    }
    // z ranks
    for (int c0 = rlo; c0 < rhi; c0 += kSortStage) {
      const int cnt = min(kSortStage, rhi - c0);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      {
        // all of the stage's loads in flight at once (clamped positions)
        double zt[kSortStage / 64];
#pragma unroll
        for (int u = 0; u < kSortStage / 64; u++)
          zt[u] = grp[pb + c0 + min(lane + 64 * u, cnt - 1)].z;
#pragma unroll
        for (int u = 0; u < kSortStage / 64; u++)
          if (lane + 64 * u < cnt) zz[lane + 64 * u] = zt[u];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int k = 0; k < NP; k++) {
        const int i = p0 + k * 64 + lane;
        if (i < p1 && ce[k] - cb[k] <= kZSortMax) {
          const int a = max(cb[k], c0) - c0, e = min(ce[k], c0 + cnt) - c0;
          const int me = i - c0;
          const double zi = v[k].z;
          int rk = 0;
          // earlier positions: z <= zi
          const int e1 = min(e, me);
          int t = a;
          for (; t + 4 <= e1; t += 4) {
            rk += (zz[t] <= zi ? 1 : 0) + (zz[t + 1] <= zi ? 1 : 0);
            rk += (zz[t + 2] <= zi ? 1 : 0) + (zz[t + 3] <= zi ? 1 : 0);
          }
          for (; t < e1; t++) rk += zz[t] <= zi ? 1 : 0;
          // later positions: z < zi
          t = max(a, me + 1);
          for (; t + 4 <= e; t += 4) {
            rk += (zz[t] < zi ? 1 : 0) + (zz[t + 1] < zi ? 1 : 0);
            rk += (zz[t + 2] < zi ? 1 : 0) + (zz[t + 3] < zi ? 1 : 0);
          }
          for (; t < e; t++) rk += zz[t] < zi ? 1 : 0;
          r[k] += rk;
        }
      }
    }
    // x, y extents: segmented min/max over the window's consecutive
    // positions, carried from block to block (segment id: the cell start)
    double cmn[2] = {DBL_MAX, DBL_MAX}, cmx[2] = {-DBL_MAX, -DBL_MAX};
    int ccb = -2;   // cell of the carry
#pragma unroll
    for (int k = 0; k < NP; k++) {
      const int i = p0 + k * 64 + lane;
      const bool ok = i < p1;
      double mn[2] = {ok ? v[k].x : DBL_MAX, ok ? v[k].y : DBL_MAX};
      double mx[2] = {ok ? v[k].x : -DBL_MAX, ok ? v[k].y : -DBL_MAX};
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int ocb = __shfl_up(cb[k], off);
        fold_xy(mn, mx, off, lane >= off && ocb == cb[k]);
      }
      if (ok && cb[k] == ccb) {
        mn[0] = fmin(mn[0], cmn[0]);
        mn[1] = fmin(mn[1], cmn[1]);
        mx[0] = fmax(mx[0], cmx[0]);
        mx[1] = fmax(mx[1], cmx[1]);
      }
      if (ok) {
        const int n = ce[k] - cb[k];
        const bool sorted = n <= kZSortMax;
        const int rk = sorted ? r[k] : i - cb[k];
        const int64_t d = pb + cb[k] + rk;
        pos[d] = v[k];
        const int cz = cell[k] % G.n[2], cxy = cell[k] / G.n[2];
        strm[d] = stream_record(G, cxy / G.n[1], cxy % G.n[1], cz, v[k], mode);
        CellBox *B = cbox + G.cbase + cell[k];
        if (sorted) {
          if (rk == 0) B->lo[2] = v[k].z;
          if (rk == n - 1) B->hi[2] = v[k].z;
          if (i == ce[k] - 1 && cb[k] >= p0) {
            B->lo[0] = mn[0];
            B->lo[1] = mn[1];
            B->hi[0] = mx[0];
            B->hi[1] = mx[1];
          }
        }
      }
      ccb = __shfl(cb[k], 63);
      cmn[0] = __shfl(mn[0], 63);
      cmn[1] = __shfl(mn[1], 63);
      cmx[0] = __shfl(mx[0], 63);
      cmx[1] = __shfl(mx[1], 63);
    }
    // the window's last cell, when it starts here and runs past the end:
    // reduce its remaining positions (sorted cells only; larger ones below)
    {
      const int l = (p1 - p0 - 1) & 63, kl = (p1 - p0 - 1) >> 6;
      int lcb = -1, lce = 0, lcell = 0;
#pragma unroll
      for (int k = 0; k < NP; k++) {
        if (k == kl) {
          lcb = __shfl(cb[k], l);
          lce = __shfl(ce[k], l);
          lcell = __shfl(cell[k], l);
        }
      }
      if (lcb >= p0 && lce > p1 && lce - lcb <= kZSortMax) {
        double mn[2] = {cmn[0], cmn[1]}, mx[2] = {cmx[0], cmx[1]};
        for (int j0 = p1; j0 < lce; j0 += 256) {
          double4 q[4];
#pragma unroll
          for (int u = 0; u < 4; u++) q[u] = grp[pb + min(j0 + 64 * u + lane, lce - 1)];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            mn[0] = fmin(mn[0], q[u].x);
            mn[1] = fmin(mn[1], q[u].y);
            mx[0] = fmax(mx[0], q[u].x);
            mx[1] = fmax(mx[1], q[u].y);
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          mn[0] = fmin(mn[0], __shfl_xor(mn[0], off));
          mn[1] = fmin(mn[1], __shfl_xor(mn[1], off));
          mx[0] = fmax(mx[0], __shfl_xor(mx[0], off));
          mx[1] = fmax(mx[1], __shfl_xor(mx[1], off));
        }
        if (lane == 0) {
          CellBox *B = cbox + G.cbase + lcell;
          B->lo[0] = mn[0];
          B->lo[1] = mn[1];
          B->hi[0] = mx[0];
          B->hi[1] = mx[1];
        }
      }
    }
    // cells above kZSortMax whose first position is in this window: the
    // whole wave reduces their box
#pragma unroll
    for (int k = 0; k < NP; k++) {
      const int i = p0 + k * 64 + lane;
      uint64_t big = __ballot(i < p1 && ce[k] - cb[k] > kZSortMax && i == cb[k]);
      while (big) {
        const int l = __builtin_ctzll(big);
        big &= big - 1;
        const int b0 = __shfl(cb[k], l), e0 = __shfl(ce[k], l), c = __shfl(cell[k], l);
        double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
        for (int j = b0 + lane; j < e0; j += 64) {
          const double4 q = grp[pb + j];
          mn[0] = fmin(mn[0], q.x); mx[0] = fmax(mx[0], q.x);
          mn[1] = fmin(mn[1], q.y); mx[1] = fmax(mx[1], q.y);
          mn[2] = fmin(mn[2], q.z); mx[2] = fmax(mx[2], q.z);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
          for (int ax = 0; ax < 3; ax++) {
            mn[ax] = fmin(mn[ax], __shfl_xor(mn[ax], off));
            mx[ax] = fmax(mx[ax], __shfl_xor(mx[ax], off));
          }
        }
        if (lane == 0) {
          CellBox B;
          for (int ax = 0; ax < 3; ax++) {
            B.lo[ax] = mn[ax];
            B.hi[ax] = mx[ax];
          }
          cbox[G.cbase + c] = B;
        }
      }
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

// The same walk with the column's nz + 1 <= 64 cell starts held one per lane
// (lane z holds cs[z]): the cell of a point and the cell where a tile ends
// come from one ballot each, the span limit from one lane read, so a tile
// costs a few instructions instead of a chain of dependent LDS reads.
__device__ inline void walk_column_lanes(const GridGeom &G, int csv, int lane, int col,
                                         int maxspan, int mock, int emit, Tile *out,
                                         int64_t &ntile) {
  const int nz = G.n[2];
  int p = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_readlane(csv, 0));
  const int pend = __builtin_amdgcn_readlane(csv, nz);
  int z = 0;
  while (p < pend) {
    // cell of point p: the first z' >= z with cs[z' + 1] > p
    const uint64_t m0 = __ballot(lane > z && lane <= nz && csv > p);
    z = (int)__builtin_ctzll(m0) - 1;
    const int zmax = min(nz - 1, z + maxspan - 1);
    const int q = min(p + kTileMax, __builtin_amdgcn_readlane(csv, zmax + 1));
    // last cell of the tile: the first z' >= z with cs[z' + 1] >= q
    const uint64_t m1 = __ballot(lane > z && lane <= nz && csv >= q);
    const int z1 = (int)__builtin_ctzll(m1) - 1;
    if (emit && lane == 0) {
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

// Pass 3: one workgroup per column (blockIdx.x, strided; catalogue
// blockIdx.y); column col spans [off[col * nblk], off[(col + 1) * nblk]) of
// colgrp (off = the catalogue's scanned matrix); grp in cell order, cell
// starts into cstart; with colcnt, the column's tile count too (the walk of
// the tiles' counting pass, on the same cell starts).
__global__ __launch_bounds__(256) void k_colcells(const GridGeom *geom, const int *off,
                                                  const double4 *colgrp, double4 *grp,
                                                  int *cstart, const int *maxspan,
                                                  const int64_t *col_prefix, int *colcnt) {
  __shared__ int cnt[kMaxAxisCells + 1];
  __shared__ int zs[kMaxAxisCells + 1];
  const int mock = blockIdx.y;
  const GridGeom &G = geom[mock];
  const int stride = G.nblk;
  off += G.mbase;
  const int ncol = G.n[0] * G.n[1], nz = G.n[2];
  const int tid = threadIdx.x, lane = tid & 63;
  for (int col = blockIdx.x; col < ncol; col += gridDim.x) {
    const int c0 = off[(int64_t)col * stride], c1 = off[(int64_t)(col + 1) * stride];
    for (int z = tid; z <= nz; z += blockDim.x) cnt[z] = 0;
    __syncthreads();
    for (int i = c0 + tid; i < c1; i += blockDim.x)
      atomicAdd(&cnt[cell_coord(G, 2, colgrp[G.pbase + i].z)], 1);
    __syncthreads();
    // exclusive scan of the nz counts by wave 0, 64 at a time
    if (tid < 64) {
      int carry = 0;
      for (int z0 = 0; z0 < nz; z0 += 64) {
        const int v = z0 + lane < nz ? cnt[z0 + lane] : 0;
        int x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int y = __shfl_up(x, d);
          if (lane >= d) x += y;
        }
        if (z0 + lane < nz) zs[z0 + lane] = carry + x - v;
        carry += __shfl(x, 63);
      }
    }
    __syncthreads();
    for (int z = tid; z < nz; z += blockDim.x) {
      cstart[G.sbase + (int64_t)col * nz + z] = c0 + zs[z];
      cnt[z] = 0;
    }
    if (col == ncol - 1 && tid == 0) cstart[G.sbase + (int64_t)ncol * nz] = c1;
    __syncthreads();
    for (int i = c0 + tid; i < c1; i += blockDim.x) {
      const double4 v = colgrp[G.pbase + i];
      const int z = cell_coord(G, 2, v.z);
      grp[G.pbase + c0 + zs[z] + atomicAdd(&cnt[z], 1)] = v;
    }
    __syncthreads();
    if (colcnt) {
      for (int z = tid; z <= nz; z += blockDim.x) zs[z] = z < nz ? c0 + zs[z] : c1;
      __syncthreads();
      if (tid < 64) {
        int64_t n = 0;
        if (nz < 64) {
          walk_column_lanes(G, zs[min(lane, nz)], lane, col, maxspan[mock], mock, 0, nullptr, n);
        } else if (lane == 0) {
          walk_column(G, zs, col, maxspan[mock], mock, 0, nullptr, n);
        }
        if (lane == 0) colcnt[col_prefix[mock] + column_rank(col, G.n[0], G.n[1])] = (int)n;
      }
      __syncthreads();
    }
  }
}

// One wave per column: the column's cell starts are held in lanes (columns of
// up to 63 z-cells) or staged in the wave's LDS slice and walked by one lane.
// Counts and offsets are indexed by the column's queue position.
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
    const int64_t q = col_prefix[lo] + column_rank(col, G.n[0], G.n[1]);
    const int *src = cstart + G.sbase + (int64_t)col * nz;
    if (nz < 64) {
      const int csv = src[min(lane, nz)];
      int64_t n = emit ? coloff[q] : 0;
      walk_column_lanes(G, csv, lane, col, maxspan[lo], lo, emit, tiles, n);
      if (!emit && lane == 0) colcnt[q] = (int)n;
      continue;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int z = lane; z <= nz; z += 64) cs[z] = src[z];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      int64_t n = emit ? coloff[q] : 0;
      walk_column(G, cs, col, maxspan[lo], lo, emit, tiles, n);
      if (!emit) colcnt[q] = (int)n;
    }
  }
}

} // namespace cp
