// Pair kernels: one persistent launch drains work queues of items.
//
// Work decomposition (MI355X, wave64).  A tile is <= 64 points of one cell
// column; lane l of a wave holds tile point l.  An item is one tile and one
// chunk of its list of neighbour columns (chunks of about equal cost); items
// sit in 8 queues, one per XCD, each a contiguous share of the box, drained
// by that XCD's waves first.  For an item the wave tests the neighbouring
// cells 64 at a time (Section 1.2: all pairs within R_max lie in the
// neighbouring cells; Section 2.1: for an auto-count only unique pairs of
// cells -- a geometric half-shell -- and within the tile's own cells unique
// pairs of points by sorted index), skips cells whose bounding box is too
// far from the tile's (Section 2.2, minimum possible separation), cuts each
// remaining (tile, cell) unit to a z-window on the z-sorted cell (Section
// 2.2, late entry and early exit; the binary64 loops join consecutive
// z-cells of a column into one unit), and streams the unit's points through
// the scalar cache, so every VALU instruction of the inner loop takes one
// wave-uniform operand from SGPRs and one per-lane operand from VGPRs.
//
// Inner loop, binary32 mode.  Coordinates are held relative to the streamed
// cell's centre, so the squared separation is evaluated as
//   s~ = |r|^2 + |p|^2 - 2 r.p     (r: tile point, p: streamed point)
// in three FMAs and one add; the stream record carries (-2p, |p|^2).  An
// error bound eps on |s~ - s| (s the binary64 value of the reference formula)
// turns each edge E_k into an uncertain band; pairs inside a band are
// re-evaluated in binary64 with the reference formula, so counts equal the
// binary64 counts exactly.
//
// Binning (Section 2.2 "Updating the histogram").  The paper scans bins from
// the outermost down with vector masks and popcounts; on a 64-wide wave that
// scan runs about as deep as the innermost bin any lane needs.  Here the
// unit's separation bounds pick the loop: a unit inside one bin is counted
// without separations, units spanning two or three slots decide each pair
// with one or two compares into register counters (and register weight
// sums), and other units look the bin up in a 2-word LDS table indexed by
// the exponent and top mantissa bits of the separation, counting into a
// private row of LDS counters per lane.
#include "cp_internal.h"

#include <float.h>
#include <type_traits>

namespace cp {

typedef const __attribute__((address_space(4))) float sfloat;
typedef const __attribute__((address_space(4))) double sdouble;
typedef const __attribute__((address_space(4))) int sint;

__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni64(int64_t v) {
  int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline double uni_d(double v) {
  return __longlong_as_double(uni64(__double_as_longlong(v)));
}

// A wave-uniform value held in a VGPR (every lane the same): loop constants
// of the heavier loops live there, so the SGPRs stay free for the streamed
// records (constants kept in SGPRs were spilled to VGPR lanes and read back
// with v_readlane on every record).
__device__ inline int in_vgpr(int v) {
  int r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
  return r;
}
__device__ inline float in_vgpr(float v) { return __int_as_float(in_vgpr(__float_as_int(v))); }

// Slot of a binary64 squared separation: 0 below E_0, k + 1 for bin k,
// nb + 1 at or above E_nb (the reference half-open rule).
__device__ inline int exact_slot(const double *E, int nb, double s) {
  if (s < E[0]) return 0;
  if (s >= E[nb]) return nb + 1;
  int k = 0;
  while (k + 1 < nb && s >= E[k + 1]) k++;
  return k + 1;
}

// Pi bin of a binary64 |dz| < pi_max: l with q_l <= pi < q_{l+1},
// q_l = fl(l * dpi).  The product with fl(1 / dpi) lands within one of l
// (|dz| / dpi < 257 and both roundings are relative), so one compare each
// way against the exact q_l and q_{l+1} settles it without a division.
__device__ inline int exact_pibin(double pz, double dpi, double inv_dpi, int npi) {
  int l = (int)(pz * inv_dpi);
  l = min(max(l, 0), npi - 1);
  l -= (l > 0 && pz < (double)l * dpi) ? 1 : 0;
  l += (l + 1 < npi && pz >= (double)(l + 1) * dpi) ? 1 : 0;
  return l;
}

// Pi bin of a binary64 |dz| < pi_max through binary32: f = fl32(fl32(|dz|) *
// fl32(1 / dpi)) and bin floor(f), unless the fraction of f lies within pd of
// an integer (the band of the binary32 loops with the estimate's error
// u |dz| < u pi_max), where exact_pibin decides.
__device__ inline int pibin_fast(double pz, float inv32, float pd, float pd1, double dpi,
                                 double inv_dpi, int npi) {
  const float f = (float)pz * inv32;
  const float fr = __builtin_amdgcn_fractf(f);   // f - floor(f), exact for f >= 0
  if (fr < pd || fr > pd1) return exact_pibin(pz, dpi, inv_dpi, npi);
  return (int)f;
}

// Table lookup: slot for v (binary32 estimate), or uncertain.
struct TabHit {
  int slot;
  bool unc;
};
__device__ inline TabHit tab_lookup(const uint2 *tab, int lo, int hi, int sh, float v) {
  int b = __float_as_int(v) >> sh;
  b = min(max(b, lo), hi);
  const uint2 e = tab[b - lo];
  const bool ch = v >= __uint_as_float(e.y);
  TabHit h;
  h.unc = (v >= __uint_as_float(e.x)) && !ch;
  h.slot = (int)(e.y & 63u) - 1 + (ch ? 1 : 0);
  return h;
}

// Slot of a binary64 value through the table of fl32(s); exact fallback.
__device__ inline int slot64(const uint2 *tab, int lo, int hi, int sh, const double *E, int nb,
                             double s) {
  TabHit h = tab_lookup(tab, lo, hi, sh, (float)s);
  if (h.unc) h.slot = exact_slot(E, nb, s);
  return h.slot;
}

// The same for s < E_B: fl32(s) <= fl32(E_B) lies at or below the table's
// top cell, so the index is clamped below only; tb = the table minus lo.
__device__ inline int slot64_below(const uint2 *tb, int lo, int sh, const double *E, int nb,
                                   double s) {
  const float v = (float)s;
  const uint2 e = tb[max(__float_as_int(v) >> sh, lo)];
  const bool ch = v >= __uint_as_float(e.y);
  if (v >= __uint_as_float(e.x) && !ch) return exact_slot(E, nb, s);
  return (int)(e.y & 63u) - 1 + (ch ? 1 : 0);
}

// Square root for the weighted mean separation (not part of any bin
// decision): the hardware reciprocal square root (relative error ~5e-8 on
// gfx950) refined by one Newton step in binary64, measured relative error
// below 5e-15, far inside the 1e-12 tolerance of the weighted sums.
__device__ inline double sep_sqrt(double x) {
  // x >= 0.  x == 0 gives r == 0 and an exact 0; x below 1e-300 (separations
  // below 1e-150) would come out inexact but still below 1e-149.
  const double y = __builtin_amdgcn_rsq(x + 1e-300);
  const double r = x * y;
  const double e = __builtin_fma(-r, r, x);
  return __builtin_fma(0.5 * y, e, r);
}

// Reference separation of the tile point (px, py, pz) and streamed point q
// under the cell shift S; wrap axes take the per-pair minimum image.
template <bool SHIFT, bool WRAP>
__device__ inline void ref_sep(double px, double py, double pz, double qx, double qy, double qz,
                               const double S[3], const int wrapax[3], double box, double half,
                               double &dx, double &dy, double &dz) {
  dx = qx - px;
  dy = qy - py;
  dz = qz - pz;
  if (SHIFT) {
    dx = dx + S[0];
    dy = dy + S[1];
    dz = dz + S[2];
  }
  if (WRAP) {
    double *d[3] = {&dx, &dy, &dz};
    for (int a = 0; a < 3; a++) {
      if (wrapax[a]) {
        if (*d[a] > half) *d[a] = *d[a] - box;
        else if (*d[a] < -half) *d[a] = *d[a] + box;
      }
    }
  }
}

// Adds (w, w r) to an interleaved pair of LDS weight sums (one address, two
// atomics at offsets 0 and 8).
__device__ inline void add_w(double *p, double w, double wr) {
  atomicAdd(p, w);
  atomicAdd(p + 1, wr);
}

// LDS byte address of a pointer into the workgroup's LDS, and back.
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ inline uint32_t lds_addr(uint32_t *p) {
  return (uint32_t)(uintptr_t)(lds_u32 *)p;
}
__device__ inline uint32_t *lds_ptr(uint32_t a) { return (uint32_t *)(lds_u32 *)(uintptr_t)a; }

struct WaveArea {
  uint32_t *hist;
  uint32_t *histx;  // WPXI: the xi counters, one row of slots per lane pair (lane mod 32)
  double *hw;   // weight sums, interleaved: hw[2 i] = sum w, hw[2 i + 1] = sum w r
  uint32_t *list;   // weighted xi, binary32 mode: (tile lane, record) pairs to evaluate
};

// a * b + c on the low 24 bits of a and b, and (a << s) + c, one
// instruction each (the compiler otherwise forms a multiply, a shift and a
// three-way add).
__device__ inline uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ inline uint32_t lshl_add(uint32_t a, uint32_t s, uint32_t c) {
  uint32_t r;
  asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(s), "v"(c));
  return r;
}

// Address of the (r_p, pi) counter of slot s and pi bin l in a wave's
// histogram, word (s * npi + l) * wpc + base (wpc copies, interleaved; wpc a
// power of two).  The table entry's low bits carry t = s + 1 - ch, where ch
// says the value lies above the entry's upper threshold: the -1 is folded
// into the lane's base address and ch picks the base one row up, so the
// address is a select, a 24-bit multiply-add and a shift-add.
struct WpIndex {
  uint32_t row4, hb, hb1;
  uint32_t lsh;
  __device__ WpIndex(uint32_t *hist, int npi, int wpc, int base) {
    row4 = (uint32_t)in_vgpr(npi * wpc * 4);
    lsh = (uint32_t)in_vgpr(wpc == 2 ? 3 : (wpc == 4 ? 4 : (wpc == 8 ? 5 : 2)));
    hb = lds_addr(hist) + 4u * (uint32_t)base - row4;
    hb1 = hb + row4;
  }
  __device__ uint32_t *at(uint32_t t, bool ch, int l) const {
    return lds_ptr(lshl_add((uint32_t)l, lsh, mad_u24(t, row4, ch ? hb1 : hb)));
  }
};

// xi counters rows[s * 32 + c] of slots s = 0 .. nb + 1, one column per
// lane pair (c = lane mod 32): lane s - 1 takes slot s's wave total, and one
// atomic instruction adds them all (every wave's totals land in the same few
// lines of the output, and per-slot atomics from one lane, one memory request
// each, queued there for tens of microseconds at the end of a launch); then
// the rows are cleared.
__device__ inline void flush_xi_rows(uint32_t *rows, unsigned long long *gh, int nb, int lane) {
  unsigned long long mine = 0;
  for (int s = 1; s <= nb; s++) {
    const unsigned long long v =
        wave_sum_u64(lane < 32 ? (unsigned long long)rows[s * 32 + lane] : 0ull);
    if (lane == s - 1) mine = v;
  }
  if (lane < nb && mine) atomicAdd(gh + lane, mine);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < 32)
    for (int s = 0; s < nb + 2; s++) rows[s * 32 + lane] = 0u;
}

template <int MODE, int W>
__device__ inline void flush_hist(const PairParams &P, WaveArea A, int mock, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int nb = P.nb, NS = P.nslots;
  unsigned long long *gh = P.hist + (int64_t)mock * P.hist_stride;
  if (MODE == XI) {
    // lane s - 1 takes slot s's wave total, and one atomic instruction adds
    // them all: every wave's totals land in the same few lines of the output,
    // and per-slot atomics from one lane (one memory request each) queued
    // there for tens of microseconds at the end of a launch
    unsigned long long mine = 0;
    for (int s = 1; s <= nb; s++) {
      const unsigned long long v = wave_sum_u64((unsigned long long)A.hist[s * 64 + lane]);
      if (lane == s - 1) mine = v;
    }
    if (lane < nb && mine) atomicAdd(gh + lane, mine);
    if (W && lane >= 1 && lane <= nb) {
      double a = 0.0, b = 0.0;
      for (int c = 0; c < kWStripe; c++) {
        a += A.hw[2 * (lane * kWStripe + c)];
        b += A.hw[2 * (lane * kWStripe + c) + 1];
      }
      if (a != 0.0) unsafeAtomicAdd(P.hw + (int64_t)mock * P.hist_stride + (lane - 1), a);
      if (b != 0.0) unsafeAtomicAdd(P.hwr + (int64_t)mock * P.hist_stride + (lane - 1), b);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int s = 0; s < NS; s++) A.hist[s * 64 + lane] = 0u;
    if (W) {
      for (int t = lane; t < 2 * NS * kWStripe; t += 64) A.hw[t] = 0.0;
    }
  } else {
    const int npi = P.npi, wpc = P.wpc;
    for (int t = lane; t < nb * npi; t += 64) {
      uint32_t v = 0;
      for (int c = 0; c < wpc; c++) v += A.hist[(npi + t) * wpc + c];
      if (v) atomicAdd(gh + t, (unsigned long long)v);
      if (W) {
        double a = 0.0, b = 0.0;
        for (int c = 0; c < wpc; c++) {
          a += A.hw[2 * ((npi + t) * wpc + c)];
          b += A.hw[2 * ((npi + t) * wpc + c) + 1];
        }
        if (a != 0.0) unsafeAtomicAdd(P.hw + (int64_t)mock * P.hist_stride + t, a);
        if (b != 0.0) unsafeAtomicAdd(P.hwr + (int64_t)mock * P.hist_stride + t, b);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < NS * npi * wpc; t += 64) {
      A.hist[t] = 0u;
      if (W) {
        A.hw[2 * t] = 0.0;
        A.hw[2 * t + 1] = 0.0;
      }
    }
    if (MODE == WPXI) flush_xi_rows(A.histx, P.histx + (int64_t)mock * P.histx_stride, P.nbx, lane);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-lane state of the tile point.
struct LanePt {
  double x, y, z, w;
  int iloc;   // sorted index relative to the catalogue (own-cell ordering)
};
constexpr double kNoPoint = 1e200;   // coordinates of the lanes beyond a tile's points

// ------------------------------------------------------------- streaming
//
// A unit's records [jb, je) are walked through the scalar cache in groups,
// each group's loads issued one group ahead.  The main loop handles two
// groups per trip so the two buffers alternate without copies; the stream
// arrays are padded by 8 records, so the look-ahead never leaves the
// allocation.  The remainder goes one record at a time: one more copy of the
// body instead of eight keeps the kernels small enough for the instruction
// cache.  The body is called once per record with its values in SGPRs.

#define CP_LOAD16(dst, src)                                                                    \
  _Pragma("unroll") for (int t_ = 0; t_ < 16; t_++) dst[t_] = (src)[t_];
#define CP_REC4(arr, jj, u) body((jj) + (u), arr[4 * (u)], arr[4 * (u) + 1], arr[4 * (u) + 2], \
                                 arr[4 * (u) + 3])

template <typename F>
__device__ inline void stream_f32(const float4 *base, int jb, int je, F &&body) {
  sfloat *p = (sfloat *)(base + jb);
  int j = jb;
  if (j + 8 <= je) {
    float a[16];
    CP_LOAD16(a, p);
    do {
      float b[16];
      CP_LOAD16(b, p + 16);
      CP_REC4(a, j, 0); CP_REC4(a, j, 1); CP_REC4(a, j, 2); CP_REC4(a, j, 3);
      CP_LOAD16(a, p + 32);
      CP_REC4(b, j + 4, 0); CP_REC4(b, j + 4, 1); CP_REC4(b, j + 4, 2); CP_REC4(b, j + 4, 3);
      j += 8;
      p += 32;
    } while (j + 8 <= je);
  }
  while (j < je) {
    const float r0 = p[0], r1 = p[1], r2 = p[2], r3 = p[3];
    body(j, r0, r1, r2, r3);
    j++;
    p += 4;
  }
}

// binary64 records only (x, y, z, w), groups of two.
#define CP_LOAD8D(dst, src)                                                                    \
  _Pragma("unroll") for (int t_ = 0; t_ < 8; t_++) dst[t_] = (src)[t_];
#define CP_REC2D(arr, jj, u) body((jj) + (u), arr[4 * (u)], arr[4 * (u) + 1], arr[4 * (u) + 2], \
                                  arr[4 * (u) + 3])
template <typename F>
__device__ inline void stream_f64(const double4 *base, int jb, int je, F &&body) {
  sdouble *p = (sdouble *)(base + jb);
  int j = jb;
  double a[8];
  CP_LOAD8D(a, p);
  while (j + 4 <= je) {
    double b[8];
    CP_LOAD8D(b, p + 8);
    CP_REC2D(a, j, 0); CP_REC2D(a, j, 1);
    CP_LOAD8D(a, p + 16);
    CP_REC2D(b, j + 2, 0); CP_REC2D(b, j + 2, 1);
    j += 4;
    p += 16;
  }
  while (j < je) {
    const double r0 = p[0], r1 = p[1], r2 = p[2], r3 = p[3];
    body(j, r0, r1, r2, r3);
    j++;
    p += 4;
  }
}

// binary32 and binary64 records together (weighted loops), groups of two.
#define CP_RECW(fa, da, jj, u)                                                                 \
  body((jj) + (u), fa[4 * (u)], fa[4 * (u) + 1], fa[4 * (u) + 2], fa[4 * (u) + 3], da[4 * (u)],  \
       da[4 * (u) + 1], da[4 * (u) + 2], da[4 * (u) + 3])
template <typename F>
__device__ inline void stream_w(const float4 *fbase, const double4 *dbase, int jb, int je,
                                F &&body) {
  sfloat *p = (sfloat *)(fbase + jb);
  sdouble *q = (sdouble *)(dbase + jb);
  int j = jb;
  float fa[8];
  double da[8];
#pragma unroll
  for (int t = 0; t < 8; t++) {
    fa[t] = p[t];
    da[t] = q[t];
  }
  while (j + 4 <= je) {
    float fb[8];
    double db[8];
#pragma unroll
    for (int t = 0; t < 8; t++) {
      fb[t] = p[8 + t];
      db[t] = q[8 + t];
    }
    CP_RECW(fa, da, j, 0); CP_RECW(fa, da, j, 1);
#pragma unroll
    for (int t = 0; t < 8; t++) {
      fa[t] = p[16 + t];
      da[t] = q[16 + t];
    }
    CP_RECW(fb, db, j + 2, 0); CP_RECW(fb, db, j + 2, 1);
    j += 4;
    p += 16;
    q += 16;
  }
  if (j < je) {
    float fb[8];
    double db[8];
#pragma unroll
    for (int t = 0; t < 8; t++) {
      fb[t] = p[8 + t];
      db[t] = q[8 + t];
    }
    if (j < je) CP_RECW(fa, da, j, 0);
    if (j + 1 < je) CP_RECW(fa, da, j, 1);
    if (j + 2 < je) CP_RECW(fb, db, j + 2, 0);
    if (j + 3 < je) CP_RECW(fb, db, j + 2, 1);
  }
}

// Narrows the records [jb, je) of a z-sorted cell to those with
// zlo <= z <= zhi: two lane-parallel searches, 64 records per step, the
// first from the front for the lower end, the second from the back for the
// upper end.  jb, je and the result are wave-uniform.
__device__ inline void zwindow(const double4 *pos, float zlo, float zhi, int lane, int &jb,
                               int &je) {
  const double *zp = (const double *)pos + 2;   // z of record j at zp[4 j]
  const double lo = (double)zlo, hi = (double)zhi;
  int b = je;
  for (int j0 = jb; j0 < je; j0 += 64) {
    const int j = j0 + lane;
    const bool ge = j < je && zp[4 * j] >= lo;
    const unsigned long long m = __builtin_amdgcn_ballot_w64(ge);
    if (m) {
      b = j0 + __builtin_ctzll(m);
      break;
    }
  }
  int e = b;
  for (int j1 = je; j1 > b; j1 -= 64) {
    const int j = j1 - 64 + lane;
    const bool le = j >= b && zp[4 * j] <= hi;
    const unsigned long long m = __builtin_amdgcn_ballot_w64(le);
    if (m) {
      e = j1 - 64 + (63 - __builtin_clzll(m)) + 1;
      break;
    }
  }
  jb = b;
  je = e;
}

// Per-unit data handed to the inner loops.
struct Unit {
  int jb, je;             // streamed records, relative to the catalogue's first point
  const float4 *strm;     // stream / positions of the catalogue (index 0 = its first point)
  const double4 *pos;
  double S[3];
  int slot_lo, slot_hi;   // every pair of the unit lands in [slot_lo, slot_hi]
};

__device__ inline float gram3(float rx, float ry, float rz, float ra, float qx, float qy, float qz,
                              float qw) {
  float v = __builtin_fmaf(rx, qx, ra);
  v = __builtin_fmaf(ry, qy, v);
  v = __builtin_fmaf(rz, qz, v);
  return v + qw;
}

// ---------------------------------------------------------------- FP32 loops

// Binary64 re-evaluation of one uncertain xi pair; adds it to its exact slot.
template <bool SHIFT>
__device__ inline void recheck_xi(WaveArea A, const LanePt &L, int lane, const Unit &U, int j,
                                  const double *sE, int nb) {
  sdouble *DP = (sdouble *)U.pos;
  const double ux = DP[4 * j], uy = DP[4 * j + 1], uz = DP[4 * j + 2];
  const int wrapax[3] = {0, 0, 0};
  double dx, dy, dz;
  ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, 0.0, 0.0, dx, dy, dz);
  const double s64 = (dx * dx + dy * dy) + dz * dz;
  atomicAdd(&A.hist[exact_slot(sE, nb, s64) * 64 + lane], 1u);
}

// xi, binary32, a unit whose pairs can only land in slot_lo or slot_hi:
// edge E_t (t = slot_lo) decides.  The edge is folded into the lane's
// constant, b = fl32(|r|^2 - E_t), so three FMAs and one add give
// d~ = s~ - E_t directly; rounding keeps the sign of the last add, so the
// decision error is that of the Gram form (the bound eps covers it).  The
// first pass, branch-free, counts the negative d~ per lane and tracks the
// smallest |d~|.  Only a lane with some |d~| < eps takes a second pass that
// re-evaluates the same binary32 values, bit for bit, and sends those pairs
// to binary64.  exec = valid lanes.
template <bool SHIFT>
__device__ inline void loop_xi_f32_two(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                       float rx, float ry, float rz, float ra, const Unit &U,
                                       const double *sE, uint32_t &nrechk) {
  const int nb = P.nb;
  const float b = (float)((double)ra - sE[U.slot_lo]);
  const float eps = P.eps32;
  uint32_t nneg = 0;
  float mn = 3.0e38f;
  stream_f32(U.strm, U.jb, U.je, [&](int, float qx, float qy, float qz, float qw) {
    const float d = gram3(rx, ry, rz, b, qx, qy, qz, qw);
    nneg += __float_as_uint(d) >> 31;
    mn = fminf(mn, fabsf(d));
  });
  uint32_t uneg = 0, upos = 0;
  if (mn < eps) {
    stream_f32(U.strm, U.jb, U.je, [&](int j, float qx, float qy, float qz, float qw) {
      const float d = gram3(rx, ry, rz, b, qx, qy, qz, qw);
      if (fabsf(d) < eps) {
        recheck_xi<SHIFT>(A, L, lane, U, j, sE, nb);
        const uint32_t ng = __float_as_uint(d) >> 31;
        uneg += ng;
        upos += 1u - ng;
      }
    });
    nrechk += uneg + upos;
  }
  const uint32_t nlo = nneg - uneg;
  const uint32_t nhi = (uint32_t)(U.je - U.jb) - nneg - upos;
  if (U.slot_lo >= 1) atomicAdd(&A.hist[U.slot_lo * 64 + lane], nlo);
  if (U.slot_hi <= nb) atomicAdd(&A.hist[U.slot_hi * 64 + lane], nhi);
}

// xi, binary32, a unit whose pairs can only land in slot_lo, slot_lo + 1 or
// slot_lo + 2: edges E_a = E[slot_lo] and E_b = E[slot_lo + 1] decide.
// d1 = s~ - E_a comes from the folded Gram form as in the two-slot loop and
// d2 = fl(d1 + fl32(E_a - E_b)) from it in one add; the add keeps the sign of
// its exact result, so d2's decision error is that of d1 plus u |E_a - E_b|,
// which eps32_3 covers.  Sign counts give the three slot counts; lanes with
// a |d| below the bound re-evaluate those pairs in a second pass.
// exec = valid lanes.
template <bool SHIFT>
__device__ inline void loop_xi_f32_three(const PairParams &P, WaveArea A, const LanePt &L,
                                         int lane, float rx, float ry, float rz, float ra,
                                         const Unit &U, const double *sE, uint32_t &nrechk) {
  const int nb = P.nb;
  const double Ea = sE[U.slot_lo], Eb = sE[U.slot_lo + 1];
  const float b = (float)((double)ra - Ea);
  const float c = (float)(Ea - Eb);
  const float eps = P.eps32_3;
  uint32_t n1 = 0, n2 = 0;
  float mn = 3.0e38f;
  stream_f32(U.strm, U.jb, U.je, [&](int, float qx, float qy, float qz, float qw) {
    const float d1 = gram3(rx, ry, rz, b, qx, qy, qz, qw);
    const float d2 = d1 + c;
    n1 += __float_as_uint(d1) >> 31;
    n2 += __float_as_uint(d2) >> 31;
    mn = fminf(mn, fminf(fabsf(d1), fabsf(d2)));
  });
  uint32_t u1 = 0, u2 = 0, un = 0;
  if (mn < eps) {
    stream_f32(U.strm, U.jb, U.je, [&](int j, float qx, float qy, float qz, float qw) {
      const float d1 = gram3(rx, ry, rz, b, qx, qy, qz, qw);
      const float d2 = d1 + c;
      if (fabsf(d1) < eps || fabsf(d2) < eps) {
        recheck_xi<SHIFT>(A, L, lane, U, j, sE, nb);
        u1 += __float_as_uint(d1) >> 31;
        u2 += __float_as_uint(d2) >> 31;
        un++;
      }
    });
    nrechk += un;
  }
  const uint32_t c0 = n1 - u1;                       // below E_a
  const uint32_t c1 = (n2 - u2) - c0;                // [E_a, E_b)
  const uint32_t c2 = (uint32_t)(U.je - U.jb) - un - (n2 - u2);   // at or above E_b
  if (U.slot_lo >= 1) atomicAdd(&A.hist[U.slot_lo * 64 + lane], c0);
  atomicAdd(&A.hist[(U.slot_lo + 1) * 64 + lane], c1);
  if (U.slot_lo + 2 <= nb) atomicAdd(&A.hist[(U.slot_lo + 2) * 64 + lane], c2);
}

// xi, binary32, general unit: per-lane table lookup.  OWN: one of the tile's
// own cells (auto-count), only j > i pairs.  An uncertain pair is
// re-evaluated in binary64 on the spot: the branch is taken on the few
// records where some lane has one, which costs less than streaming the unit
// a second time (measured).
template <bool OWN, bool SHIFT>
__device__ inline void loop_xi_f32(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                   float rx, float ry, float rz, float ra, const Unit &U,
                                   const uint2 *tab32, const double *sE, uint32_t &nrechk) {
  const float AB = P.AB32;
  const int lo = P.tab32_lo, sh = P.tab_shift;
  const uint2 *tb = tab32 - lo;   // s~ < AB32, the table's top: clamped below only
  const int nb = P.nb;
  uint32_t nunc = 0;
  stream_f32(U.strm, U.jb, U.je, [&](int j, float qx, float qy, float qz, float qw) {
    const float s = gram3(rx, ry, rz, ra, qx, qy, qz, qw);
    bool inr = s < AB;
    if (OWN) inr = inr && (j > L.iloc);
    if (inr) {
      const uint2 e = tb[max(__float_as_int(s) >> sh, lo)];
      const bool ch = s >= __uint_as_float(e.y);
      TabHit h;
      h.unc = (s >= __uint_as_float(e.x)) && !ch;
      h.slot = (int)(e.y & 63u) - 1 + (ch ? 1 : 0);
      if (!h.unc) atomicAdd(&A.hist[h.slot * 64 + lane], 1u);
      else {
        recheck_xi<SHIFT>(A, L, lane, U, j, sE, nb);
        nunc++;
      }
    }
  });
  nrechk += nunc;
}

// wp, binary32 filter (the loops below): the r_p^2 estimate v~ (Gram form in
// the streamed cell's frame) goes through the decision table, the line of
// sight pi~ = |qz - rz| (cell-local coordinates) is binned by multiplying
// with 1/dpi, and a pair is in range when v~ < AB32 and pi~ < pi_hi32 (not
// surely beyond r_p,max or pi_max); it is uncertain when v~ lies in an edge's
// band or when the fraction of f = pi~ / dpi lies within pi_delta of an
// integer.  pi_max is the edge at the integer npi and the band covers the
// pre-filter's slack, so a certain pair is below pi_max and its bin floor(f)
// is at most npi - 1.  v~ < AB32 keeps the table index at or below the
// table's top, so the index is clamped below only.

// Binary64 re-evaluation of one uncertain wp pair (unweighted).
template <bool SHIFT>
__device__ inline void recheck_wp(const PairParams &P, WaveArea A, const LanePt &L, const Unit &U,
                                  int j, const double *sE, int cpy) {
  sdouble *DP = (sdouble *)U.pos;
  const double ux = DP[4 * j], uy = DP[4 * j + 1], uz = DP[4 * j + 2];
  const int wrapax[3] = {0, 0, 0};
  double dx, dy, dz;
  ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, 0.0, 0.0, dx, dy, dz);
  const double rp2 = dx * dx + dy * dy;
  const double pz64 = fabs(dz);
  if (pz64 < P.pimax && rp2 < P.EB)
    atomicAdd(&A.hist[(exact_slot(sE, P.nb, rp2) * P.npi +
                       exact_pibin(pz64, P.dpi, P.inv_dpi, P.npi)) * P.wpc + cpy], 1u);
}

// wp, unweighted: certain pairs are counted at once, uncertain ones
// re-evaluated in binary64 on the spot (as in the general xi loop).
template <bool OWN, bool SHIFT>
__device__ inline void loop_wp_f32(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                   float rx, float ry, float rz, float ra, const Unit &U,
                                   const uint2 *tab32, const double *sE, uint32_t &nrechk) {
  const int npi = in_vgpr(P.npi), wpc = in_vgpr(P.wpc), lo = in_vgpr(P.tab32_lo);
  const int sh = in_vgpr(P.tab_shift);
  const int base = lane & (wpc - 1);
  const uint2 *tb = tab32 - P.tab32_lo;
  const float AB = in_vgpr(P.AB32), phi = in_vgpr(P.pi_hi32);
  const float inv = in_vgpr(P.inv_dpi32);
  const float pd = in_vgpr(P.pi_delta), pd1 = in_vgpr(1.0f - P.pi_delta);
  const WpIndex H(A.hist, npi, wpc, base);
  uint32_t nunc = 0;
  stream_f32(U.strm, U.jb, U.je, [&](int j, float qx, float qy, float qz, float qw) {
    const float v = __builtin_fmaf(ry, qy, __builtin_fmaf(rx, qx, ra)) + qw;
    const float pz = fabsf(qz - rz);
    bool pre = (v < AB) && (pz < phi);
    if (OWN) pre = pre && (j > L.iloc);
    if (pre) {
      const uint2 e = tb[max(__float_as_int(v) >> sh, lo)];
      const float f = pz * inv;
      const float fr = __builtin_amdgcn_fractf(f);   // f - floor(f), exact for f >= 0
      const bool ch = v >= __uint_as_float(e.y);
      const bool unc = (v >= __uint_as_float(e.x) && !ch) || fr < pd || fr > pd1;
      if (unc) {
        recheck_wp<SHIFT>(P, A, L, U, j, sE, base);
        nunc++;
      } else {
        atomicAdd(H.at(e.y & 63u, ch, (int)f), 1u);
      }
    }
  });
  nrechk += nunc;
}

// w_p and xi in one pass (WPXI, unweighted): the w_p decisions of
// loop_wp_f32, and for xi the estimate s~ = fl32(pi~^2 + rp~^2) from the same
// binary32 values, decided through its own table (bands of the WPXI error
// bound); an uncertain xi pair is re-evaluated in binary64.  Pairs are
// counted once for each statistic they belong to.
template <bool OWN>
__device__ inline void loop_wpxi_f32(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                     float rx, float ry, float rz, float ra, const Unit &U,
                                     const uint2 *tab32, const double *sE, const uint2 *tabx,
                                     const double *sEx, uint32_t &nrechk) {
  const int npi = in_vgpr(P.npi), wpc = in_vgpr(P.wpc), lo = in_vgpr(P.tab32_lo);
  const int sh = in_vgpr(P.tab_shift);
  const int base = lane & (wpc - 1);
  const uint2 *tb = tab32 - P.tab32_lo;
  const float AB = in_vgpr(P.AB32), phi = in_vgpr(P.pi_hi32);
  const float inv = in_vgpr(P.inv_dpi32);
  const float pd = in_vgpr(P.pi_delta), pd1 = in_vgpr(1.0f - P.pi_delta);
  const int lox = in_vgpr(P.tabx_lo), shx = in_vgpr(P.tabx_shift), nbx = P.nbx;
  const uint2 *tbx = tabx - P.tabx_lo;
  const float ABx = in_vgpr(P.AB32x);
  const WpIndex H(A.hist, npi, wpc, base);
  // xi counter of slot s at row s, column lane mod 32: byte address (s + 1) * 128 + hx
  const uint32_t hx = lds_addr(A.histx) + 4u * (uint32_t)(lane & 31) - 128u, hx1 = hx + 128u;
  uint32_t nunc = 0;
  stream_f32(U.strm, U.jb, U.je, [&](int j, float qx, float qy, float qz, float qw) {
    const float v = __builtin_fmaf(ry, qy, __builtin_fmaf(rx, qx, ra)) + qw;
    const float pz = fabsf(qz - rz);
    const bool ok = OWN ? (j > L.iloc) : true;
    if (ok && v < AB && pz < phi) {
      const uint2 e = tb[max(__float_as_int(v) >> sh, lo)];
      const float f = pz * inv;
      const float fr = __builtin_amdgcn_fractf(f);   // f - floor(f), exact for f >= 0
      const bool ch = v >= __uint_as_float(e.y);
      const bool unc = (v >= __uint_as_float(e.x) && !ch) || fr < pd || fr > pd1;
      if (unc) {
        recheck_wp<true>(P, A, L, U, j, sE, base);
        nunc++;
      } else {
        atomicAdd(H.at(e.y & 63u, ch, (int)f), 1u);
      }
    }
    const float sx = __builtin_fmaf(pz, pz, v);
    if (ok && sx < ABx) {
      const uint2 e = tbx[max(__float_as_int(sx) >> shx, lox)];
      const bool ch = sx >= __uint_as_float(e.y);
      uint32_t ad;
      if (sx >= __uint_as_float(e.x) && !ch) {
        // binary64 re-evaluation (the reference separation)
        sdouble *DP = (sdouble *)U.pos;
        const int wz[3] = {0, 0, 0};
        double dx, dy, dz;
        ref_sep<true, false>(L.x, L.y, L.z, DP[4 * j], DP[4 * j + 1], DP[4 * j + 2], U.S, wz, 0.0,
                             0.0, dx, dy, dz);
        ad = ((uint32_t)exact_slot(sEx, nbx, (dx * dx + dy * dy) + dz * dz) << 7) + hx1;
        nunc++;
      } else {
        ad = lshl_add(e.y & 63u, 7u, ch ? hx1 : hx);
      }
      atomicAdd(lds_ptr(ad), 1u);
    }
  });
  nrechk += nunc;
}

// wp, weighted: every in-range pair is evaluated in binary64 for its rp.
template <bool OWN, bool SHIFT>
__device__ inline void loop_wp_f32_w(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                     float rx, float ry, float rz, float ra, const Unit &U,
                                     const uint2 *tab32, const double *sE, uint32_t &nrechk) {
  const int nb = P.nb;
  const int npi = in_vgpr(P.npi), wpc = in_vgpr(P.wpc), lo = in_vgpr(P.tab32_lo);
  const int sh = in_vgpr(P.tab_shift);
  const int row = npi * wpc, cpy = lane & (wpc - 1);
  const uint2 *tb = tab32 - P.tab32_lo;
  const float AB = in_vgpr(P.AB32), phi = in_vgpr(P.pi_hi32);
  const float inv = in_vgpr(P.inv_dpi32);
  const float pd = in_vgpr(P.pi_delta), pd1 = in_vgpr(1.0f - P.pi_delta);
  const int wrapax[3] = {0, 0, 0};
  stream_w(U.strm, U.pos, U.jb, U.je,
           [&](int j, float qx, float qy, float qz, float qw, double ux, double uy, double uz,
               double uw) {
             const float v = __builtin_fmaf(ry, qy, __builtin_fmaf(rx, qx, ra)) + qw;
             const float pz = fabsf(qz - rz);
             bool inr = (v < AB) && (pz < phi);
             if (OWN) inr = inr && (j > L.iloc);
             if (inr) {
               const uint2 e = tb[max(__float_as_int(v) >> sh, lo)];
               const float f = pz * inv;
               const float fr = __builtin_amdgcn_fractf(f);   // f - floor(f), exact for f >= 0
               const bool ch = v >= __uint_as_float(e.y);
               const bool unc = (v >= __uint_as_float(e.x) && !ch) || fr < pd || fr > pd1;
               double dx, dy, dz;
               ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, 0.0, 0.0, dx, dy,
                                     dz);
               int sl = (int)(e.y & 63u) - 1 + (ch ? 1 : 0), ll = (int)f;
               bool keep = true;
               if (unc) {
                 nrechk++;
                 const double rp2 = dx * dx + dy * dy;
                 const double pz64 = fabs(dz);
                 keep = pz64 < P.pimax && rp2 < P.EB;
                 sl = exact_slot(sE, nb, rp2);
                 ll = exact_pibin(pz64, P.dpi, P.inv_dpi, P.npi);
               }
               if (keep) {
                 const double ww = L.w * uw;
                 const int c = __umul24(sl, row) + __umul24(ll, wpc) + cpy;
                 atomicAdd(&A.hist[c], 1u);
                 add_w(A.hw + 2 * c, ww, ww * sep_sqrt(__builtin_fma(dx, dx, dy * dy)));
               }
             }
           });
}

// Waits for every scalar load and LDS operation issued so far (s_waitcnt
// lgkmcnt(0)).  Scalar loads complete out of order, so before a group of
// streamed records is used the compiler waits for all of them; issuing the
// look-ahead load of the next group only after this wait lets it overlap the
// work on the current group.
__device__ inline void wait_lgkm() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Weighted xi, binary32 filter with compaction, for units whose separation
// range reaches E_B (or lies below E_0).  The weighted mean needs the
// binary64 separation of every counted pair.  Evaluated for every candidate
// on the wave, that binary64 work runs on every record where any lane is in
// range, although most candidates of such units are not.  Here the binary32
// Gram form s~ screens every candidate: a pair with s~ >= AB32 (= up(E_B +
// eps), so its binary64 s is at or beyond E_B) is dropped, every other pair is
// appended to the wave's list.  The list is evaluated 64 pairs at a time, one
// pair per lane: the canonical binary64 separation decides the bin (so the
// counts are those of the binary64 definition by construction; the screen
// only removes pairs that the definition drops), and the same value gives
// sqrt(s) for the weighted sums.  A batch's binary64 records are loaded after
// one group of records and evaluated after the next, so the loads overlap
// the screening.  nrechk counts the listed pairs that binary64 places at or
// beyond E_B.
//   CLS 1: slots [nb, nb + 1]: every kept pair lies in the last bin.
//   CLS 2: slots [nb - 1, nb + 1]: one compare against E_{nb-1}.
//   CLS 0: any other range: decision table, counts and sums in LDS.
// SH: the unit has a periodic shift (added to each binary64 difference).
// A list entry holds byte offsets: (record << 11) | (tile lane << 5), so the
// unit may have at most 2^21 records.  Records go four at a time; the list
// holds at most 63 + 4 x 64 entries.  The look-ahead
// may read up to 7 records past the unit (the stream arrays are padded past
// their end); the last group masks the records past the unit.
// exec = all lanes: list entries go to lanes regardless of the tile's size.
template <int CLS, bool SH>
__device__ inline void loop_xi_f32_w(const PairParams &P, WaveArea A, int lane, float rx,
                                     float ry, float rz, float ra, const Unit &U,
                                     const double4 *tpts, const uint2 *tab64, const double *sE,
                                     uint32_t &nrechk) {
  const int nb = P.nb;
  const float AB = P.AB32;
  const double EB = P.EB;
  const double Em = sE[nb > 1 ? nb - 1 : nb];
  const int st = lane & (kWStripe - 1);
  uint32_t *list = A.list;
  const char *pos = (const char *)(U.pos + U.jb);
  const char *tp = (const char *)tpts;
  const int nrec = U.je - U.jb;
  const uint32_t lane32 = (uint32_t)lane << 5;
  uint32_t c1 = 0, c2 = 0, nout = 0;
  double w1 = 0, r1 = 0, w2 = 0, r2 = 0;   // last bin (w1, r1); CLS 2 also bin nb - 2
  int head = 0, tail = 0;                   // wave-uniform: pending entries list[head, tail)
  int listed = 0;                           // wave-uniform: pairs evaluated in binary64
  int pn = 0;                               // lanes of the batch in flight (0: none)
  double4 pq = make_double4(0, 0, 0, 0), pt = pq;
  auto issue = [&](int n) {
    const uint32_t e = list[head + lane];
    // idle lanes read tile point 0 and record 0 (a short last tile has no
    // point 63, and stale entries may name any record)
    const bool v = lane < n;
    const uint32_t toff = v ? (e & 0x7E0u) : 0u;
    const uint32_t joff = v ? ((e >> 6) & ~31u) : 0u;
    pq = *(const double4 *)(pos + joff);
    pt = *(const double4 *)(tp + toff);
    pn = n;
    listed += n;
    head += 64;
  };
  // FULL: all 64 lanes hold a pair
  auto finish = [&](auto full) {
    constexpr bool FULL = decltype(full)::value;
    const bool v = FULL || lane < pn;
    double dx = pq.x - pt.x, dy = pq.y - pt.y, dz = pq.z - pt.z;
    if (SH) {
      dx = dx + U.S[0];
      dy = dy + U.S[1];
      dz = dz + U.S[2];
    }
    const double s = (dx * dx + dy * dy) + dz * dz;
    const double r = sep_sqrt(s);
    if (CLS == 0) {
      if (v) {
        const int slot = slot64(tab64, P.tab64_lo, P.tab64_hi, P.tab_shift, sE, nb, s);
        const double ww = pt.w * pq.w;
        atomicAdd(&A.hist[slot * 64 + lane], 1u);
        add_w(A.hw + 2 * (slot * kWStripe + st), ww, ww * r);
        nout += slot > nb ? 1u : 0u;
      }
    } else {
      const bool in = v && s < EB;
      const double ww = in ? pt.w * pq.w : 0.0;
      if (CLS == 1) {
        c1 += in ? 1u : 0u;
        w1 += ww;
        r1 = __builtin_fma(ww, r, r1);
      } else {
        const bool hi = s >= Em;
        const double a = hi ? ww : 0.0;
        const double b = ww - a;   // exact: ww or 0
        c1 += (in && hi) ? 1u : 0u;
        c2 += (in && !hi) ? 1u : 0u;
        w1 += a;
        r1 = __builtin_fma(a, r, r1);
        w2 += b;
        r2 = __builtin_fma(b, r, r2);
      }
    }
    pn = 0;
  };
  // full batches: evaluate the one in flight, load the next; the fewer than
  // 64 entries left over move to the front of the list
  auto service = [&]() {
    __builtin_amdgcn_wave_barrier();
    if (tail - head >= 64) {
      do {
        if (pn) finish(std::true_type());
        issue(64);
      } while (tail - head >= 64);
      const uint32_t rest = list[min(head + lane, kListCap - 1)];
      __builtin_amdgcn_wave_barrier();
      if (lane < tail - head) list[lane] = rest;
      tail -= head;
      head = 0;
    }
    __builtin_amdgcn_wave_barrier();
  };
  auto screen = [&](int jr, bool check, float qx, float qy, float qz, float qw) {
    const float d = gram3(rx, ry, rz, ra, qx, qy, qz, qw);
    const bool keep = d < AB && (!check || jr < nrec);
    const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
    if (m) {
      const uint32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      if (keep) list[tail + at] = ((uint32_t)jr << 11) | lane32;
      tail += (int)__popcll(m);
    }
  };
  sfloat *p = (sfloat *)(U.strm + U.jb);
  float a[16];
  CP_LOAD16(a, p);
  for (int jr = 0; jr < nrec; jr += 4) {
    wait_lgkm();
    service();
    float b[16];
    CP_LOAD16(b, p + 16);
    if (jr + 4 <= nrec) {
#pragma unroll
      for (int u = 0; u < 4; u++)
        screen(jr + u, false, a[4 * u], a[4 * u + 1], a[4 * u + 2], a[4 * u + 3]);
    } else {
#pragma unroll
      for (int u = 0; u < 4; u++)
        screen(jr + u, true, a[4 * u], a[4 * u + 1], a[4 * u + 2], a[4 * u + 3]);
    }
#pragma unroll
    for (int t = 0; t < 16; t++) a[t] = b[t];
    p += 16;
  }
  service();
  if (pn) finish(std::true_type());
  if (tail > head) {
    issue(tail - head);
    finish(std::false_type());
  }
  if (CLS == 0) {
    nrechk += nout;
  } else {
    // listed pairs that binary64 placed at or beyond E_B
    const unsigned long long kept = wave_sum_u64((unsigned long long)(c1 + c2));
    if (lane == 0) nrechk += (uint32_t)(listed - (int)kept);
    atomicAdd(&A.hist[nb * 64 + lane], c1);
    add_w(A.hw + 2 * (nb * kWStripe + st), w1, r1);
  }
  if (CLS == 2 && nb > 1) {
    atomicAdd(&A.hist[(nb - 1) * 64 + lane], c2);
    add_w(A.hw + 2 * ((nb - 1) * kWStripe + st), w2, r2);
  }
}

// ---------------------------------------------------------------- FP64 loops

// xi, binary64, two-slot unit: one exact compare per pair.  exec = valid lanes.
template <bool SHIFT>
__device__ inline void loop_xi_f64_two(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                       const Unit &U, const double *sE) {
  const double Et = sE[U.slot_lo];
  const int nb = P.nb;
  const int wrapax[3] = {0, 0, 0};
  uint32_t chi = 0;
  stream_f64(U.pos, U.jb, U.je, [&](int j, double ux, double uy, double uz, double uw) {
    double dx, dy, dz;
    ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, 0.0, 0.0, dx, dy, dz);
    const double s64 = (dx * dx + dy * dy) + dz * dz;
    chi += s64 >= Et ? 1u : 0u;
  });
  const uint32_t clo = (uint32_t)(U.je - U.jb) - chi;
  if (U.slot_lo >= 1) atomicAdd(&A.hist[U.slot_lo * 64 + lane], clo);
  if (U.slot_hi <= nb) atomicAdd(&A.hist[U.slot_hi * 64 + lane], chi);
}

// Weighted xi, binary64, two-slot unit (register sums of w_j and w_j r per
// slot; w_i is applied once at the end).  HIREAL: both slots are bins, so
// every pair is counted; otherwise the upper slot lies beyond R_max and
// only pairs below E_t count.  exec = valid lanes.
template <bool SHIFT, bool HIREAL>
__device__ inline void loop_xi_f64_two_w(const PairParams &P, WaveArea A, const LanePt &L,
                                         int lane, const Unit &U, const double *sE) {
  const double Et = sE[U.slot_lo];
  const int wrapax[3] = {0, 0, 0};
  uint32_t nhi = 0;
  double wlo = 0, whi = 0, rlo = 0, rhi = 0;
  stream_f64(U.pos, U.jb, U.je, [&](int j, double ux, double uy, double uz, double uw) {
    double dx, dy, dz;
    ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, 0.0, 0.0, dx, dy, dz);
    const double s64 = (dx * dx + dy * dy) + dz * dz;
    const bool hi = s64 >= Et;
    nhi += hi ? 1u : 0u;
    if (HIREAL) {
      const double r = sep_sqrt(s64);
      const double a = hi ? uw : 0.0;
      const double c = uw - a;   // exact: uw or 0
      wlo += c;
      rlo = __builtin_fma(c, r, rlo);
      whi += a;
      rhi = __builtin_fma(a, r, rhi);
    } else if (!hi) {
      wlo += uw;
      rlo = __builtin_fma(uw, sep_sqrt(s64), rlo);
    }
  });
  const uint32_t nlo = (uint32_t)(U.je - U.jb) - nhi;
  if (U.slot_lo >= 1) {
    atomicAdd(&A.hist[U.slot_lo * 64 + lane], nlo);
    add_w(A.hw + 2 * (U.slot_lo * kWStripe + (lane & (kWStripe - 1))), L.w * wlo, L.w * rlo);
  }
  if (HIREAL) {
    atomicAdd(&A.hist[U.slot_hi * 64 + lane], nhi);
    add_w(A.hw + 2 * (U.slot_hi * kWStripe + (lane & (kWStripe - 1))), L.w * whi, L.w * rhi);
  }
}

// xi, binary64, a unit whose pairs can only land in slot_lo .. slot_lo + 2:
// two exact compares per pair against E_a = E[slot_lo], E_b = E[slot_lo + 1]
// and register counts (and, weighted, register sums of w_j and w_j r per
// slot, w_i applied once at the end), so the pairs need neither the decision
// table nor LDS atomics.  A slot below E_0 is evaluated and then dropped;
// HIREAL: the top slot is a bin, otherwise it lies beyond E_B and its pairs
// skip the square root.  exec = valid lanes.
template <bool SHIFT, int W, bool HIREAL>
__device__ inline void loop_xi_f64_three(const PairParams &P, WaveArea A, const LanePt &L,
                                         int lane, const Unit &U, const double *sE) {
  const int s0 = U.slot_lo, nb = P.nb;
  const double Ea = sE[s0], Eb = sE[s0 + 1];
  const int wrapax[3] = {0, 0, 0};
  uint32_t n0 = 0, n2 = 0;
  double w0 = 0, w1 = 0, w2 = 0, r0 = 0, r1 = 0, r2 = 0;
  stream_f64(U.pos, U.jb, U.je, [&](int, double ux, double uy, double uz, double uw) {
    double dx, dy, dz;
    ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, 0.0, 0.0, dx, dy, dz);
    const double s64 = (dx * dx + dy * dy) + dz * dz;
    const bool lo = s64 < Ea, hi = s64 >= Eb;
    n0 += lo ? 1u : 0u;
    n2 += hi ? 1u : 0u;
    if (W && HIREAL) {
      const double r = sep_sqrt(s64);
      const double a = lo ? uw : 0.0;
      const double c = hi ? uw : 0.0;
      const double b = (uw - a) - c;   // exact: uw or 0
      w0 += a;
      r0 = __builtin_fma(a, r, r0);
      w1 += b;
      r1 = __builtin_fma(b, r, r1);
      w2 += c;
      r2 = __builtin_fma(c, r, r2);
    } else if (W && !hi) {
      const double r = sep_sqrt(s64);
      const double a = lo ? uw : 0.0;
      const double b = uw - a;         // exact: uw or 0
      w0 += a;
      r0 = __builtin_fma(a, r, r0);
      w1 += b;
      r1 = __builtin_fma(b, r, r1);
    }
  });
  const uint32_t n1 = (uint32_t)(U.je - U.jb) - n0 - n2;
  const int st = lane & (kWStripe - 1);
  if (s0 >= 1) {
    atomicAdd(&A.hist[s0 * 64 + lane], n0);
    if (W) add_w(A.hw + 2 * (s0 * kWStripe + st), L.w * w0, L.w * r0);
  }
  atomicAdd(&A.hist[(s0 + 1) * 64 + lane], n1);
  if (W) add_w(A.hw + 2 * ((s0 + 1) * kWStripe + st), L.w * w1, L.w * r1);
  if (s0 + 2 <= nb) {
    atomicAdd(&A.hist[(s0 + 2) * 64 + lane], n2);
    if (W) add_w(A.hw + 2 * ((s0 + 2) * kWStripe + st), L.w * w2, L.w * r2);
  }
}

template <int MODE, bool OWN, bool SHIFT, bool WRAP, int W>
__device__ inline void loop_f64(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                const Unit &U, const int wrapax[3], double box, double half,
                                const uint2 *tab64, const double *sE) {
  const double EB = P.EB;
  const int lo = P.tab64_lo, sh = P.tab_shift;
  const uint2 *tb = tab64 - lo;
  const int nb = P.nb, npi = P.npi;
  const float inv32 = P.inv_dpi32, pd = P.pi_delta64, pd1 = 1.0f - P.pi_delta64;
  stream_f64(U.pos, U.jb, U.je, [&](int j, double ux, double uy, double uz, double uw) {
    double dx, dy, dz;
    ref_sep<SHIFT, WRAP>(L.x, L.y, L.z, ux, uy, uz, U.S, wrapax, box, half, dx, dy, dz);
    const double rp2 = dx * dx + dy * dy;
    if (MODE == XI) {
      const double s64 = rp2 + dz * dz;
      bool inr = s64 < EB;
      if (OWN) inr = inr && (j > L.iloc);
      if (inr) {
        const int slot = slot64_below(tb, lo, sh, sE, nb, s64);
        atomicAdd(&A.hist[slot * 64 + lane], 1u);
        if (W) {
          const double ww = L.w * uw;
          add_w(A.hw + 2 * (slot * kWStripe + (lane & (kWStripe - 1))), ww, ww * sep_sqrt(s64));
        }
      }
    } else {
      const double pz64 = fabs(dz);
      bool inr = (rp2 < EB) && (pz64 < P.pimax);
      if (OWN) inr = inr && (j > L.iloc);
      if (inr) {
        const int slot = slot64_below(tb, lo, sh, sE, nb, rp2);
        const int l = pibin_fast(pz64, inv32, pd, pd1, P.dpi, P.inv_dpi, npi);
        const int c = (slot * npi + l) * P.wpc + (lane & (P.wpc - 1));
        atomicAdd(&A.hist[c], 1u);
        if (W) {
          const double ww = L.w * uw;
          add_w(A.hw + 2 * c, ww, ww * sep_sqrt(rp2));
        }
      }
    }
  });
}

// ------------------------------------------------------------------ kernel

// Waves per SIMD the register allocation aims at: five (96 VGPRs) for most
// instances; weighted xi with the binary32 filter holds a pair list per wave
// and fits four workgroups per CU in LDS, so it takes the 128 VGPRs of four.
template <int MODE, int PREC, int W> struct PairOcc {
  static constexpr int waves = xi_f32_weighted(MODE, PREC, W) ? 4 : 5;
};

template <int MODE, int PREC, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PairOcc<MODE, PREC, W>::waves)))
void k_pairs(PairParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  // bit k: a wave of this workgroup found queue k drained.  Queues only
  // drain, so the other waves skip it without another device-scope atomic:
  // at the end of a launch every wave otherwise tried all eight heads, and
  // those atomics queued at the memory side with other waves' misses behind
  // them.
  __shared__ uint32_t qdrained;
  if (threadIdx.x == 0) qdrained = 0u;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int n32 = (PREC == F32R && !xi_f32_weighted(MODE, PREC, W)) ? P.tab32_hi - P.tab32_lo + 1 : 0;
  const int n64 = P.tab64_hi - P.tab64_lo + 1;
  const int nx = MODE == WPXI ? P.tabx_hi - P.tabx_lo + 1 : 0;
  const LdsLayout LY = lds_layout(MODE, PREC, W, n32, n64, P.nb, P.npi, P.wpc, nx, P.nbx);
  uint2 *tab32 = (uint2 *)(smem + LY.tab32);
  uint2 *tab64 = (uint2 *)(smem + LY.tab64);
  double *sE = (double *)(smem + LY.E);
  for (int t = threadIdx.x; t < n32; t += blockDim.x) tab32[t] = P.tab32[t];
  for (int t = threadIdx.x; t < n64; t += blockDim.x) tab64[t] = P.tab64[t];
  for (int t = threadIdx.x; t <= P.nb; t += blockDim.x) sE[t] = P.E[t];
  uint2 *tabx = (uint2 *)(smem + LY.tabx);
  double *sEx = (double *)(smem + LY.Ex);
  if (MODE == WPXI) {
    for (int t = threadIdx.x; t < nx; t += blockDim.x) tabx[t] = P.tabx[t];
    for (int t = threadIdx.x; t <= P.nbx; t += blockDim.x) sEx[t] = P.Ex[t];
  }
  unsigned char *wb = smem + LY.common + (size_t)wid * LY.wave_bytes;
  WaveArea A;
  A.hist = (uint32_t *)wb;
  A.hw = (double *)(wb + LY.wave_hist);
  A.list = (uint32_t *)(wb + LY.wave_list);
  A.histx = (uint32_t *)(wb + LY.wave_histx);
  if (MODE == WPXI) {
    for (int t = lane; t < (P.nbx + 2) * 32; t += 64) A.histx[t] = 0u;
  }
  const int NS = P.nslots;
  const int hwords = MODE == XI ? NS * 64 : NS * P.npi * P.wpc;
  const int wwords = MODE == XI ? NS * kWStripe : hwords;
  for (int t = lane; t < hwords; t += 64) A.hist[t] = 0u;
  if (W) {
    for (int t = lane; t < wwords; t += 64) {
      A.hw[2 * t] = 0.0;
      A.hw[2 * t + 1] = 0.0;
    }
  }
  __syncthreads();

  unsigned long long st_cand = 0, st_cells = 0, st_pruned = 0;
  uint32_t nrechk = 0;
  const int64_t nsplit = P.nsplit;
  const int64_t ntiles = *P.ntiles;
  const int64_t nitems = ntiles * nsplit;
  if (blockIdx.x == 0 && threadIdx.x == 0) P.stats[4] = (unsigned long long)ntiles;
  unsigned long long *heads = P.stats + 5;
  const int home = (int)(blockIdx.x % kQueues);
  int victim = 0;   // queues found empty so far, counted from the home queue
  int cur_mock = -1;
  unsigned long long since_flush = 0;
  const unsigned long long flush_limit = MODE == XI ? (1ull << 30) : (1ull << 24);

  for (;;) {
    int64_t tix = -1;
    if (lane == 0) {
      while (victim < kQueues) {
        const int k = (home + victim) % kQueues;
        const int64_t qb = nitems * k / kQueues, qe = nitems * (k + 1) / kQueues;
        if ((*(volatile uint32_t *)&qdrained >> k) & 1u) {
          victim++;
          continue;
        }
        const int64_t i = (int64_t)atomicAdd(&heads[k * kQStride], 1ull);
        if (qb + i < qe) {
          tix = qb + i;
          break;
        }
        atomicOr(&qdrained, 1u << k);
        victim++;
      }
    }
    tix = uni64(__shfl(tix, 0));
    if (tix < 0) break;
    // item = (tile, chunk of its neighbour columns): consecutive items share
    // a tile, so its chunks run on different waves at the same time
    const int64_t tile_ix = tix / nsplit;
    const int part = (int)(tix - tile_ix * nsplit);
    const Tile T = P.tiles[tile_ix];
    const int mock = uni(T.mock);
    if (mock != cur_mock) {
      if (cur_mock >= 0) flush_hist<MODE, W>(P, A, cur_mock, lane);
      cur_mock = mock;
      since_flush = 0;
    }
    const GridGeom &G1 = P.geom1[mock];
    const GridGeom &G2 = P.geom2[mock];
    const int tn = uni(T.n);
    const int64_t tp0 = uni64(T.p0);
    const int tcol = uni(T.col), tz0 = uni(T.cz0), tz1 = uni(T.cz1);
    const bool valid = lane < tn;
    const double4 pp = P.pos1[tp0 + (valid ? lane : 0)];
    LanePt L;
    L.x = valid ? pp.x : kNoPoint;
    L.y = valid ? pp.y : kNoPoint;
    L.z = valid ? pp.z : kNoPoint;
    L.w = pp.w;
    L.iloc = (int)(tp0 + lane - G1.pbase);
    // tile bounding box
    const double blx = uni_d(wave_min(valid ? pp.x : DBL_MAX));
    const double bly = uni_d(wave_min(valid ? pp.y : DBL_MAX));
    const double blz = uni_d(wave_min(valid ? pp.z : DBL_MAX));
    const double bhx = uni_d(wave_max(valid ? pp.x : -DBL_MAX));
    const double bhy = uni_d(wave_max(valid ? pp.y : -DBL_MAX));
    const double bhz = uni_d(wave_max(valid ? pp.z : -DBL_MAX));
    const int nvalid = tn;

    const int ny = G2.n[1], nz = G2.n[2];
    const int cx = tcol / ny, cy = tcol % ny;
    const int rx = G2.r[0], ry = G2.r[1], rz = G2.r[2];
    const int nzr = (tz1 - tz0) + 2 * rz + 1;
    const int ncy = 2 * ry + 1;
    const int col0 = P.chunk[part];
    const int total = (P.chunk[part + 1] - col0) * nzr;
    const double box = G2.box, half = G2.halfbox;
    const int wrapax[3] = {G2.wrap[0], G2.wrap[1], G2.wrap[2]};
    const bool anywrap = wrapax[0] | wrapax[1] | wrapax[2];
    const int64_t pbase2 = G2.pbase;

    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      int keep = 0, pruned = 0, cell = 0, packed = 0, slots = 0, win = 0, wzlo = 0, wzhi = 0;
      int mrg = 0;   // binary64: may join a run of z-cells (z-sorted, windows computable)
      if (t < total) {
        // column of the tile's list (order fixed by the host's split) and
        // z offset; an auto-count searches its own column forward in z only,
        // cells inside the tile's own z range with a per-pair j > i test
        const int oz = t % nzr;
        const int col = col0 + t / nzr;
        int ox, oy;
        if (P.autocorr) {
          if (col <= ry) {
            ox = 0;
            oy = col;
          } else {
            ox = 1 + (col - 1 - ry) / ncy;
            oy = (col - 1 - ry) % ncy - ry;
          }
        } else {
          ox = col / ncy - rx;
          oy = col % ncy - ry;
        }
        int X = cx + ox, Y = cy + oy, Z = tz0 - rz + oz;
        int sx = 0, sy = 0, sz = 0;
        bool ok = true;
        int own = 0;
        if (P.autocorr && col == 0) {
          if (oz < rz) ok = false;
          else if (oz - rz <= tz1 - tz0) own = 1;
        }
        if (X < 0) { if (G2.periodic) { X += G2.n[0]; sx = -1; } else ok = false; }
        else if (X >= G2.n[0]) { if (G2.periodic) { X -= G2.n[0]; sx = 1; } else ok = false; }
        if (Y < 0) { if (G2.periodic) { Y += ny; sy = -1; } else ok = false; }
        else if (Y >= ny) { if (G2.periodic) { Y -= ny; sy = 1; } else ok = false; }
        if (Z < 0) { if (G2.periodic) { Z += nz; sz = -1; } else ok = false; }
        else if (Z >= nz) { if (G2.periodic) { Z -= nz; sz = 1; } else ok = false; }
        if (ok) cell = (X * ny + Y) * nz + Z;
        if (ok) {
          const int b = P.cstart2[G2.sbase + cell], e = P.cstart2[G2.sbase + cell + 1];
          if (e == b) {
            ok = false;
          } else {
            // Minimum possible separation of the tile's and the cell's
            // bounding boxes, evaluated with the reference operation
            // sequence so the bound never exceeds any member pair's s.
            const CellBox B = P.cbox2[G2.cbase + cell];
            const double S0 = sx * box, S1 = sy * box, S2 = sz * box;
            const double tl[3] = {blx, bly, blz}, th[3] = {bhx, bhy, bhz};
            const double Sv[3] = {S0, S1, S2};
            // The largest possible separation is bounded the same way, so
            // every pair of the unit falls in [slot(lower), slot(upper)].
            double m[3], M[3];
            for (int a = 0; a < 3; a++) {
              double gl = B.lo[a] - th[a];
              double gh = B.hi[a] - tl[a];
              if (Sv[a] != 0.0) {
                gl = gl + Sv[a];
                gh = gh + Sv[a];
              }
              m[a] = gl > 0.0 ? gl : (gh < 0.0 ? -gh : 0.0);
              M[a] = fmax(fabs(gl), fabs(gh));
              if (wrapax[a]) {
                m[a] = 0.0;
                M[a] = half;
              }
            }
            const double rp = m[0] * m[0] + m[1] * m[1];
            bool far;
            if (MODE == XI) far = (rp + m[2] * m[2]) >= P.EB;
            else far = (rp >= P.EB) || (m[2] >= P.pimax);
            if (far && !P.noprune) {
              ok = false;
              pruned = 1;
            } else {
              if (MODE == XI) {
                const double slo = rp + m[2] * m[2];
                const double shi = (M[0] * M[0] + M[1] * M[1]) + M[2] * M[2];
                slots = exact_slot(sE, P.nb, slo) | (exact_slot(sE, P.nb, shi) << 8);
              }
              // z-window of the unit in the cell's own coordinates (Section
              // 2.2, late entry / early exit): a pair within reach has
              // |dz| <= hz, so only the cell's z-sorted points in
              // [zmin_tile - S - hz, zmax_tile - S + hz] can pair; the slack
              // terms cover binary64 rounding many times over.
              if (!P.noprune && !anywrap && e - b <= kZSortMax) {
                // (binary32 square root with a 1e-5 relative allowance: the
                // window needs no more precision and stays free of binary64
                // FMAs)
                double hz = MODE == XI
                                ? (double)sqrtf((float)(fmax(P.EB - rp, 0.0) + 1e-12 * P.EB)) *
                                      (1.0 + 1e-5)
                                : P.pimax * (1.0 + 1e-9);
                hz = hz + 1e-9 * (fabs(blz) + fabs(bhz) + fabs(S2) + 1.0);
                const double zl = blz - S2 - hz, zh = bhz - S2 + hz;
                const bool cut = zl > B.lo[2] || zh < B.hi[2];
                // (a run of cells takes the union of their windows, so each
                // keeps its bounds)
                if (cut || PREC == F64) {
                  wzlo = __float_as_int(__double2float_rd(zl));
                  wzhi = __float_as_int(__double2float_ru(zh));
                }
                win = cut ? 1 : 0;
                mrg = PREC == F64 && MODE != WPXI ? 1 : 0;
              }
            }
          }
        }
        if (ok) {
          // shift code per axis (-1, 0, +1 -> 0, 1, 2) in bits 1..6 of keep,
          // z-window flag in bit 7, run flag in bit 8
          keep = 1 | ((sx + 1) << 1) | ((sy + 1) << 3) | ((sz + 1) << 5) | (win << 7) | (mrg << 8);
          packed = X | (Y << 10) | (Z << 20) | (own << 30);
        }
      }
      unsigned long long mk = __builtin_amdgcn_ballot_w64(keep != 0);
      st_pruned += __popcll(__builtin_amdgcn_ballot_w64(pruned != 0));
      while (mk) {
        const int src = __builtin_ctzll(mk);
        mk &= mk - 1;
        const int c2 = __builtin_amdgcn_readlane(cell, src);
        const int pk = __builtin_amdgcn_readlane(packed, src);
        const int kc = __builtin_amdgcn_readlane(keep, src);
        const int sl = __builtin_amdgcn_readlane(slots, src);
        // binary64: the following lanes' cells that continue this column
        // upwards in z with the same shift and own flag join the unit (cells
        // are stored z-fastest, so the run's records are contiguous and,
        // z-sorted per cell, sorted as a whole; the binary64 loops read
        // absolute positions, while the binary32 records are in each cell's
        // own frame, which a run would have to switch at every cell).  xi
        // joins cells of the same slot range, or any cells the general loop
        // takes (own, or more than three slots); the run's z-window is the
        // union of its cells' windows.
        int nrun = 1, winr = kc & 128, slr = sl;
        float wl = 0.f, wh = 0.f;
        if (PREC == F64 && MODE != WPXI && (kc & 256)) {
          auto general = [&](int v, int p) {
            return ((p >> 30) & 1) || ((v >> 8) & 255) - (v & 255) > 2;
          };
          const bool gen = MODE == XI && general(sl, pk);
          int last = src, pl = pk;
          wl = __int_as_float(__builtin_amdgcn_readlane(wzlo, src));
          wh = __int_as_float(__builtin_amdgcn_readlane(wzhi, src));
          while (last < 63 && ((mk >> (last + 1)) & 1ull)) {
            const int pk2 = __builtin_amdgcn_readlane(packed, last + 1);
            const int kc2 = __builtin_amdgcn_readlane(keep, last + 1);
            if (pk2 != pl + (1 << 20) || ((kc2 ^ kc) & 0x7E) || !(kc2 & 256)) break;
            if (MODE == XI) {
              const int sl2 = __builtin_amdgcn_readlane(slots, last + 1);
              if (gen ? !general(sl2, pk2) : sl2 != sl) break;
              slr = min(slr & 255, sl2 & 255) | (max((slr >> 8) & 255, (sl2 >> 8) & 255) << 8);
            }
            last++;
            mk &= ~(1ull << last);
            nrun++;
            pl = pk2;
            winr |= kc2 & 128;
            wl = fminf(wl, __int_as_float(__builtin_amdgcn_readlane(wzlo, last)));
            wh = fmaxf(wh, __int_as_float(__builtin_amdgcn_readlane(wzhi, last)));
          }
        }
        const int X = pk & 1023, Y = (pk >> 10) & 1023, Z = (pk >> 20) & 1023;
        const bool own = (pk >> 30) & 1;
        const int sxx = ((kc >> 1) & 3) - 1, syy = ((kc >> 3) & 3) - 1, szz = ((kc >> 5) & 3) - 1;
        const bool shifted = (sxx | syy | szz) != 0;
        sint *CS = (sint *)P.cstart2;
        Unit U;
        U.S[0] = sxx * box;
        U.S[1] = syy * box;
        U.S[2] = szz * box;
        U.strm = P.strm2 + pbase2;
        U.pos = P.pos2 + pbase2;
        U.jb = CS[G2.sbase + c2];
        U.je = CS[G2.sbase + c2 + nrun];
        U.slot_lo = slr & 255;
        U.slot_hi = (slr >> 8) & 255;
        if (winr) {
          const float zlo = nrun > 1 ? wl : __int_as_float(__builtin_amdgcn_readlane(wzlo, src));
          const float zhi = nrun > 1 ? wh : __int_as_float(__builtin_amdgcn_readlane(wzhi, src));
          zwindow(U.pos, zlo, zhi, lane, U.jb, U.je);
          if (U.je <= U.jb) continue;
        }
        const unsigned long long nj = (unsigned long long)(U.je - U.jb);
        st_cells += (unsigned long long)nrun;
        since_flush += nj;
        if (since_flush > flush_limit) {
          flush_hist<MODE, W>(P, A, cur_mock, lane);
          since_flush = nj;
        }
        // all pairs of the unit in one bin: count them without separations
        if (MODE == XI && !W && !own && !anywrap && !P.noprune && U.slot_lo == U.slot_hi) {
          if (U.slot_lo >= 1 && U.slot_lo <= P.nb && valid)
            atomicAdd(&A.hist[U.slot_lo * 64 + lane], (uint32_t)nj);
          continue;
        }
        st_cand += (unsigned long long)nvalid * nj;
        const bool two = MODE == XI && !own && !anywrap && U.slot_hi == U.slot_lo + 1;
        // weighted xi in binary32 mode: units with every pair in [E_0, E_B)
        // need the binary64 separation of every pair anyway (binary64 loops);
        // units that reach past E_B are screened in binary32 and only the
        // kept pairs are evaluated in binary64
        const bool f32w = xi_f32_weighted(MODE, PREC, W);
        const bool allin = U.slot_lo >= 1 && U.slot_hi <= P.nb;
        if (f32w && !anywrap && !own && !allin && nj < (1ull << 21)) {
          const double ox = frame_origin(G2, 0, X) + U.S[0];
          const double oy = frame_origin(G2, 1, Y) + U.S[1];
          const double oz = frame_origin(G2, 2, Z) + U.S[2];
          const float rxf = valid ? (float)(L.x - ox) : 1e18f;
          const float ryf = valid ? (float)(L.y - oy) : 1e18f;
          const float rzf = valid ? (float)(L.z - oz) : 1e18f;
          const float ra = __builtin_fmaf(rzf, rzf, __builtin_fmaf(ryf, ryf, rxf * rxf));
          const double4 *tpts = P.pos1 + tp0;
          const int nb = P.nb;
#define CP_XW(C, SH) loop_xi_f32_w<C, SH>(P, A, lane, rxf, ryf, rzf, ra, U, tpts, tab64, sE, nrechk)
          if (U.slot_lo == nb && U.slot_hi == nb + 1) {
            if (shifted) CP_XW(1, true); else CP_XW(1, false);
          } else if (nb >= 2 && U.slot_lo == nb - 1 && U.slot_hi == nb + 1) {
            if (shifted) CP_XW(2, true); else CP_XW(2, false);
          } else {
            if (shifted) CP_XW(0, true); else CP_XW(0, false);
          }
#undef CP_XW
        } else if (PREC == F32R && !anywrap && !f32w) {
          const double ox = frame_origin(G2, 0, X) + U.S[0];
          const double oy = frame_origin(G2, 1, Y) + U.S[1];
          const double oz = frame_origin(G2, 2, Z) + U.S[2];
          const float rxf = valid ? (float)(L.x - ox) : 1e18f;
          const float ryf = valid ? (float)(L.y - oy) : 1e18f;
          const float rzf = valid ? (float)(L.z - oz) : 1e18f;
          // The binary32 loops take the shift as data: it only enters the
          // rare binary64 re-evaluations, where adding a zero shift is exact,
          // so one instance serves shifted and unshifted units (a smaller
          // kernel, kinder to the instruction cache).
          if (MODE == XI) {
            const float ra = __builtin_fmaf(rzf, rzf, __builtin_fmaf(ryf, ryf, rxf * rxf));
            if (two) {
              if (valid) loop_xi_f32_two<true>(P, A, L, lane, rxf, ryf, rzf, ra, U, sE, nrechk);
            } else if (!own && U.slot_hi == U.slot_lo + 2) {
              if (valid) loop_xi_f32_three<true>(P, A, L, lane, rxf, ryf, rzf, ra, U, sE, nrechk);
            } else {
              if (own) loop_xi_f32<true, true>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, nrechk);
              else loop_xi_f32<false, true>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, nrechk);
            }
          } else if (MODE == WPXI) {
            const float ra = __builtin_fmaf(ryf, ryf, rxf * rxf);
            if (own) loop_wpxi_f32<true>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, tabx, sEx, nrechk);
            else loop_wpxi_f32<false>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, tabx, sEx, nrechk);
          } else if (!W) {
            const float ra = __builtin_fmaf(ryf, ryf, rxf * rxf);
            if (own) loop_wp_f32<true, true>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, nrechk);
            else loop_wp_f32<false, true>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, nrechk);
          } else {
            // weighted: every in-range pair takes the binary64 separation,
            // where the shift costs an add per axis
            const float ra = __builtin_fmaf(ryf, ryf, rxf * rxf);
#define CP_WP(O, SH) loop_wp_f32_w<O, SH>(P, A, L, lane, rxf, ryf, rzf, ra, U, tab32, sE, nrechk)
            if (own) { if (shifted) CP_WP(true, true); else CP_WP(true, false); }
            else { if (shifted) CP_WP(false, true); else CP_WP(false, false); }
#undef CP_WP
          }
        } else if ((PREC == F64 || f32w) && MODE == XI && !own && !anywrap &&
                   U.slot_hi == U.slot_lo + 2) {
          if (valid) {
            if (!W || U.slot_hi <= P.nb) {
              if (shifted) loop_xi_f64_three<true, W, true>(P, A, L, lane, U, sE);
              else loop_xi_f64_three<false, W, true>(P, A, L, lane, U, sE);
            } else {
              if (shifted) loop_xi_f64_three<true, W, false>(P, A, L, lane, U, sE);
              else loop_xi_f64_three<false, W, false>(P, A, L, lane, U, sE);
            }
          }
        } else if ((PREC == F64 || f32w) && two) {
          if (valid) {
            if (W) {
              if (U.slot_hi <= P.nb) {
                if (shifted) loop_xi_f64_two_w<true, true>(P, A, L, lane, U, sE);
                else loop_xi_f64_two_w<false, true>(P, A, L, lane, U, sE);
              } else {
                if (shifted) loop_xi_f64_two_w<true, false>(P, A, L, lane, U, sE);
                else loop_xi_f64_two_w<false, false>(P, A, L, lane, U, sE);
              }
            } else {
              if (shifted) loop_xi_f64_two<true>(P, A, L, lane, U, sE);
              else loop_xi_f64_two<false>(P, A, L, lane, U, sE);
            }
          }
        } else {
#define CP_F64(O, SH, WR) loop_f64<MODE, O, SH, WR, W>(P, A, L, lane, U, wrapax, box, half, tab64, sE)
          if (anywrap) {
            if (own) CP_F64(true, true, true); else CP_F64(false, true, true);
          } else if (shifted) {
            if (own) CP_F64(true, true, false); else CP_F64(false, true, false);
          } else {
            if (own) CP_F64(true, false, false); else CP_F64(false, false, false);
          }
#undef CP_F64
        }
      }
    }
  }
  if (cur_mock >= 0) flush_hist<MODE, W>(P, A, cur_mock, lane);
  const unsigned long long rc = wave_sum_u64((unsigned long long)nrechk);
  // one atomic instruction for the four statistics (lane k adds word k)
  const unsigned long long sv = lane == 0 ? st_cand : lane == 1 ? rc : lane == 2 ? st_cells : st_pruned;
  if (lane < 4 && sv) atomicAdd(P.stats + lane, sv);
}

template __global__ void k_pairs<XI, F32R, 0>(PairParams);
template __global__ void k_pairs<XI, F32R, 1>(PairParams);
template __global__ void k_pairs<XI, F64, 0>(PairParams);
template __global__ void k_pairs<XI, F64, 1>(PairParams);
template __global__ void k_pairs<WP, F32R, 0>(PairParams);
template __global__ void k_pairs<WP, F32R, 1>(PairParams);
template __global__ void k_pairs<WP, F64, 0>(PairParams);
template __global__ void k_pairs<WP, F64, 1>(PairParams);
template __global__ void k_pairs<WPXI, F32R, 0>(PairParams);

} // namespace cp
