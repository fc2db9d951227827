// Pair kernels: one persistent launch drains a queue of primary tiles.
//
// Work decomposition (MI355X, wave64).  A tile is <= 64 points of one cell
// column; lane l of a wave holds tile point l for the whole tile.  The wave
// walks the neighbouring cells of the tile (Section 1.2: all pairs within
// R_max lie in the neighbouring cells; Section 2.1: for an auto-count only
// unique pairs of cells, here unique pairs of points by sorted index), skips
// cells whose bounding box is too far from the tile's (Section 2.2, minimum
// possible separation), and streams each remaining cell's points through
// the scalar cache so every VALU instruction of the inner loop takes one
// wave-uniform operand from SGPRs and one per-lane operand from VGPRs.
//
// Inner loop, binary32 mode.  Coordinates are held relative to the streamed
// cell's centre, so the squared separation is evaluated as
//   s~ = |r|^2 + |p|^2 - 2 r.p     (r: tile point, p: streamed point)
// in three FMAs and one add; the stream record carries (-2p, |p|^2).  An
// error bound eps on |s~ - s| (s the binary64 value of the reference formula)
// turns each edge E_k into an uncertain band [E_k - eps, E_k + eps); a
// 2-word LDS lookup indexed by the exponent and top mantissa bits of s~ gives
// the bin, or flags the pair for re-evaluation in binary64 with the reference
// formula.  Counts therefore equal the binary64 counts exactly.
//
// Binning (Section 2.2 "Updating the histogram"): the paper scans bins from
// the outermost down with vector masks and popcounts; on a 64-wide wave that
// scan runs about as deep as the innermost bin any lane needs, so here each
// lane instead owns a private row of LDS counters indexed by its bin.
#include "cp_internal.h"

#include <float.h>

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
// q_l = fl(l * dpi).
__device__ inline int exact_pibin(double pz, double dpi, int npi) {
  int l = (int)(pz / dpi);
  if (l < 0) l = 0;
  if (l > npi - 1) l = npi - 1;
  while (l > 0 && pz < (double)l * dpi) l--;
  while (l + 1 < npi && pz >= (double)(l + 1) * dpi) l++;
  return l;
}

// Table lookup: slot for v (binary32 estimate), or uncertain.
struct TabHit {
  int slot;
  bool unc;
};
__device__ inline TabHit tab_lookup(const uint2 *tab, int lo, int hi, int sh, float v) {
  int b = __float_as_int(v) >> sh;
  b = b < lo ? lo : (b > hi ? hi : b);
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

struct WaveArea {
  uint32_t *hist;
  double *hw, *hwr;
};

template <int MODE, int W>
__device__ inline void flush_hist(const PairParams &P, WaveArea A, int mock, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int nb = P.nb, NS = P.nslots;
  unsigned long long *gh = P.hist + (int64_t)mock * P.hist_stride;
  if (MODE == XI) {
    for (int s = 1; s <= nb; s++) {
      unsigned long long v = wave_sum_u64((unsigned long long)A.hist[s * 64 + lane]);
      if (lane == 0 && v) atomicAdd(gh + (s - 1), v);
      if (W) {
        double a = wave_sum_f64(A.hw[s * 64 + lane]);
        double b = wave_sum_f64(A.hwr[s * 64 + lane]);
        if (lane == 0) {
          unsafeAtomicAdd(P.hw + (int64_t)mock * P.hist_stride + (s - 1), a);
          unsafeAtomicAdd(P.hwr + (int64_t)mock * P.hist_stride + (s - 1), b);
        }
      }
    }
    for (int s = 0; s < NS; s++) {
      A.hist[s * 64 + lane] = 0u;
      if (W) {
        A.hw[s * 64 + lane] = 0.0;
        A.hwr[s * 64 + lane] = 0.0;
      }
    }
  } else {
    const int npi = P.npi;
    for (int t = lane; t < nb * npi; t += 64) {
      uint32_t v = A.hist[npi + t];
      if (v) atomicAdd(gh + t, (unsigned long long)v);
      if (W) {
        double a = A.hw[npi + t], b = A.hwr[npi + t];
        if (a != 0.0) unsafeAtomicAdd(P.hw + (int64_t)mock * P.hist_stride + t, a);
        if (b != 0.0) unsafeAtomicAdd(P.hwr + (int64_t)mock * P.hist_stride + t, b);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < NS * npi; t += 64) {
      A.hist[t] = 0u;
      if (W) {
        A.hw[t] = 0.0;
        A.hwr[t] = 0.0;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-lane state of the tile point.
struct LanePt {
  double x, y, z, w;
  int iloc;   // sorted index relative to the catalogue (own-cell ordering)
};

// ---------------------------------------------------------------- FP32 loops

// xi, binary32 filter.  OWN: the streamed cell is one of the tile's own
// cells (auto-count): only j > i pairs.
template <bool OWN, bool SHIFT, int W>
__device__ inline void loop_xi_f32(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                   float rx, float ry, float rz, float ra, int64_t jb, int64_t je,
                                   int64_t pbase, const double S[3], const uint2 *tab32,
                                   const uint2 *tab64, const double *sE, uint32_t &nrechk) {
  sfloat *SP = (sfloat *)P.strm2;
  sdouble *DP = (sdouble *)P.pos2;
  const float AB = P.AB32;
  const int lo = P.tab32_lo, hi = P.tab32_hi, sh = P.tab_shift;
  const int nb = P.nb;
  const int wrapax[3] = {0, 0, 0};
  for (int64_t j = jb; j < je; ++j) {
    const float qx = SP[4 * j], qy = SP[4 * j + 1], qz = SP[4 * j + 2], qw = SP[4 * j + 3];
    float t = __builtin_fmaf(rx, qx, ra);
    t = __builtin_fmaf(ry, qy, t);
    t = __builtin_fmaf(rz, qz, t);
    const float s = t + qw;
    bool inr = s < AB;
    if (OWN) inr = inr && ((int)(j - pbase) > L.iloc);
    if (!inr) continue;
    if (!W) {
      const TabHit h = tab_lookup(tab32, lo, hi, sh, s);
      if (!h.unc) {
        atomicAdd(&A.hist[h.slot * 64 + lane], 1u);
      } else {
        const double ux = DP[4 * j], uy = DP[4 * j + 1], uz = DP[4 * j + 2];
        double dx, dy, dz;
        ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, S, wrapax, 0.0, 0.0, dx, dy, dz);
        const double s64 = (dx * dx + dy * dy) + dz * dz;
        atomicAdd(&A.hist[exact_slot(sE, nb, s64) * 64 + lane], 1u);
        nrechk++;
      }
    } else {
      // weighted: the binary32 bin stands when certain; the separation
      // itself is always taken in binary64 for the weighted sum
      const TabHit h = tab_lookup(tab32, lo, hi, sh, s);
      const double ux = DP[4 * j], uy = DP[4 * j + 1], uz = DP[4 * j + 2], uw = DP[4 * j + 3];
      double dx, dy, dz;
      ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, S, wrapax, 0.0, 0.0, dx, dy, dz);
      const double s64 = (dx * dx + dy * dy) + dz * dz;
      int slot = h.slot;
      if (h.unc) {
        slot = exact_slot(sE, nb, s64);
        nrechk++;
      }
      const double ww = L.w * uw;
      const int a = slot * 64 + lane;
      atomicAdd(&A.hist[a], 1u);
      atomicAdd(&A.hw[a], ww);
      atomicAdd(&A.hwr[a], ww * sqrt(s64));
    }
  }
}

// wp, binary32 filter.
template <bool OWN, bool SHIFT, int W>
__device__ inline void loop_wp_f32(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                   float rx, float ry, float rz, float ra, int64_t jb, int64_t je,
                                   int64_t pbase, const double S[3], const uint2 *tab32,
                                   const uint2 *tab64, const double *sE, uint32_t &nrechk) {
  sfloat *SP = (sfloat *)P.strm2;
  sdouble *DP = (sdouble *)P.pos2;
  const float AB = P.AB32, PIHI = P.pi_hi32, PILO = P.pi_lo32, invd = P.inv_dpi32,
              dlt = P.pi_delta;
  const int lo = P.tab32_lo, hi = P.tab32_hi, sh = P.tab_shift;
  const int nb = P.nb, npi = P.npi;
  const int wrapax[3] = {0, 0, 0};
  for (int64_t j = jb; j < je; ++j) {
    const float qx = SP[4 * j], qy = SP[4 * j + 1], qz = SP[4 * j + 2], qw = SP[4 * j + 3];
    float t = __builtin_fmaf(rx, qx, ra);
    t = __builtin_fmaf(ry, qy, t);
    const float s = t + qw;
    const float pz = fabsf(qz - rz);
    bool inr = (s < AB) && (pz < PIHI);
    if (OWN) inr = inr && ((int)(j - pbase) > L.iloc);
    if (!inr) continue;
    bool unc = true;
    int slot = 0, l = 0;
    if (!W) {
      const TabHit h = tab_lookup(tab32, lo, hi, sh, s);
      const float f = pz * invd;
      const float fl = floorf(f);
      const float fr = f - fl;
      l = min((int)fl, npi - 1);
      slot = h.slot;
      unc = h.unc || (fr < dlt) || (fr > 1.0f - dlt) || (pz >= PILO);
      if (!unc) atomicAdd(&A.hist[slot * npi + l], 1u);
    }
    if (unc) {
      const double ux = DP[4 * j], uy = DP[4 * j + 1], uz = DP[4 * j + 2], uw = DP[4 * j + 3];
      double dx, dy, dz;
      ref_sep<SHIFT, false>(L.x, L.y, L.z, ux, uy, uz, S, wrapax, 0.0, 0.0, dx, dy, dz);
      const double rp2 = dx * dx + dy * dy;
      const double pz64 = fabs(dz);
      if (!W) nrechk++;
      if (pz64 < P.pimax && rp2 < P.EB) {
        const int sl = W ? slot64(tab64, P.tab64_lo, P.tab64_hi, sh, sE, nb, rp2)
                         : exact_slot(sE, nb, rp2);
        const int ll = exact_pibin(pz64, P.dpi, npi);
        atomicAdd(&A.hist[sl * npi + ll], 1u);
        if (W) {
          const double ww = L.w * uw;
          atomicAdd(&A.hw[sl * npi + ll], ww);
          atomicAdd(&A.hwr[sl * npi + ll], ww * sqrt(rp2));
        }
      }
    }
  }
}

// ---------------------------------------------------------------- FP64 loops

template <int MODE, bool OWN, bool SHIFT, bool WRAP, int W>
__device__ inline void loop_f64(const PairParams &P, WaveArea A, const LanePt &L, int lane,
                                int64_t jb, int64_t je, int64_t pbase, const double S[3],
                                const int wrapax[3], double box, double half, const uint2 *tab64,
                                const double *sE) {
  sdouble *DP = (sdouble *)P.pos2;
  const double EB = P.EB;
  const int lo = P.tab64_lo, hi = P.tab64_hi, sh = P.tab_shift;
  const int nb = P.nb, npi = P.npi;
  for (int64_t j = jb; j < je; ++j) {
    const double ux = DP[4 * j], uy = DP[4 * j + 1], uz = DP[4 * j + 2];
    double dx, dy, dz;
    ref_sep<SHIFT, WRAP>(L.x, L.y, L.z, ux, uy, uz, S, wrapax, box, half, dx, dy, dz);
    const double rp2 = dx * dx + dy * dy;
    if (MODE == XI) {
      const double s64 = rp2 + dz * dz;
      bool inr = s64 < EB;
      if (OWN) inr = inr && ((int)(j - pbase) > L.iloc);
      if (!inr) continue;
      const int slot = slot64(tab64, lo, hi, sh, sE, nb, s64);
      atomicAdd(&A.hist[slot * 64 + lane], 1u);
      if (W) {
        const double ww = L.w * DP[4 * j + 3];
        atomicAdd(&A.hw[slot * 64 + lane], ww);
        atomicAdd(&A.hwr[slot * 64 + lane], ww * sqrt(s64));
      }
    } else {
      const double pz64 = fabs(dz);
      bool inr = (rp2 < EB) && (pz64 < P.pimax);
      if (OWN) inr = inr && ((int)(j - pbase) > L.iloc);
      if (!inr) continue;
      const int slot = slot64(tab64, lo, hi, sh, sE, nb, rp2);
      const int l = exact_pibin(pz64, P.dpi, npi);
      atomicAdd(&A.hist[slot * npi + l], 1u);
      if (W) {
        const double ww = L.w * DP[4 * j + 3];
        atomicAdd(&A.hw[slot * npi + l], ww);
        atomicAdd(&A.hwr[slot * npi + l], ww * sqrt(rp2));
      }
    }
  }
}

// ------------------------------------------------------------------ kernel

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

struct LdsLayout {
  size_t tab32, tab64, E, common, wave_hist, wave_w, wave_bytes;
};

__host__ __device__ inline LdsLayout lds_layout(int mode, int prec, int weighted, int n32, int n64,
                                               int nb, int npi) {
  LdsLayout L;
  size_t off = 0;
  L.tab32 = off;
  off += (size_t)(prec == F32R ? n32 : 0) * 8;
  L.tab64 = off;
  off += (size_t)n64 * 8;
  L.E = off;
  off += (size_t)(nb + 1) * 8;
  L.common = align16(off);
  const int NS = nb + 2;
  const size_t words = mode == XI ? (size_t)NS * 64 : (size_t)NS * npi;
  L.wave_hist = align16(words * 4);
  L.wave_w = weighted ? words * 8 : 0;
  L.wave_bytes = L.wave_hist + 2 * L.wave_w;
  return L;
}

template <int MODE, int PREC, int W>
__global__ __launch_bounds__(256) void k_pairs(PairParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int n32 = PREC == F32R ? P.tab32_hi - P.tab32_lo + 1 : 0;
  const int n64 = P.tab64_hi - P.tab64_lo + 1;
  const LdsLayout LY = lds_layout(MODE, PREC, W, n32, n64, P.nb, P.npi);
  uint2 *tab32 = (uint2 *)(smem + LY.tab32);
  uint2 *tab64 = (uint2 *)(smem + LY.tab64);
  double *sE = (double *)(smem + LY.E);
  for (int t = threadIdx.x; t < n32; t += blockDim.x) tab32[t] = P.tab32[t];
  for (int t = threadIdx.x; t < n64; t += blockDim.x) tab64[t] = P.tab64[t];
  for (int t = threadIdx.x; t <= P.nb; t += blockDim.x) sE[t] = P.E[t];
  unsigned char *wb = smem + LY.common + (size_t)wid * LY.wave_bytes;
  WaveArea A;
  A.hist = (uint32_t *)wb;
  A.hw = (double *)(wb + LY.wave_hist);
  A.hwr = (double *)(wb + LY.wave_hist + LY.wave_w);
  const int NS = P.nslots;
  const int hwords = MODE == XI ? NS * 64 : NS * P.npi;
  for (int t = lane; t < hwords; t += 64) {
    A.hist[t] = 0u;
    if (W) {
      A.hw[t] = 0.0;
      A.hwr[t] = 0.0;
    }
  }
  __syncthreads();

  unsigned long long st_cand = 0, st_cells = 0, st_pruned = 0;
  uint32_t nrechk = 0;
  const int64_t ntiles = *P.ntiles;
  int cur_mock = -1;
  unsigned long long since_flush = 0;
  const unsigned long long flush_limit = MODE == XI ? (1ull << 30) : (1ull << 24);

  for (;;) {
    int64_t tix = 0;
    if (lane == 0) tix = (int64_t)atomicAdd(P.qhead, 1ull);
    tix = uni64(__shfl(tix, 0));
    if (tix >= ntiles) break;
    const Tile T = P.tiles[tix];
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
    L.x = valid ? pp.x : 1e200;
    L.y = valid ? pp.y : 1e200;
    L.z = valid ? pp.z : 1e200;
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
    const int total = (2 * rx + 1) * ncy * nzr;
    const double box = G2.box, half = G2.halfbox;
    const int wrapax[3] = {G2.wrap[0], G2.wrap[1], G2.wrap[2]};
    const bool anywrap = wrapax[0] | wrapax[1] | wrapax[2];
    const int64_t pbase2 = G2.pbase;

    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      int keep = 0, pruned = 0, cell = 0, packed = 0;
      if (t < total) {
        const int oz = t % nzr;
        const int rest = t / nzr;
        const int oy = rest % ncy;
        const int ox = rest / ncy;
        int X = cx + ox - rx, Y = cy + oy - ry, Z = tz0 - rz + oz;
        int sx = 0, sy = 0, sz = 0;
        bool ok = true;
        if (X < 0) { if (G2.periodic) { X += G2.n[0]; sx = -1; } else ok = false; }
        else if (X >= G2.n[0]) { if (G2.periodic) { X -= G2.n[0]; sx = 1; } else ok = false; }
        if (Y < 0) { if (G2.periodic) { Y += ny; sy = -1; } else ok = false; }
        else if (Y >= ny) { if (G2.periodic) { Y -= ny; sy = 1; } else ok = false; }
        if (Z < 0) { if (G2.periodic) { Z += nz; sz = -1; } else ok = false; }
        else if (Z >= nz) { if (G2.periodic) { Z -= nz; sz = 1; } else ok = false; }
        int own = 0;
        if (ok) {
          cell = (X * ny + Y) * nz + Z;
          const int colp = X * ny + Y;
          if (P.autocorr) {
            if (colp < tcol) ok = false;
            else if (colp == tcol) {
              if (Z < tz0) ok = false;
              else if (Z <= tz1) own = 1;
            }
          }
        }
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
            double m[3];
            for (int a = 0; a < 3; a++) {
              double gl = B.lo[a] - th[a];
              double gh = B.hi[a] - tl[a];
              if (Sv[a] != 0.0) {
                gl = gl + Sv[a];
                gh = gh + Sv[a];
              }
              m[a] = gl > 0.0 ? gl : (gh < 0.0 ? -gh : 0.0);
              if (wrapax[a]) m[a] = 0.0;
            }
            const double rp = m[0] * m[0] + m[1] * m[1];
            bool far;
            if (MODE == XI) far = (rp + m[2] * m[2]) >= P.EB;
            else far = (rp >= P.EB) || (m[2] >= P.pimax);
            if (far) {
              ok = false;
              pruned = 1;
            }
          }
        }
        if (ok) {
          // shift code per axis (-1, 0, +1 -> 0, 1, 2) in bits 1..6 of keep
          keep = 1 | ((sx + 1) << 1) | ((sy + 1) << 3) | ((sz + 1) << 5);
          packed = X | (Y << 10) | (Z << 20) | (own << 30);
        }
      }
      unsigned long long mk = __ballot(keep != 0);
      st_pruned += __popcll(__ballot(pruned != 0));
      while (mk) {
        const int src = __builtin_ctzll(mk);
        mk &= mk - 1;
        const int c2 = __builtin_amdgcn_readlane(cell, src);
        const int pk = __builtin_amdgcn_readlane(packed, src);
        const int kc = __builtin_amdgcn_readlane(keep, src);
        const int X = pk & 1023, Y = (pk >> 10) & 1023, Z = (pk >> 20) & 1023;
        const bool own = (pk >> 30) & 1;
        const int sxx = ((kc >> 1) & 3) - 1, syy = ((kc >> 3) & 3) - 1, szz = ((kc >> 5) & 3) - 1;
        const double S[3] = {sxx * box, syy * box, szz * box};
        const bool shifted = (sxx | syy | szz) != 0;
        sint *CS = (sint *)P.cstart2;
        const int64_t jb = pbase2 + CS[G2.sbase + c2];
        const int64_t je = pbase2 + CS[G2.sbase + c2 + 1];
        st_cells++;
        st_cand += (unsigned long long)nvalid * (unsigned long long)(je - jb);
        since_flush += (unsigned long long)(je - jb);
        if (since_flush > flush_limit) {
          flush_hist<MODE, W>(P, A, cur_mock, lane);
          since_flush = (unsigned long long)(je - jb);
        }
        if (PREC == F32R && !anywrap) {
          const double ox = frame_origin(G2, 0, X) + S[0];
          const double oy = frame_origin(G2, 1, Y) + S[1];
          const double oz = frame_origin(G2, 2, Z) + S[2];
          const float rxf = valid ? (float)(L.x - ox) : 1e18f;
          const float ryf = valid ? (float)(L.y - oy) : 1e18f;
          const float rzf = valid ? (float)(L.z - oz) : 1e18f;
          if (MODE == XI) {
            const float ra = __builtin_fmaf(rzf, rzf, __builtin_fmaf(ryf, ryf, rxf * rxf));
#define CP_XI(O, SH)                                                                      \
  loop_xi_f32<O, SH, W>(P, A, L, lane, rxf, ryf, rzf, ra, jb, je, pbase2, S, tab32, tab64, sE,  \
                        nrechk)
            if (own) { if (shifted) CP_XI(true, true); else CP_XI(true, false); }
            else { if (shifted) CP_XI(false, true); else CP_XI(false, false); }
#undef CP_XI
          } else {
            const float ra = __builtin_fmaf(ryf, ryf, rxf * rxf);
#define CP_WP(O, SH)                                                                      \
  loop_wp_f32<O, SH, W>(P, A, L, lane, rxf, ryf, rzf, ra, jb, je, pbase2, S, tab32, tab64, sE,  \
                        nrechk)
            if (own) { if (shifted) CP_WP(true, true); else CP_WP(true, false); }
            else { if (shifted) CP_WP(false, true); else CP_WP(false, false); }
#undef CP_WP
          }
        } else {
          if (anywrap) {
            if (own)
              loop_f64<MODE, true, true, true, W>(P, A, L, lane, jb, je, pbase2, S, wrapax, box,
                                                 half, tab64, sE);
            else
              loop_f64<MODE, false, true, true, W>(P, A, L, lane, jb, je, pbase2, S, wrapax, box,
                                                  half, tab64, sE);
          } else if (shifted) {
            if (own)
              loop_f64<MODE, true, true, false, W>(P, A, L, lane, jb, je, pbase2, S, wrapax, box,
                                                  half, tab64, sE);
            else
              loop_f64<MODE, false, true, false, W>(P, A, L, lane, jb, je, pbase2, S, wrapax,
                                                   box, half, tab64, sE);
          } else {
            if (own)
              loop_f64<MODE, true, false, false, W>(P, A, L, lane, jb, je, pbase2, S, wrapax,
                                                   box, half, tab64, sE);
            else
              loop_f64<MODE, false, false, false, W>(P, A, L, lane, jb, je, pbase2, S, wrapax,
                                                    box, half, tab64, sE);
          }
        }
      }
    }
  }
  if (cur_mock >= 0) flush_hist<MODE, W>(P, A, cur_mock, lane);
  const unsigned long long rc = wave_sum_u64((unsigned long long)nrechk);
  if (lane == 0) {
    if (st_cand) atomicAdd(P.stats + 0, st_cand);
    if (rc) atomicAdd(P.stats + 1, rc);
    if (st_cells) atomicAdd(P.stats + 2, st_cells);
    if (st_pruned) atomicAdd(P.stats + 3, st_pruned);
  }
}

template __global__ void k_pairs<XI, F32R, 0>(PairParams);
template __global__ void k_pairs<XI, F32R, 1>(PairParams);
template __global__ void k_pairs<XI, F64, 0>(PairParams);
template __global__ void k_pairs<XI, F64, 1>(PairParams);
template __global__ void k_pairs<WP, F32R, 0>(PairParams);
template __global__ void k_pairs<WP, F32R, 1>(PairParams);
template __global__ void k_pairs<WP, F64, 0>(PairParams);
template __global__ void k_pairs<WP, F64, 1>(PairParams);

} // namespace cp
