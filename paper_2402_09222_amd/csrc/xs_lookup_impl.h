// Lookup kernels, templated on grid method, precision, lookups per lane
// (LPT) and nuclides in flight per lane (U).  Included by one translation
// unit per grid method so they compile in parallel.
//
// Per lookup (paper section 5.1, hash-bin paragraph after Table 1): for each
// nuclide of the material, in list order, find the bracket of E in the
// nuclide's grid, interpolate the five channels linearly and add the
// density-weighted values.  The arithmetic of one (lookup, nuclide) step is
// fixed (same operations, same order, no fused multiply-add: the library is
// built with -ffp-contract=off), so every grid method, sort order and launch
// shape gives bit-identical sums within one precision.
//
// The walk over a material's nuclides is latency-bound (dependent loads:
// index, then the bracketing records), so each lane keeps U nuclides in
// flight: it issues the index loads of U nuclides, then their record loads,
// then adds the U terms in list order.  When every lane of a wave holds the
// same material (the usual case after a sort) the material list is read with
// scalar loads.
#pragma once

#include <type_traits>

#include "xs_internal.h"

namespace xs {

// Largest p in [0, n-1] with g[p] <= e, or 0 when g[0] > e.  Branch-free
// bisection: ceil(log2 n) probes, a trip count that depends on n only.
__device__ __forceinline__ int bisect_le(const double* __restrict__ g, int n,
                                         double e) {
  int lo = 0, len = n;
  while (len > 1) {
    const int half = len >> 1;
    lo = (g[lo + half] <= e) ? lo + half : lo;
    len -= half;
  }
  return lo;
}

// bisect_le's result for a full wave searching one sorted array for one
// energy: each step the 64 lanes probe 64 points that split the remaining
// range into 65 parts, and the count of probes <= e (a prefix, the array
// being sorted) names the part that holds the answer.  The range shrinks 65
// times per step: 4 dependent loads for the 4M-point union grid instead of
// 22, for 64 cache lines per step instead of one.  It is the fallback of
// wave_union_row below, which reads one logarithmic bin's points instead.
// Every lane of the wave must call it with the same arguments.
__device__ __forceinline__ int wave_bisect_le(const double* __restrict__ g,
                                              int n, double e, int lane) {
  int lo = 0, len = n;  // answer in [lo, lo + len); g[lo] <= e unless lo == 0
  while (len > 64) {
    const int p = lo + (int)((int64_t)(lane + 1) * len / 65);
    const int c = __popcll(__ballot(g[p] <= e));
    const int hi = c == 64 ? lo + len : lo + (int)((int64_t)(c + 1) * len / 65);
    lo = c == 0 ? lo : lo + (int)((int64_t)c * len / 65);
    len = hi - lo;
  }
  const int c = __popcll(__ballot(lane < len && g[lo + lane] <= e));
  return c == 0 ? lo : lo + c - 1;
}

__device__ __forceinline__ bool valid_query(double e, int m, int M) {
  return __builtin_isfinite(e) && e > 0.0 && (unsigned)m < (unsigned)M;
}

// Reads through the constant address space: with a wave-uniform address the
// compiler emits a scalar load; with a per-lane address a vector load.  Only
// used for tables that no kernel writes.
template <class T>
__device__ __forceinline__ T ld_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized types only");
  typedef const __attribute__((address_space(4))) uint32_t* WordPtr;
  const WordPtr q = (WordPtr)p;
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) w[i] = q[i];
  T v;
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}

// Block index remapped so that each XCD (blocks are dealt round-robin to
// the 8 XCDs) runs one contiguous eighth of the blocks: neighbouring blocks,
// which after a sort touch neighbouring grid segments, then share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t x = bid & 7, s = bid >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + s;
}

// This block's index among the blocks that hold queue positions, remapped as
// above, or -1 when it holds none.  With a device-side queue length (a
// compacted queue, or the active head of a sorted one) the grid is sized
// for the whole batch: only the first ceil(count / per_block) blocks have
// work, and remapping over those (not the grid) spreads them over all XCDs.
__device__ __forceinline__ int64_t queue_block(const LookupArgs& a,
                                               int64_t per_block) {
  int64_t nb = gridDim.x;
  if (a.count_dev) {
    const int64_t c = (*a.count_dev + per_block - 1) / per_block;
    nb = c < nb ? c : nb;
  }
  if ((int64_t)blockIdx.x >= nb) return -1;
  return xcd_remap(blockIdx.x, nb);
}

// Largest block for LPT lookups per lane with U nuclides in flight: more
// independent chains per lane need more registers, so fewer lanes fit per
// compute unit.
constexpr int max_block_for(int lpt, int unroll) {
  return lpt * unroll <= 1 ? 1024 : (lpt * unroll <= 4 ? 512 : 256);
}

// ---- records per precision ---------------------------------------------------

template <int PREC>
struct RecOf;
template <>
struct RecOf<XS_FP64> {
  using T = Rec64;
  __device__ static const Rec64* base(const DevTables& t) { return t.rec64; }
};
template <>
struct RecOf<XS_FP32> {
  using T = Rec32;
  __device__ static const Rec32* base(const DevTables& t) { return t.rec32; }
};

// Bracket test against the pair's energies (with the clamp cases).
template <class R>
__device__ __forceinline__ bool bracket_ok(int i, int n, double e, const R& lo,
                                           const R& hi) {
  return (i == 0 || lo.e <= e) && (i == n - 2 || e < hi.e);
}

// ---- hash-bin search ------------------------------------------------------------
//
// H[b][k] is nuclide k's bracket at the lower edge of bin b, so for E in bin b
// the bracket lies in [H[b][k], H[b+1][k]].  The fast path assumes it is
// H[b][k] or H[b][k] + 1 (true whenever a bin holds at most one grid point of
// the nuclide): it reads the three records from H[b][k] on and keeps the pair
// that brackets E.  Otherwise the slow path scans the bin's window and, if
// rounding of log() put E in a neighbouring bin, bisects the whole grid.
// Either way the result is the unique bracket.

__device__ __forceinline__ int hash_slow(const DevTables& t, const MatRec& r,
                                         const int32_t* hrow1, int lo,
                                         double e) {
  const double* g = t.E + r.base;
  const int hi = hrow1[r.k];
  int p = lo;
  while (p < hi && g[p + 1] <= e) ++p;
  const bool ok = (p == 0 || g[p] <= e) && (p == r.n - 2 || e < g[p + 1]);
  if (t.dbg) {
    atomicAdd(t.dbg + kDbgHashScans, 1ull);
    if (!ok) atomicAdd(t.dbg + kDbgHashFull, 1ull);
  }
  return ok ? p : min(bisect_le(g, r.n, e), r.n - 2);
}

// ---- per-lookup search state ---------------------------------------------------

template <int GRID>
struct Locator;

template <>
struct Locator<XS_GRID_NUCLIDE> {
  __device__ __forceinline__ void init(const DevTables&, double, int) {}
  __device__ __forceinline__ int start(const DevTables& t, const MatRec& r,
                                       int, double e) const {
    return min(bisect_le(t.E + r.base, r.n, e), r.n - 2);
  }
  __device__ __forceinline__ const int32_t* next_row(const DevTables&) const {
    return nullptr;
  }
};

template <>
struct Locator<XS_GRID_HASH> {
  const int32_t* hrow;  // H[b]
  __device__ __forceinline__ void init(const DevTables& t, double e, int) {
    double x = (log(e) - t.ln_emin) * t.inv_dln;
    x = fmin(fmax(x, 0.0), (double)(t.B - 1));
    hrow = t.H + (int64_t)(int)x * t.K;
  }
  __device__ __forceinline__ int start(const DevTables&, const MatRec& r, int,
                                       double) const {
    return hrow[r.k];
  }
  __device__ __forceinline__ const int32_t* next_row(const DevTables& t) const {
    return hrow + t.K;  // H[b+1]
  }
};

// The union bracket of E (bisect_le over the union grid): the logarithmic
// bin of E bounds it between two bin edges' brackets, about 32 points apart,
// and the bracket found there is verified; the rounding of log can only put E
// in a neighbouring bin, where the verify fails and the whole grid is
// bisected.  Three or four dependent loads instead of 22 for 4M points.
__device__ __forceinline__ int union_row(const DevTables& t, double e) {
  double x = (log(e) - t.u_ln_min) * t.u_inv_dln;
  x = fmin(fmax(x, 0.0), (double)(t.UB - 1));
  const int b = (int)x;
  const int lo = t.uh[b], hi = t.uh[b + 1];
  const int j = lo + bisect_le(t.u + lo, hi - lo + 1, e);
  const int U = (int)t.U;
  const bool ok = (j == 0 || t.u[j] <= e) && (j == U - 1 || e < t.u[j + 1]);
  return ok ? j : bisect_le(t.u, U, e);
}

// union_row for a whole wave searching one energy (every lane passes the
// same e): the bin's edge brackets take one scalar load; then lane i reads
// union point lo + i for the bin's points and the one after them (one round
// of contiguous loads), and the count of points <= e, a prefix since the
// grid is sorted, is the bracket.  That count is exact when it ends inside
// the points read (or at the grid's ends); otherwise (the rounding of log
// put E in a neighbouring bin, or a bin holds 64 points or more) the wave
// searches the whole grid.  Two dependent loads instead of union_row's
// eight (bin edges, six bisection probes over ~32 points, the verify).
__device__ __forceinline__ int wave_union_row(const DevTables& t, double e,
                                              int lane) {
  double x = (log(e) - t.u_ln_min) * t.u_inv_dln;
  x = fmin(fmax(x, 0.0), (double)(t.UB - 1));
  const int b = (int)x;
  const int lo = ld_const(t.uh + b), hi = ld_const(t.uh + b + 1);
  const int U = (int)t.U;
  const int np = min(hi + 2, U) - lo;  // points lo .. min(hi + 1, U - 1)
  if (np <= 64) {
    const int p = lo + lane;
    const int c = __popcll(__ballot(lane < np && t.u[p] <= e));
    if (c >= 1 && (c < np || lo + np == U)) return lo + c - 1;
    if (c == 0 && lo == 0) return 0;
  }
  return wave_bisect_le(t.u, U, e, lane);
}

// Row j of the index table: [U][K] (column = nuclide id) or, when built by
// material, material m's block [U][L_m] (column = position in m's list).
template <>
struct Locator<XS_GRID_UNIONIZED> {
  const int32_t* urow;
  int jbase;  // first list position of the material (by-material layout)
  __device__ __forceinline__ void init(const DevTables& t, double e, int m) {
    init_row(t, union_row(t, e), m);
  }
  // State for union point j (the bracket of E in the union grid).
  __device__ __forceinline__ void init_row(const DevTables& t, int64_t j,
                                           int m) {
    if (t.union_by_material) {
      jbase = t.moff[m];
      const int64_t L = t.moff[m + 1] - jbase;
      urow = t.uidx + t.U * jbase + j * L;
    } else {
      jbase = 0;
      urow = t.uidx + j * t.K;
    }
  }
  __device__ __forceinline__ int start(const DevTables& t, const MatRec& r,
                                       int jg, double) const {
    return urow[t.union_by_material ? jg - jbase : r.k];
  }
  __device__ __forceinline__ const int32_t* next_row(const DevTables&) const {
    return nullptr;
  }
};

// Keeps a record's fields in registers at this point: the compiler may not
// move the loads that produced them past it (used to keep LDS reads and
// global reads of the same record type in their own branches instead of
// merging them into one load through a generic pointer).
// The FP32 record's reciprocal is pinned only where it is used (the lower
// record of a bracket).
template <class R>
__device__ __forceinline__ void pin_rec(R& r, bool with_rcp) {
#pragma unroll
  for (int k = 0; k < XS_CHANNELS; ++k) asm volatile("" : "+v"(r.x[k]));
  asm volatile("" : "+v"(r.e));
  if constexpr (sizeof(R) == sizeof(Rec32))
    if (with_rcp) asm volatile("" : "+v"(r.rcp));
}

// Field-wise out = c ? a : b.  Selecting whole records by reference would
// make the compiler select an address and keep the records on the stack.
template <class R>
__device__ __forceinline__ void select_rec(bool c, const R& a, const R& b,
                                           R& out) {
#pragma unroll
  for (int k = 0; k < XS_CHANNELS; ++k) out.x[k] = c ? a.x[k] : b.x[k];
  out.e = c ? a.e : b.e;
  if constexpr (sizeof(R) == sizeof(Rec32)) out.rcp = c ? a.rcp : b.rcp;
}

// Records around a candidate index: three for the hash grid (candidate and
// the next two), two (the bracket) otherwise.
template <int GRID, int PREC>
struct Window {
  using R = typename RecOf<PREC>::T;
  static constexpr bool kHash = GRID == XS_GRID_HASH;
  R r0, r1, r2;
  __device__ __forceinline__ void load(const DevTables& t, const MatRec& m,
                                       int i) {
    const R* p = RecOf<PREC>::base(t) + m.base;
    r0 = p[i];
    r1 = p[i + 1];
    if (kHash) r2 = p[min(i + 2, m.n - 1)];
  }
  // Final bracket pair into lo/hi.
  __device__ __forceinline__ void finish(const DevTables& t, const MatRec& m,
                                         const Locator<GRID>& loc, int cand,
                                         double e, R& lo, R& hi) const {
    if (!kHash) {
      lo = r0;
      hi = r1;
      return;
    }
    const bool up = cand + 1 <= m.n - 2 && r1.e <= e;
    const int i = up ? cand + 1 : cand;
    select_rec(up, r1, r0, lo);
    select_rec(up, r2, r1, hi);
    if (!bracket_ok(i, m.n, e, lo, hi)) {
      const int j = hash_slow(t, m, loc.next_row(t), cand, e);
      const R* p = RecOf<PREC>::base(t) + m.base;
      lo = p[j];
      hi = p[j + 1];
    }
  }
};

// max / min of two FP64 values that are never NaN (validated energies and
// table energies), one instruction each.  The compiler's fmax/fmin would
// first quiet each operand, which no value here needs.
__device__ __forceinline__ double max_nonnan(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double min_nonnan(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Correctly rounded n / d for the operands a lookup can produce from tables
// whose energies lie in [2^-400, 2^400] (checked at table creation): d is a
// positive difference of two such energies, so d is in [2^-452, 2^401], and
// n is 0 or in [2^-452, d].  This is the division the compiler emits (a
// reciprocal refined by two Newton steps, the quotient and one residual
// correction) without its range scaling and special-case fix-up, which never
// act on such operands (no exponent near the limits, no zero, infinity, NaN
// or subnormal divisor): the result is the same correctly rounded quotient.
__device__ __forceinline__ double div_in_range(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double q = n * r;
  const double rem = __builtin_fma(-d, q, n);
  return __builtin_fma(rem, r, q);
}

// The same correctly rounded quotient when a 24-bit approximation of 1 / d
// is at hand (the FP32 records carry RN32(1 / d) for their interval): two
// Newton steps take it from 2^-24 to well below the last bit of the double
// reciprocal, as from the hardware reciprocal, and the quotient and its
// residual correction follow unchanged.  Saves the reciprocal instruction.
__device__ __forceinline__ double div_seeded(double n, double d, float seed) {
  double r = (double)seed;
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double q = n * r;
  const double rem = __builtin_fma(-d, q, n);
  return __builtin_fma(rem, r, q);
}

// Clamped energy and fraction.  min(max(E, E_k[0]), E_k[n-1]) equals
// min(max(E, E_k[i]), E_k[i+1]) for the bracket i, so only the bracket's
// own energies are needed.
__device__ __forceinline__ double fraction(double e, double e0, double e1) {
  const double eh = min_nonnan(max_nonnan(e, e0), e1);
  return div_in_range(eh - e0, e1 - e0);
}
__device__ __forceinline__ double fraction(double e, double e0, double e1,
                                           float rcp) {
  const double eh = min_nonnan(max_nonnan(e, e0), e1);
  return div_seeded(eh - e0, e1 - e0, rcp);
}

// ---- accumulators and output per precision --------------------------------

template <int PREC>
struct Acc;

template <>
struct Acc<XS_FP64> {
  using Term = double;
  double v[XS_CHANNELS];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) v[c] = 0.0;
  }
  // One nuclide's terms: sigma = g*lo + f*hi (two products, one add), then
  // rho * sigma.
  __device__ __forceinline__ static void terms(const Rec64& lo, const Rec64& hi,
                                               double e, double rho,
                                               double (&t)[XS_CHANNELS]) {
    const double f = fraction(e, lo.e, hi.e);
    const double g = 1.0 - f;
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) {
      const double a = g * lo.x[c];
      const double b = f * hi.x[c];
      const double sigma = a + b;
      t[c] = rho * sigma;
    }
  }
  // sum += term, one channel.
  __device__ __forceinline__ static void step(double& v, double term) {
    v = v + term;
  }
  __device__ __forceinline__ void add(const Rec64& lo, const Rec64& hi,
                                      double e, double rho) {
    double t[XS_CHANNELS];
    terms(lo, hi, e, rho, t);
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) step(v[c], t[c]);
  }
  __device__ __forceinline__ static double rho(const DevTables& t,
                                               const MatRec&, int j) {
    return ld_const(t.rho64 + j);
  }
  __device__ __forceinline__ void store(void* out, int64_t o) const {
    double* p = (double*)out + o * XS_CHANNELS;
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) p[c] = v[c];
  }
  __device__ __forceinline__ static void store_nan(void* out, int64_t o) {
    double* p = (double*)out + o * XS_CHANNELS;
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) p[c] = __builtin_nan("");
  }
};

template <>
struct Acc<XS_FP32> {
  using Term = float;
  float s[XS_CHANNELS];
  float c[XS_CHANNELS];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < XS_CHANNELS; ++k) {
      s[k] = 0.0f;
      c[k] = 0.0f;
    }
  }
  // f and g = 1 - f are formed in FP64 and each rounded to FP32; channels
  // interpolate in FP32; the term is rho * sigma in FP32.
  __device__ __forceinline__ static void terms(const Rec32& lo, const Rec32& hi,
                                               double e, float rho,
                                               float (&t)[XS_CHANNELS]) {
    const double f = fraction(e, lo.e, hi.e, lo.rcp);
    const float f32 = (float)f;
    const float g32 = (float)(1.0 - f);
#pragma unroll
    for (int k = 0; k < XS_CHANNELS; ++k) {
      const float a = g32 * lo.x[k];
      const float b = f32 * hi.x[k];
      const float sigma = a + b;
      t[k] = rho * sigma;
    }
  }
  // The sum over nuclides is compensated (Kahan), one channel:
  // y = term - c; t = s + y; c = (t - s) - y; s = t.
  __device__ __forceinline__ static void step(float& s, float& c, float term) {
    const float y = term - c;
    const float tt = s + y;
    c = (tt - s) - y;
    s = tt;
  }
  __device__ __forceinline__ void add(const Rec32& lo, const Rec32& hi,
                                      double e, float rho) {
    float t[XS_CHANNELS];
    terms(lo, hi, e, rho, t);
#pragma unroll
    for (int k = 0; k < XS_CHANNELS; ++k) step(s[k], c[k], t[k]);
  }
  __device__ __forceinline__ static float rho(const DevTables&, const MatRec& r,
                                              int) {
    return r.rho32;
  }
  __device__ __forceinline__ void store(void* out, int64_t o) const {
    float* p = (float*)out + o * XS_CHANNELS;
#pragma unroll
    for (int k = 0; k < XS_CHANNELS; ++k) p[k] = s[k];
  }
  __device__ __forceinline__ static void store_nan(void* out, int64_t o) {
    float* p = (float*)out + o * XS_CHANNELS;
#pragma unroll
    for (int k = 0; k < XS_CHANNELS; ++k) p[k] = __builtin_nanf("");
  }
};

// One channel's running sum, for kernels that give each channel its own
// lane: the same step as Acc<PREC>.
template <int PREC>
struct Chan;
template <>
struct Chan<XS_FP64> {
  double v = 0.0;
  __device__ __forceinline__ void add(double t) { Acc<XS_FP64>::step(v, t); }
  __device__ __forceinline__ void store(void* out, int64_t i) const {
    ((double*)out)[i] = v;
  }
};
template <>
struct Chan<XS_FP32> {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float t) { Acc<XS_FP32>::step(s, c, t); }
  __device__ __forceinline__ void store(void* out, int64_t i) const {
    ((float*)out)[i] = s;
  }
};

// ---- walk of one material's nuclide list for LPT lookups ---------------------------
//
// `mat` is either wave-uniform (scalar loads of the list) or per lane.  U
// nuclides are processed per iteration in three phases (index loads, record
// loads, in-order accumulation), so a lane has U x LPT independent load
// chains in flight.

// Candidate indices of U nuclides for LPT lookups.  Bisection runs the
// LPT x U searches in lock step so their probes overlap; the other methods
// issue one index load each.
template <int GRID, int LPT, int U>
__device__ __forceinline__ void candidates(const DevTables& t,
                                           const MatRec (&r)[U], int j,
                                           const double (&e)[LPT],
                                           const Locator<GRID> (&loc)[LPT],
                                           int (&cand)[LPT][U]) {
  if (GRID == XS_GRID_NUCLIDE) {
    int lo[LPT][U], len[LPT][U];
#pragma unroll
    for (int l = 0; l < LPT; ++l)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        lo[l][u] = 0;
        len[l][u] = r[u].n;
      }
    bool more = true;
    while (more) {
      more = false;
#pragma unroll
      for (int l = 0; l < LPT; ++l)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (len[l][u] > 1) {
            const int half = len[l][u] >> 1;
            const double* g = t.E + r[u].base;
            lo[l][u] = (g[lo[l][u] + half] <= e[l]) ? lo[l][u] + half : lo[l][u];
            len[l][u] -= half;
            more = more || len[l][u] > 1;
          }
        }
    }
#pragma unroll
    for (int l = 0; l < LPT; ++l)
#pragma unroll
      for (int u = 0; u < U; ++u) cand[l][u] = min(lo[l][u], r[u].n - 2);
    return;
  }
#pragma unroll
  for (int l = 0; l < LPT; ++l)
#pragma unroll
    for (int u = 0; u < U; ++u) cand[l][u] = loc[l].start(t, r[u], j + u, e[l]);
}

template <int GRID, int PREC, int LPT, int U>
__device__ __forceinline__ void walk_material(const DevTables& t, int mat,
                                              const double (&e)[LPT],
                                              const Locator<GRID> (&loc)[LPT],
                                              Acc<PREC> (&acc)[LPT]) {
  using W = Window<GRID, PREC>;
  using R = typename W::R;
  const int j0 = ld_const(t.moff + mat), j1 = ld_const(t.moff + mat + 1);
  int j = j0;
  if (U > 1) {
    for (; j + U <= j1; j += U) {
      MatRec r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) r[u] = ld_const(t.mrec + j + u);
      int cand[LPT][U];
      candidates<GRID, LPT, U>(t, r, j, e, loc, cand);
      W w[LPT][U];
#pragma unroll
      for (int l = 0; l < LPT; ++l)
#pragma unroll
        for (int u = 0; u < U; ++u) w[l][u].load(t, r[u], cand[l][u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const auto rho = Acc<PREC>::rho(t, r[u], j + u);
#pragma unroll
        for (int l = 0; l < LPT; ++l) {
          R lo, hi;
          w[l][u].finish(t, r[u], loc[l], cand[l][u], e[l], lo, hi);
          acc[l].add(lo, hi, e[l], rho);
        }
      }
    }
  }
  for (; j < j1; ++j) {
    const MatRec r[1] = {ld_const(t.mrec + j)};
    int cand[LPT][1];
    candidates<GRID, LPT, 1>(t, r, j, e, loc, cand);
    W w[LPT];
#pragma unroll
    for (int l = 0; l < LPT; ++l) w[l].load(t, r[0], cand[l][0]);
    const auto rho = Acc<PREC>::rho(t, r[0], j);
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      R lo, hi;
      w[l].finish(t, r[0], loc[l], cand[l][0], e[l], lo, hi);
      acc[l].add(lo, hi, e[l], rho);
    }
  }
}

// ---- the lookup kernel -------------------------------------------------------
//
// A block covers blockDim * LPT consecutive queue positions; lane l of the
// block takes positions base + l, base + l + blockDim, ... (coalesced).

template <int GRID, int PREC, int LPT, int U>
__global__ __launch_bounds__(max_block_for(LPT, U)) void k_lookup(
    const DevTables t, const LookupArgs a) {
  const int64_t per_block = (int64_t)blockDim.x * LPT;
  const int64_t blk = queue_block(a, per_block);
  if (blk < 0) return;
  const int64_t n = a.count_dev ? *a.count_dev : a.n;
  const int64_t first = blk * per_block + threadIdx.x;

  double e[LPT];
  int m[LPT];
  int64_t o[LPT];
  bool act[LPT];
#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    const int64_t q = first + (int64_t)l * blockDim.x;
    act[l] = q < n;
    o[l] = 0;
    e[l] = 1.0;
    m[l] = -1;
    if (act[l]) {
      o[l] = a.perm ? (int64_t)a.perm[q] : q;
      // a permutation entry outside [0, n) cannot occur; never dereference one
      if ((uint64_t)o[l] >= (uint64_t)a.n) act[l] = false;
      else if (a.active && !a.active[o[l]]) act[l] = false;
    }
    if (act[l]) {
      e[l] = a.E[o[l]];
      m[l] = a.mat[o[l]];
      if (!valid_query(e[l], m[l], t.M)) {
        Acc<PREC>::store_nan(a.out, o[l]);
        act[l] = false;
      }
    }
  }

  // All of this lane's lookups active and in one material?
  bool same = true;
#pragma unroll
  for (int l = 0; l < LPT; ++l) same = same && act[l] && m[l] == m[0];
  // ... and the whole wave in that material?
  const int mu = __builtin_amdgcn_readfirstlane(m[0]);
  const bool wave_uniform = __all(same && m[0] == mu);

  if (wave_uniform || same) {
    Locator<GRID> loc[LPT];
    Acc<PREC> acc[LPT];
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      loc[l].init(t, e[l], m[0]);
      acc[l].zero();
    }
    if (wave_uniform)
      walk_material<GRID, PREC, LPT, U>(t, mu, e, loc, acc);
    else
      walk_material<GRID, PREC, LPT, U>(t, m[0], e, loc, acc);
#pragma unroll
    for (int l = 0; l < LPT; ++l) acc[l].store(a.out, o[l]);
    return;
  }

#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    if (!act[l]) continue;
    const double e1[1] = {e[l]};
    Locator<GRID> loc[1];
    Acc<PREC> acc[1];
    loc[0].init(t, e[l], m[l]);
    acc[0].zero();
    walk_material<GRID, PREC, 1, U>(t, m[l], e1, loc, acc);
    acc[0].store(a.out, o[l]);
  }
}

// ---- exact bracket from the search grid -----------------------------------------
//
// The same candidate and window logic as the lookup, reading energies from the
// search grid instead of the records (validation path, LDS staging).

struct GridRec {
  double e;
};

template <int GRID>
__device__ __forceinline__ int exact_bracket(const DevTables& t,
                                             const Locator<GRID>& loc,
                                             const MatRec& r, int j,
                                             double e) {
  const int cand = loc.start(t, r, j, e);
  if (GRID != XS_GRID_HASH) return cand;
  const double* g = t.E + r.base;
  const GridRec g0{g[cand]}, g1{g[cand + 1]}, g2{g[min(cand + 2, r.n - 1)]};
  const bool up = cand + 1 <= r.n - 2 && g1.e <= e;
  const int i = up ? cand + 1 : cand;
  const GridRec lo{up ? g1.e : g0.e}, hi{up ? g2.e : g1.e};
  if (bracket_ok(i, r.n, e, lo, hi)) return i;
  return hash_slow(t, r, loc.next_row(t), cand, e);
}

template <int GRID>
__global__ __launch_bounds__(256) void k_indices(const DevTables t, int64_t n,
                                                 const double* __restrict__ E,
                                                 const int32_t* __restrict__ mat,
                                                 const int64_t* __restrict__ off,
                                                 int32_t* __restrict__ idx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double e = E[q];
  const int m = mat[q];
  if ((unsigned)m >= (unsigned)t.M) return;
  const int j0 = t.moff[m], j1 = t.moff[m + 1];
  int32_t* out = idx + off[q];
  if (!valid_query(e, m, t.M)) {
    for (int j = j0; j < j1; ++j) out[j - j0] = -1;
    return;
  }
  Locator<GRID> loc;
  loc.init(t, e, m);
  for (int j = j0; j < j1; ++j) out[j - j0] = exact_bracket(t, loc, t.mrec[j], j, e);
}

// ---- LDS-staged lookup -------------------------------------------------------------
//
// For a block whose lookups all share one material (the usual case after a
// sort), each nuclide's bracket lies between the brackets of the block's
// lowest and highest energies.  The material's nuclides are taken in groups
// of lds_group: lane i of the block finds the window of nuclide i of the
// group (from the lower edge's bracket to the upper edge's bracket + 1), the
// block copies every window of at most lds_window records into LDS with one
// cooperative read, and each lane then walks the group's nuclides in list
// order, bisecting its window in LDS and interpolating from it.  A nuclide
// whose window is wider takes the per-lane search for that nuclide; a block
// holding several materials (or a partial last block) takes the per-lane
// walk.  Same arithmetic, same order: the sums are bit-identical to
// k_lookup's.  Three barriers per group of nuclides instead of a search and
// a window load per (lookup, nuclide).  Each lane handles LPT (1 or 2)
// lookups; the block's energy range covers all of them and their in-LDS
// searches run in lock step.

// Stage shapes (lds_stage = 1, 2, 3): 32 nuclides per round with windows of
// at most 8 records, 16 with 16, or 8 with 32 — the same LDS either way.
// Dense batches (about 10M lookups) keep the windows narrow and favour many
// nuclides per round; sparser ones (1e6 to 2e6) need wider windows, or most
// nuclides fall back to the per-lane search (measured: 0.39 ms against 0.81
// for the lookup of 1e6 banded lookups).  FP64 windows hold three quarters
// as many of its 48-byte records, which would otherwise limit the blocks per
// compute unit by LDS (10M banded lookups: 1.82 ms against 2.0).
template <int SHAPE>
constexpr int lds_group() {
  return SHAPE == 1 ? 32 : (SHAPE == 2 ? 16 : 8);
}
template <int PREC, int SHAPE>
constexpr int lds_window() {
  return (PREC == XS_FP64 ? 3 : 4) * (256 / lds_group<SHAPE>()) / 4;
}
//
// Over a sorted queue cut at every group of the sort key (a.blocks), a
// block's range holds one material, and the lanes past the range's end (the
// group's last, partial piece) idle through the staged walk.  A block with
// lookups of several materials (an uncut queue straddling two groups), or
// whose first lookup is invalid, takes the per-lane walk.
template <int GRID, int PREC, int LPT, int SHAPE>
__global__ __launch_bounds__(1024 / LPT) void k_lookup_lds(const DevTables t,
                                                           const LookupArgs a) {
  using R = typename RecOf<PREC>::T;
  constexpr int kLdsGroup = lds_group<SHAPE>();
  constexpr int kLdsW = lds_window<PREC, SHAPE>();
  __shared__ R stage[kLdsGroup * kLdsW];
  __shared__ int s_first[kLdsGroup];  // first staged record
  // records in the staged window (0: too wide, each lane searches itself)
  __shared__ __align__(8) int s_win[kLdsGroup];
  __shared__ int s_mat;
  __shared__ int64_t s_row[2];
  __shared__ double s_red[2][16];
  const int tid = threadIdx.x;
  int64_t blk, first, end;  // this block's queue positions: first .. end - 1
  if (a.blocks) {
    // The grid is sized for the most ranges a queue can have; the ranges
    // actually cut are dealt evenly over the XCDs and the rest leave.
    const int64_t nr = *a.n_blocks;
    if ((int64_t)blockIdx.x >= nr) return;  // the whole block leaves
    blk = xcd_remap(blockIdx.x, nr);
    first = a.blocks[2 * blk];
    end = a.blocks[2 * blk + 1];
  } else {
    blk = queue_block(a, (int64_t)blockDim.x * LPT);
    if (blk < 0) return;  // the whole block leaves
    first = blk * (int64_t)blockDim.x * LPT;
    end = a.count_dev ? *a.count_dev : a.n;
  }

  // Lane tid takes queue positions first + tid, + blockDim, ... (coalesced).
  bool act[LPT];
  int64_t o[LPT];
  double e[LPT];
  int m[LPT];
#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    const int64_t q = first + tid + (int64_t)l * blockDim.x;
    act[l] = q < end;
    o[l] = 0;
    e[l] = 1.0;
    m[l] = -1;
    if (act[l]) {
      o[l] = a.perm ? (int64_t)a.perm[q] : q;
      if ((uint64_t)o[l] >= (uint64_t)a.n) act[l] = false;
      else if (a.active && !a.active[o[l]]) act[l] = false;
    }
    if (act[l]) {
      e[l] = a.E[o[l]];
      m[l] = a.mat[o[l]];
      if (!valid_query(e[l], m[l], t.M)) {
        Acc<PREC>::store_nan(a.out, o[l]);
        act[l] = false;
      }
    }
  }
  // One material: every active lane's is the first lane's (lanes past the
  // range's end and invalid queries do not count).
  if (tid == 0) s_mat = act[0] ? m[0] : -1;
  __syncthreads();
  const int mb = s_mat;
  bool mine = mb >= 0, full = true;
#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    mine = mine && (!act[l] || m[l] == mb);
    full = full && act[l];
  }
  const bool uniform = __syncthreads_and(mine);

  if (!uniform) {
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      if (!act[l]) continue;
      const double e1[1] = {e[l]};
      Locator<GRID> l1[1];
      Acc<PREC> a1[1];
      l1[0].init(t, e[l], m[l]);
      a1[0].zero();
      walk_material<GRID, PREC, 1, 1>(t, m[l], e1, l1, a1);
      a1[0].store(a.out, o[l]);
    }
    return;
  }
  const bool whole = __syncthreads_and(full);

  // The staged walk; with idle lanes (masked), they compute nothing they
  // keep and stay out of the block's energy range.
  auto staged = [&](auto masked) {
  constexpr bool kMasked = decltype(masked)::value;
  // Block energy range (over the active lookups).
  double lo_e, hi_e;
  if constexpr (kMasked) {
    lo_e = __builtin_inf();
    hi_e = -__builtin_inf();
#pragma unroll
    for (int l = 0; l < LPT; ++l)
      if (act[l]) {
        lo_e = fmin(lo_e, e[l]);
        hi_e = fmax(hi_e, e[l]);
      }
  } else {
    lo_e = e[0];
    hi_e = e[0];
#pragma unroll
    for (int l = 1; l < LPT; ++l) {
      lo_e = fmin(lo_e, e[l]);
      hi_e = fmax(hi_e, e[l]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo_e = fmin(lo_e, __shfl_xor(lo_e, off, 64));
    hi_e = fmax(hi_e, __shfl_xor(hi_e, off, 64));
  }
  const int w = tid >> 6, lane = tid & 63, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) {
    s_red[0][w] = lo_e;
    s_red[1][w] = hi_e;
  }
  __syncthreads();
  lo_e = s_red[0][0];
  hi_e = s_red[1][0];
  for (int i = 1; i < nw; ++i) {
    lo_e = fmin(lo_e, s_red[0][i]);
    hi_e = fmax(hi_e, s_red[1][i]);
  }

  // Search state of the two edge energies: the union grid is searched once
  // per edge by a whole wave (the edge's logarithmic bin read in one round,
  // two dependent loads; measured against a 64-way search of the whole grid,
  // four: 2-3 % faster from 1e6 to 1e7 lookups); the hash bin is
  // arithmetic; bisection keeps no state.
  Locator<GRID> edge_lo, edge_hi;
  if constexpr (GRID == XS_GRID_UNIONIZED) {
    // waves 0 and 1 (or wave 0 twice in a one-wave block)
    for (int k = w; k < 2; k += nw) {
      const int row = wave_union_row(t, k == 0 ? lo_e : hi_e, lane);
      if (lane == 0) s_row[k] = row;
    }
    __syncthreads();
    edge_lo.init_row(t, s_row[0], mb);
    edge_hi.init_row(t, s_row[1], mb);
  } else {
    edge_lo.init(t, lo_e, mb);
    edge_hi.init(t, hi_e, mb);
  }

  Locator<GRID> loc[LPT];  // this lane's own search states, made on first need
  bool have_loc = false;
  Acc<PREC> acc[LPT];
#pragma unroll
  for (int l = 0; l < LPT; ++l) acc[l].zero();
  const R* recs = RecOf<PREC>::base(t);
  const int j0 = ld_const(t.moff + mb), j1 = ld_const(t.moff + mb + 1);
  for (int jg = j0; jg < j1; jg += kLdsGroup) {
    const int cnt = min(kLdsGroup, j1 - jg);
    if (tid < cnt) {
      const MatRec r = t.mrec[jg + tid];
      const int lo = exact_bracket(t, edge_lo, r, jg + tid, lo_e);
      const int hi = exact_bracket(t, edge_hi, r, jg + tid, hi_e);
      const int width = hi - lo + 2;  // grid points lo .. hi + 1
      s_first[tid] = r.base + lo;
      s_win[tid] = width <= kLdsW ? width : 0;
    }
    __syncthreads();
    for (int s = tid; s < cnt * kLdsW; s += blockDim.x) {
      const int i = s / kLdsW, k = s % kLdsW;
      if (k < s_win[i]) stage[s] = recs[s_first[i] + k];
    }
    __syncthreads();
    // One nuclide of the group: its records (from LDS, or the lane's own
    // search when the window was too wide), then the arithmetic.
    // `width` is the block-uniform s_win[i], held in a scalar register so
    // the branch and the probe count cost no vector instructions.
    auto step = [&](int i, int width) {
      const int j = jg + i;
      const MatRec r = ld_const(t.mrec + j);
      const auto rho = Acc<PREC>::rho(t, r, j);
      R lo[LPT], hi[LPT];
      if (width > 0) {
        // the record p in [0, width-2] with the largest win[p].e <= e,
        // else 0; the LPT searches run in lock step.  Positions are byte
        // offsets from the stage (one add per probe, no scaling), and the
        // reads stay LDS reads because every address is the stage plus an
        // offset.
        const char* sb = reinterpret_cast<const char*>(stage);
        int qb[LPT];
#pragma unroll
        for (int l = 0; l < LPT; ++l) qb[l] = i * kLdsW * (int)sizeof(R);
        int len = width - 1;
        while (len > 1) {
          const int half = len >> 1;
          const int hb = half * (int)sizeof(R);
#pragma unroll
          for (int l = 0; l < LPT; ++l) {
            // the probe's offset is kept as is (opaque to the compiler), so
            // the step is one add, the read, a compare and a select between
            // two registers
            int cand = qb[l] + hb;
            asm volatile("" : "+v"(cand));
            const double pe = reinterpret_cast<const R*>(sb + cand)->e;
            qb[l] = pe <= e[l] ? cand : qb[l];
          }
          len -= half;
        }
#pragma unroll
        for (int l = 0; l < LPT; ++l) {
          lo[l] = *reinterpret_cast<const R*>(sb + qb[l]);
          hi[l] = *reinterpret_cast<const R*>(sb + qb[l] + sizeof(R));
          pin_rec(lo[l], true);
          pin_rec(hi[l], false);
        }
      } else {
        if (!have_loc) {
#pragma unroll
          for (int l = 0; l < LPT; ++l) loc[l].init(t, e[l], mb);
          have_loc = true;
        }
#pragma unroll
        for (int l = 0; l < LPT; ++l) {
          const int cand = loc[l].start(t, r, j, e[l]);
          Window<GRID, PREC> win;
          win.load(t, r, cand);
          win.finish(t, r, loc[l], cand, e[l], lo[l], hi[l]);
        }
      }
      // one copy of the arithmetic for both paths
#pragma unroll
      for (int l = 0; l < LPT; ++l) acc[l].add(lo[l], hi[l], e[l], rho);
    };
    // FP32: two nuclides per trip (in list order), so the Kahan accumulators
    // alternate between two register sets instead of being copied back every
    // nuclide.  FP64 keeps one per trip (measured: the second set of wide
    // records costs more occupancy than the copies).
    int i = 0;
    if constexpr (PREC == XS_FP32) {
      for (; i + 1 < cnt; i += 2) {
        const int2 w2 = *reinterpret_cast<const int2*>(&s_win[i]);
        step(i, __builtin_amdgcn_readfirstlane(w2.x));
        step(i + 1, __builtin_amdgcn_readfirstlane(w2.y));
      }
    }
    for (; i < cnt; ++i) step(i, __builtin_amdgcn_readfirstlane(s_win[i]));
    __syncthreads();  // the stage and window tables are rewritten next group
  }
#pragma unroll
  for (int l = 0; l < LPT; ++l)
    if (!kMasked || act[l]) acc[l].store(a.out, o[l]);
  };
  if (whole)
    staged(std::false_type{});
  else
    staged(std::true_type{});
}

// ---- one wave per lookup ------------------------------------------------------------
//
// For small batches one lane per lookup leaves most of the chip idle, and
// each lane walks its material's nuclides one after another, each behind a
// chain of dependent loads (search, then records).  Here the 64 lanes of a
// wave share one lookup: lane l takes nuclides l, l + 64, ... of the
// material, finds its bracket, interpolates and forms its density-weighted
// terms, which go through LDS to five lanes (one per channel) that add them
// in list order.  Same terms, same order: the sums are bit-identical to
// k_lookup's.  No block barrier is used, so a wave whose lookup is inactive
// or invalid simply leaves.

constexpr int kWaveBlock = 256;  // largest block: four waves

// PAIRS (FP32, union or bisection grid, XS_BUILD_FP32_PAIRS built): a
// bracket's two records come from one aligned 64-byte block of the pair
// table instead of two neighbouring records (same values, same results).
template <int GRID, int PREC, bool PAIRS>
__global__ __launch_bounds__(kWaveBlock) void k_lookup_wave(const DevTables t,
                                                            const LookupArgs a) {
  static_assert(!PAIRS || (PREC == XS_FP32 && GRID != XS_GRID_HASH),
                "pairs serve FP32 brackets found exactly");
  using R = typename RecOf<PREC>::T;
  using T = typename Acc<PREC>::Term;
  __shared__ T terms[kWaveBlock / 64][64][XS_CHANNELS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n = a.count_dev ? *a.count_dev : a.n;
  const int64_t blk = queue_block(a, blockDim.x >> 6);
  if (blk < 0) return;
  const int64_t q = blk * (blockDim.x >> 6) + w;
  if (q >= n) return;
  const int64_t o = a.perm ? (int64_t)a.perm[q] : q;
  if ((uint64_t)o >= (uint64_t)a.n) return;
  if (a.active && !a.active[o]) return;
  const double e = a.E[o];
  const int m = a.mat[o];
  if (!valid_query(e, m, t.M)) {
    if (lane == 0) Acc<PREC>::store_nan(a.out, o);
    return;
  }
  // Every lane searches the union grid for the same energy: the logarithmic
  // bin, then one contiguous read of the bin's points (wave_union_row).  (A
  // 64-way search of the whole grid, wave_bisect_le, was slower here: with
  // every wave searching, its 64 lines per step cost more than its shorter
  // chain saved.)
  Locator<GRID> loc;
  if constexpr (GRID == XS_GRID_UNIONIZED)
    loc.init_row(t, wave_union_row(t, e, lane), m);
  else
    loc.init(t, e, m);
  Chan<PREC> sum;  // lanes 0..4: channel `lane`
  const int j0 = t.moff[m], j1 = t.moff[m + 1];
  for (int jc = j0; jc < j1; jc += 64) {
    const int j = jc + lane;
    if (j < j1) {
      const MatRec r = t.mrec[j];
      const int cand = loc.start(t, r, j, e);
      R lo, hi;
      if constexpr (PAIRS) {
        const R* pp = t.pair32 + 2 * ((int64_t)r.base + cand);
        lo = pp[0];
        hi = pp[1];
      } else {
        Window<GRID, PREC> win;
        win.load(t, r, cand);
        win.finish(t, r, loc, cand, e, lo, hi);
      }
      T tm[XS_CHANNELS];
      Acc<PREC>::terms(lo, hi, e, Acc<PREC>::rho(t, r, j), tm);
#pragma unroll
      for (int c = 0; c < XS_CHANNELS; ++c) terms[w][lane][c] = tm[c];
    }
    // the wave's LDS writes are visible to its own reads after this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < XS_CHANNELS) {
      const int cnt = min(64, j1 - jc);
      for (int i = 0; i < cnt; ++i) sum.add(terms[w][i][lane]);
    }
    // the terms are rewritten by the next chunk
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (lane < XS_CHANNELS) sum.store(a.out, o * XS_CHANNELS + lane);
}

// ---- launchers ------------------------------------------------------------------

// (LPT, U) pairs instantiated: every LPT with one nuclide in flight, and 2 or
// 4 nuclides in flight for one or two lookups per lane.
constexpr bool variant_exists(int lpt, int unroll) {
  return (unroll == 1 && lpt >= 1 && lpt <= 8) ||
         ((unroll == 2 || unroll == 4) && (lpt == 1 || lpt == 2));
}

template <int GRID, int PREC>
hipError_t launch_variant(const DevTables& t, int lpt, int unroll, dim3 grid,
                          dim3 block, const LookupArgs& a, hipStream_t s) {
#define XS_CASE(L, U)                                                          \
  if (lpt == L && unroll == U) {                                               \
    hipLaunchKernelGGL((k_lookup<GRID, PREC, L, U>), grid, block, 0, s, t, a); \
    return hipGetLastError();                                                  \
  }
  XS_CASE(1, 1)
  XS_CASE(2, 1)
  XS_CASE(3, 1)
  XS_CASE(4, 1)
  XS_CASE(5, 1)
  XS_CASE(6, 1)
  XS_CASE(7, 1)
  XS_CASE(8, 1)
  XS_CASE(1, 2)
  XS_CASE(2, 2)
  XS_CASE(1, 4)
  XS_CASE(2, 4)
#undef XS_CASE
  return hipErrorInvalidValue;
}

template <int GRID>
hipError_t launch_grid_method(const DevTables& t, const xs_params& p,
                              const LookupArgs& a, hipStream_t s) {
  if (p.wave_per_lookup) {
    if (p.lookups_per_thread != 1 || p.unroll != 1 || p.lds_stage ||
        p.block_size > kWaveBlock)
      return hipErrorInvalidValue;
    const int64_t per_block = p.block_size / 64;
    const int64_t nb = (a.n + per_block - 1) / per_block;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (p.precision == XS_FP64) {
      hipLaunchKernelGGL((k_lookup_wave<GRID, XS_FP64, false>),
                         dim3((unsigned)nb), dim3(p.block_size), 0, s, t, a);
    } else if constexpr (GRID != XS_GRID_HASH) {
      if (t.pair32)
        hipLaunchKernelGGL((k_lookup_wave<GRID, XS_FP32, true>),
                           dim3((unsigned)nb), dim3(p.block_size), 0, s, t, a);
      else
        hipLaunchKernelGGL((k_lookup_wave<GRID, XS_FP32, false>),
                           dim3((unsigned)nb), dim3(p.block_size), 0, s, t, a);
    } else {
      hipLaunchKernelGGL((k_lookup_wave<GRID, XS_FP32, false>),
                         dim3((unsigned)nb), dim3(p.block_size), 0, s, t, a);
    }
    return hipGetLastError();
  }
  if (p.lds_stage) {
    const int lpt = p.lookups_per_thread;
    if ((lpt != 1 && lpt != 2) || p.unroll != 1 ||
        p.block_size > 1024 / lpt)
      return hipErrorInvalidValue;
    if (p.lds_stage < 1 || p.lds_stage > 3) return hipErrorInvalidValue;
    const int64_t per_block = (int64_t)p.block_size * lpt;
    const int64_t nb =
        a.blocks ? a.max_blocks : (a.n + per_block - 1) / per_block;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb), block((unsigned)p.block_size);
#define XS_LDS(P, L, S) hipLaunchKernelGGL((k_lookup_lds<GRID, P, L, S>), grid, block, 0, s, t, a)
#define XS_LDS_SHAPES(P, L)        \
  switch (p.lds_stage) {           \
    case 1: XS_LDS(P, L, 1); break; \
    case 2: XS_LDS(P, L, 2); break; \
    default: XS_LDS(P, L, 3); break; \
  }
    if (p.precision == XS_FP64) {
      if (lpt == 1) { XS_LDS_SHAPES(XS_FP64, 1) } else { XS_LDS_SHAPES(XS_FP64, 2) }
    } else {
      if (lpt == 1) { XS_LDS_SHAPES(XS_FP32, 1) } else { XS_LDS_SHAPES(XS_FP32, 2) }
    }
#undef XS_LDS_SHAPES
#undef XS_LDS
    return hipGetLastError();
  }
  if (!variant_exists(p.lookups_per_thread, p.unroll) ||
      p.block_size > max_block_for(p.lookups_per_thread, p.unroll))
    return hipErrorInvalidValue;
  const int64_t per_block = (int64_t)p.block_size * p.lookups_per_thread;
  const int64_t nb = (a.n + per_block - 1) / per_block;
  if (nb == 0) return hipSuccess;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nb), block((unsigned)p.block_size);
  if (p.precision == XS_FP64)
    return launch_variant<GRID, XS_FP64>(t, p.lookups_per_thread, p.unroll,
                                         grid, block, a, s);
  return launch_variant<GRID, XS_FP32>(t, p.lookups_per_thread, p.unroll, grid,
                                       block, a, s);
}

template <int GRID>
hipError_t launch_indices_grid(const DevTables& t, int64_t n, const double* E,
                               const int32_t* mat, const int64_t* off,
                               int32_t* idx, hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL((k_indices<GRID>), dim3((unsigned)nb), dim3(256), 0, s, t,
                     n, E, mat, off, idx);
  return hipGetLastError();
}

}  // namespace xs
