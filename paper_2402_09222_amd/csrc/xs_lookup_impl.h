// Lookup kernels, templated on grid method, precision and lookups per lane.
// Included by one translation unit per grid method so they compile in
// parallel.
//
// Per lookup (paper section 5.1, hash-bin paragraph after Table 1): for each
// nuclide of the material, in list order, find the bracket of E in the
// nuclide's grid, interpolate the five channels linearly and add the
// density-weighted values.  The arithmetic of one (lookup, nuclide) step is
// fixed (same operations, same order, no fused multiply-add: the library is
// built with -ffp-contract=off), so every grid method, sort order and launch
// shape gives bit-identical sums within one precision.
#pragma once

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

__device__ __forceinline__ bool valid_query(double e, int m, int M) {
  return __builtin_isfinite(e) && e > 0.0 && (unsigned)m < (unsigned)M;
}

// Block index remapped so that each XCD (blocks are dealt round-robin to
// the 8 XCDs) runs one contiguous eighth of the blocks: neighbouring blocks,
// which after a sort touch neighbouring grid segments, then share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t x = bid & 7, s = bid >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + s;
}

// ---- bracket search per grid method --------------------------------------

template <int GRID>
struct Locator;

// Bisection of the nuclide's own grid.
template <>
struct Locator<XS_GRID_NUCLIDE> {
  static constexpr bool kVerify = false;
  __device__ __forceinline__ void init(const DevTables&, double) {}
  __device__ __forceinline__ int bracket(const DevTables& t, const MatRec& r,
                                         double e) const {
    return min(bisect_le(t.E + r.base, r.n, e), r.n - 2);
  }
};

// Logarithmic hash bins: bin b of E is computed once per lookup; H[b][k] and
// H[b+1][k] bound nuclide k's bracket, found by a short forward scan.  A
// verification against the bracketing energies (done by the caller) falls
// back to bisection when rounding of log() put E in a neighbouring bin.
template <>
struct Locator<XS_GRID_HASH> {
  static constexpr bool kVerify = true;
  int b;
  __device__ __forceinline__ void init(const DevTables& t, double e) {
    double x = (log(e) - t.ln_emin) * t.inv_dln;
    x = fmin(fmax(x, 0.0), (double)(t.B - 1));
    b = (int)x;
  }
  __device__ __forceinline__ int bracket(const DevTables& t, const MatRec& r,
                                         double e) const {
    const int32_t* h = t.H + (int64_t)b * t.K + r.k;
    const int lo = h[0], hi = h[t.K];
    const double* g = t.E + r.base;
    int p = lo;
    while (p < hi && g[p + 1] <= e) ++p;
    return p;
  }
};

// Unionized grid: one bisection of the union of all grids per lookup, then
// one index-table read per nuclide.
template <>
struct Locator<XS_GRID_UNIONIZED> {
  static constexpr bool kVerify = false;
  int j;
  __device__ __forceinline__ void init(const DevTables& t, double e) {
    j = bisect_le(t.u, (int)t.U, e);
  }
  __device__ __forceinline__ int bracket(const DevTables& t, const MatRec& r,
                                         double) const {
    return t.uidx[(int64_t)j * t.K + r.k];
  }
};

// ---- one (lookup, nuclide) step --------------------------------------------

template <class R>
__device__ __forceinline__ bool bracket_ok(int i, int n, double e,
                                           const R& lo, const R& hi) {
  return (i == 0 || lo.e <= e) && (i == n - 2 || e < hi.e);
}

// Clamped energy and fraction.  min(max(E, E_k[0]), E_k[n-1]) equals
// min(max(E, E_k[i]), E_k[i+1]) for the bracket i, so only the bracket's
// own energies are needed.
__device__ __forceinline__ double fraction(double e, double e0, double e1) {
  double eh = e < e0 ? e0 : e;
  eh = eh > e1 ? e1 : eh;
  return (eh - e0) / (e1 - e0);
}

template <int GRID>
__device__ __forceinline__ void step64(const DevTables& t,
                                       const Locator<GRID>& loc, int j,
                                       double e, double acc[XS_CHANNELS]) {
  const MatRec r = t.mrec[j];
  int i = loc.bracket(t, r, e);
  const Rec64* rp = t.rec64 + r.base + i;
  Rec64 lo = rp[0], hi = rp[1];
  if (Locator<GRID>::kVerify && !bracket_ok(i, r.n, e, lo, hi)) {
    i = min(bisect_le(t.E + r.base, r.n, e), r.n - 2);
    rp = t.rec64 + r.base + i;
    lo = rp[0];
    hi = rp[1];
  }
  const double f = fraction(e, lo.e, hi.e);
  const double g = 1.0 - f;
  const double rho = t.rho64[j];
#pragma unroll
  for (int c = 0; c < XS_CHANNELS; ++c) {
    const double a = g * lo.x[c];
    const double b = f * hi.x[c];
    const double sigma = a + b;
    const double term = rho * sigma;
    acc[c] = acc[c] + term;
  }
}

struct Kahan32 {
  float s[XS_CHANNELS];
  float c[XS_CHANNELS];
};

template <int GRID>
__device__ __forceinline__ void step32(const DevTables& t,
                                       const Locator<GRID>& loc, int j,
                                       double e, Kahan32& acc) {
  const MatRec r = t.mrec[j];
  int i = loc.bracket(t, r, e);
  const Rec32* rp = t.rec32 + r.base + i;
  Rec32 lo = rp[0], hi = rp[1];
  if (Locator<GRID>::kVerify && !bracket_ok(i, r.n, e, lo, hi)) {
    i = min(bisect_le(t.E + r.base, r.n, e), r.n - 2);
    rp = t.rec32 + r.base + i;
    lo = rp[0];
    hi = rp[1];
  }
  const double f = fraction(e, lo.e, hi.e);
  const float f32 = (float)f;
  const float g32 = (float)(1.0 - f);
  const float rho = r.rho32;
#pragma unroll
  for (int c = 0; c < XS_CHANNELS; ++c) {
    const float a = g32 * lo.x[c];
    const float b = f32 * hi.x[c];
    const float sigma = a + b;
    const float term = rho * sigma;
    const float y = term - acc.c[c];
    const float tt = acc.s[c] + y;
    acc.c[c] = (tt - acc.s[c]) - y;
    acc.s[c] = tt;
  }
}

// ---- accumulators and output per precision --------------------------------

template <int PREC>
struct Acc;

template <>
struct Acc<XS_FP64> {
  double v[XS_CHANNELS];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) v[c] = 0.0;
  }
  template <int GRID>
  __device__ __forceinline__ void step(const DevTables& t,
                                       const Locator<GRID>& loc, int j,
                                       double e) {
    step64<GRID>(t, loc, j, e, v);
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
  Kahan32 k;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) {
      k.s[c] = 0.0f;
      k.c[c] = 0.0f;
    }
  }
  template <int GRID>
  __device__ __forceinline__ void step(const DevTables& t,
                                       const Locator<GRID>& loc, int j,
                                       double e) {
    step32<GRID>(t, loc, j, e, k);
  }
  __device__ __forceinline__ void store(void* out, int64_t o) const {
    float* p = (float*)out + o * XS_CHANNELS;
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) p[c] = k.s[c];
  }
  __device__ __forceinline__ static void store_nan(void* out, int64_t o) {
    float* p = (float*)out + o * XS_CHANNELS;
#pragma unroll
    for (int c = 0; c < XS_CHANNELS; ++c) p[c] = __builtin_nanf("");
  }
};

// ---- the lookup kernel -------------------------------------------------------
//
// A block covers blockDim * LPT consecutive queue positions; lane l of the
// block takes positions base + l, base + l + blockDim, ... (coalesced).  When
// all of a lane's lookups share one material they walk its nuclide list
// together, giving LPT independent searches per step.

// Largest block for LPT lookups per lane: more lookups per lane need more
// registers, so fewer lanes fit per compute unit.
constexpr int max_block_for_lpt(int lpt) {
  return lpt <= 2 ? 1024 : (lpt <= 4 ? 512 : 256);
}

template <int GRID, int PREC, int LPT>
__global__ __launch_bounds__(max_block_for_lpt(LPT)) void k_lookup(
    const DevTables t, const LookupArgs a) {
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t n = a.count_dev ? *a.count_dev : a.n;
  const int64_t first = blk * (int64_t)blockDim.x * LPT + threadIdx.x;

  double e[LPT];
  int m[LPT];
  int64_t o[LPT];
  bool act[LPT];
#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    const int64_t q = first + (int64_t)l * blockDim.x;
    act[l] = q < n;
    o[l] = 0;
    e[l] = 0.0;
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

  bool fuse = LPT > 1;
#pragma unroll
  for (int l = 0; l < LPT; ++l) fuse = fuse && act[l] && m[l] == m[0];

  if (fuse) {
    Locator<GRID> loc[LPT];
    Acc<PREC> acc[LPT];
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      loc[l].init(t, e[l]);
      acc[l].zero();
    }
    const int j0 = t.moff[m[0]], j1 = t.moff[m[0] + 1];
    for (int j = j0; j < j1; ++j) {
#pragma unroll
      for (int l = 0; l < LPT; ++l) acc[l].template step<GRID>(t, loc[l], j, e[l]);
    }
#pragma unroll
    for (int l = 0; l < LPT; ++l) acc[l].store(a.out, o[l]);
    return;
  }

#pragma unroll
  for (int l = 0; l < LPT; ++l) {
    if (!act[l]) continue;
    Locator<GRID> loc;
    loc.init(t, e[l]);
    Acc<PREC> acc;
    acc.zero();
    const int j0 = t.moff[m[l]], j1 = t.moff[m[l] + 1];
    for (int j = j0; j < j1; ++j) acc.template step<GRID>(t, loc, j, e[l]);
    acc.store(a.out, o[l]);
  }
}

// ---- validation path: brackets of every (lookup, nuclide) ---------------------

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
  loc.init(t, e);
  for (int j = j0; j < j1; ++j) {
    const MatRec r = t.mrec[j];
    int i = loc.bracket(t, r, e);
    if (Locator<GRID>::kVerify) {
      const double* g = t.E + r.base;
      const bool ok = (i == 0 || g[i] <= e) && (i == r.n - 2 || e < g[i + 1]);
      if (!ok) i = min(bisect_le(g, r.n, e), r.n - 2);
    }
    out[j - j0] = i;
  }
}

// ---- launchers ------------------------------------------------------------------

template <int GRID, int PREC>
hipError_t launch_lpt(const DevTables& t, int lpt, dim3 grid, dim3 block,
                      const LookupArgs& a, hipStream_t s) {
  switch (lpt) {
#define XS_LPT_CASE(L)                                                      \
  case L:                                                                   \
    hipLaunchKernelGGL((k_lookup<GRID, PREC, L>), grid, block, 0, s, t, a); \
    break;
    XS_LPT_CASE(1)
    XS_LPT_CASE(2)
    XS_LPT_CASE(3)
    XS_LPT_CASE(4)
    XS_LPT_CASE(5)
    XS_LPT_CASE(6)
    XS_LPT_CASE(7)
    XS_LPT_CASE(8)
#undef XS_LPT_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int GRID>
hipError_t launch_grid_method(const DevTables& t, const xs_params& p,
                              const LookupArgs& a, hipStream_t s) {
  if (p.block_size > max_block_for_lpt(p.lookups_per_thread))
    return hipErrorInvalidValue;
  const int64_t per_block = (int64_t)p.block_size * p.lookups_per_thread;
  const int64_t nb = (a.n + per_block - 1) / per_block;
  if (nb == 0) return hipSuccess;
  if (nb > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nb), block((unsigned)p.block_size);
  if (p.precision == XS_FP64)
    return launch_lpt<GRID, XS_FP64>(t, p.lookups_per_thread, grid, block, a, s);
  return launch_lpt<GRID, XS_FP32>(t, p.lookups_per_thread, grid, block, a, s);
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
