// One-time builders of the search accelerators (run by xs_create_tables).
//
// Hash bins (paper section 5.1, "number of logarithmic hash grid bins"): the
// energy range [e_min, e_max] is cut into B bins of equal width in ln E, and
// H[b][k] is nuclide k's bracket at the lower edge of bin b (H[B][k] = n_k-2).
// A lookup in bin b then only scans [H[b][k], H[b+1][k]] of nuclide k.  One
// bin reduces to a bisection of the whole grid; very many bins make the
// search a direct access, at the cost of (B+1) K int32 of memory.
//
// Unionized grid: u = all grid energies of all nuclides, sorted, without
// duplicates; uidx[j][k] = nuclide k's bracket at u[j].  Because no grid point
// of any nuclide lies strictly between u[j] and u[j+1], the bracket of any E
// in [u[j], u[j+1]) equals uidx[j][k].  The by-material layout stores, for
// each material m, the block [U][L_m] of its list's brackets, so a lookup
// reads its material's L_m indices contiguously instead of a K-wide row.
#include "xs_lookup_impl.h"

namespace xs {

namespace {

__global__ __launch_bounds__(256) void k_hash_build(const DevTables t,
                                                    const int32_t* __restrict__ goff,
                                                    double dln,
                                                    int32_t* __restrict__ H) {
  const int64_t total = (int64_t)(t.B + 1) * t.K;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(id / t.K), k = (int)(id % t.K);
    const int base = goff[k], n = goff[k + 1] - base;
    int v;
    if (b == t.B) {
      v = n - 2;
    } else {
      const double edge = exp(t.ln_emin + (double)b * dln);
      v = min(bisect_le(t.E + base, n, edge), n - 2);
    }
    H[id] = v;
  }
}

constexpr int kUnionChunk = 32;

// One lane per (chunk of kUnionChunk union points, nuclide), nuclide
// fastest so that the writes of a row are contiguous.  The bracket is found
// by bisection at the chunk's first point and then walked forward, since it
// never decreases along the sorted union grid.
__global__ __launch_bounds__(256) void k_union_index(const DevTables t,
                                                     const int32_t* __restrict__ goff,
                                                     int32_t* __restrict__ uidx) {
  const int64_t nchunks = (t.U + kUnionChunk - 1) / kUnionChunk;
  const int64_t total = nchunks * t.K;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(id % t.K);
    const int64_t j0 = (id / t.K) * kUnionChunk;
    const int64_t j1 = j0 + kUnionChunk < t.U ? j0 + kUnionChunk : t.U;
    const int base = goff[k], n = goff[k + 1] - base;
    const double* g = t.E + base;
    int i = min(bisect_le(g, n, t.u[j0]), n - 2);
    for (int64_t j = j0; j < j1; ++j) {
      const double x = t.u[j];
      while (i < n - 2 && g[i + 1] <= x) ++i;
      uidx[j * t.K + k] = i;
    }
  }
}

// By material: one lane per (chunk of union points, list position jg),
// list position fastest, so a row [L_m] of a material's block is written
// contiguously.  mrec[jg] gives the nuclide's grid; the material is found by
// a bisection of the material offsets.
__global__ __launch_bounds__(256) void k_union_index_by_material(
    const DevTables t, int32_t Ltot, int32_t* __restrict__ uidx) {
  const int64_t nchunks = (t.U + kUnionChunk - 1) / kUnionChunk;
  const int64_t total = nchunks * Ltot;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int jg = (int)(id % Ltot);
    const int64_t j0 = (id / Ltot) * kUnionChunk;
    const int64_t j1 = j0 + kUnionChunk < t.U ? j0 + kUnionChunk : t.U;
    int lo = 0, hi = t.M - 1;  // material m with moff[m] <= jg < moff[m+1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (t.moff[mid] <= jg) lo = mid; else hi = mid - 1;
    }
    const int m = lo;
    const int64_t L = t.moff[m + 1] - t.moff[m];
    const int jj = jg - t.moff[m];
    int32_t* block = uidx + t.U * (int64_t)t.moff[m];
    const MatRec r = t.mrec[jg];
    const double* g = t.E + r.base;
    int i = min(bisect_le(g, r.n, t.u[j0]), r.n - 2);
    for (int64_t j = j0; j < j1; ++j) {
      const double x = t.u[j];
      while (i < r.n - 2 && g[i + 1] <= x) ++i;
      block[j * L + jj] = i;
    }
  }
}

}  // namespace

hipError_t launch_union_index_by_material(const DevTables& t, int32_t Ltot,
                                          int32_t* uidx, hipStream_t s) {
  hipLaunchKernelGGL(k_union_index_by_material, dim3(8192), dim3(256), 0, s, t,
                     Ltot, uidx);
  return hipGetLastError();
}

hipError_t launch_hash_build(const DevTables& t, const int32_t* goff_dev,
                             double dln, int32_t* H, hipStream_t s) {
  hipLaunchKernelGGL(k_hash_build, dim3(4096), dim3(256), 0, s, t, goff_dev,
                     dln, H);
  return hipGetLastError();
}

hipError_t launch_union_index(const DevTables& t, const int32_t* goff_dev,
                              int32_t* uidx, hipStream_t s) {
  hipLaunchKernelGGL(k_union_index, dim3(8192), dim3(256), 0, s, t, goff_dev,
                     uidx);
  return hipGetLastError();
}

}  // namespace xs
