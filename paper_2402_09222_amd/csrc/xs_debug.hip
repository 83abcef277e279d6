// Debug-mode query check (xs_set_debug): counts the invalid queries of one
// lookup call and the lowest position among them.  A query is invalid when
// its energy is not finite and positive or its material is out of range, the
// same test the lookup kernels apply before writing a NaN row.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xs_lookup_impl.h"

namespace xs {
namespace {

constexpr int kDbgThreads = 256;

__global__ __launch_bounds__(1) void k_debug_call_reset(unsigned long long* c) {
  c[kDbgCallInvalid] = 0;
  c[kDbgCallFirst] = ~0ull;
}

__global__ __launch_bounds__(kDbgThreads) void k_debug_count(
    int64_t n, const double* __restrict__ E, const int32_t* __restrict__ mat,
    const uint8_t* __restrict__ active, int M, unsigned long long* c) {
  const int64_t stride = (int64_t)gridDim.x * kDbgThreads;
  for (int64_t i = (int64_t)blockIdx.x * kDbgThreads + threadIdx.x; i < n;
       i += stride) {
    if (active && !active[i]) continue;
    if (!valid_query(E[i], mat[i], M)) {
      atomicAdd(c + kDbgCallInvalid, 1ull);
      atomicAdd(c + kDbgInvalid, 1ull);
      atomicMin(c + kDbgCallFirst, (unsigned long long)i);
    }
  }
}

}  // namespace

hipError_t launch_debug_count(int64_t n, const double* E, const int32_t* mat,
                              const uint8_t* active, int M,
                              unsigned long long* counters, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_call_reset, dim3(1), dim3(1), 0, s, counters);
  if (hipError_t e = hipGetLastError()) return e;
  if (n <= 0) return hipSuccess;
  const int64_t blocks =
      std::min<int64_t>((n + kDbgThreads - 1) / kDbgThreads, 8192);
  hipLaunchKernelGGL(k_debug_count, dim3((unsigned)blocks), dim3(kDbgThreads),
                     0, s, n, E, mat, active, M, counters);
  return hipGetLastError();
}

}  // namespace xs
