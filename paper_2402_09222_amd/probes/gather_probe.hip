// Achievable rate of random gathers on one GPU, the reference for kernels
// whose time is set by scattered reads (the lookup of small, unsorted
// batches reads one record pair per (lookup, nuclide) at a random place).
//
// Each lane reads `bytes` contiguous bytes (16-byte vector loads) at a
// random multiple of `align` bytes inside a buffer, sums them and writes one
// float; the launch covers n lanes.  Printed per shape: microseconds per
// launch (best of `reps`) and the rate in reads per second.  Usage:
//   gather_probe [reps] [buffer MiB] [reads]
// Output: one JSON line.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

namespace {

__device__ __forceinline__ uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;  // SplitMix64 (Steele, Lea, Flood 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int ALIGN, int NV>
__global__ __launch_bounds__(256) void k_gather(const float4* __restrict__ buf,
                                                uint64_t slots, uint64_t n,
                                                uint64_t seed,
                                                float* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t s = mix(i ^ (seed << 40)) % slots;
  const float4* p = buf + s * (ALIGN / 16);
  float acc = 0.f;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const float4 x = p[v];
    acc += x.x + x.y + x.z + x.w;
  }
  out[i] = acc;
}

#define CHECK(call)                                                         \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));            \
      exit(1);                                                              \
    }                                                                       \
  } while (0)

template <int ALIGN, int NV>
double best_us(const float4* buf, size_t bytes, uint64_t n, float* out,
               int reps) {
  // slots chosen so that the last slot's read ends inside the buffer
  const uint64_t slots = (bytes - (size_t)NV * 16) / ALIGN + 1;
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  const unsigned grid = (unsigned)((n + 255) / 256);
  double best = 1e30;
  for (int r = 0; r <= reps; ++r) {
    CHECK(hipEventRecord(a, 0));
    hipLaunchKernelGGL((k_gather<ALIGN, NV>), dim3(grid), dim3(256), 0, 0,
                       buf, slots, n, (uint64_t)r + 1, out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    if (r > 0 && ms * 1e3 < best) best = ms * 1e3;  // first run warms up
  }
  CHECK(hipEventDestroy(a));
  CHECK(hipEventDestroy(b));
  return best;
}

}  // namespace

int main(int argc, char** argv) {
  const int reps = argc > 1 ? atoi(argv[1]) : 20;
  const size_t mib = argc > 2 ? (size_t)atoll(argv[2]) : 128;
  const uint64_t n = argc > 3 ? (uint64_t)atoll(argv[3]) : 6500000;
  if (reps < 1 || mib < 1 || n < 1) return 2;
  const size_t bytes = mib << 20;
  float4* buf = nullptr;
  float* out = nullptr;
  CHECK(hipMalloc(&buf, bytes));
  CHECK(hipMalloc(&out, n * sizeof(float)));
  CHECK(hipMemset(buf, 0, bytes));
  CHECK(hipDeviceSynchronize());
  struct Row {
    const char* name;
    int bytes, align;
    double us;
  } rows[] = {
      {"32B_at_32", 32, 32, best_us<32, 2>(buf, bytes, n, out, reps)},
      {"64B_at_32", 64, 32, best_us<32, 4>(buf, bytes, n, out, reps)},
      {"64B_at_64", 64, 64, best_us<64, 4>(buf, bytes, n, out, reps)},
      {"96B_at_16", 96, 16, best_us<16, 6>(buf, bytes, n, out, reps)},
      {"128B_at_128", 128, 128, best_us<128, 8>(buf, bytes, n, out, reps)},
  };
  printf("{\"probe\": \"random gather\", \"buffer_mib\": %zu, \"reads\": %llu, "
         "\"shapes\": {", mib, (unsigned long long)n);
  for (size_t i = 0; i < sizeof(rows) / sizeof(rows[0]); ++i)
    printf("%s\"%s\": {\"bytes\": %d, \"align\": %d, \"us\": %.2f, "
           "\"reads_per_s\": %.4g}", i ? ", " : "", rows[i].name, rows[i].bytes,
           rows[i].align, rows[i].us, n / (rows[i].us * 1e-6));
  printf("}}\n");
  CHECK(hipFree(buf));
  CHECK(hipFree(out));
  return 0;
}
