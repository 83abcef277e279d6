// Request descriptors of the request kernels and the mapping of a batch's
// 1024-lookup tiles to requests.  Plain host/device functions with no
// kernel state, so a CPU build can check them on arbitrary memory contents.
//
// A batch of requests (the paper's particles in flight refilled between
// kernel calls, section 5.1) is cut into tiles: request r owns tiles
// [tile_begin_r, tile_begin_r + ceil(n_r / 1024)), and the tiles of the
// batch are numbered consecutively over its requests.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace xs {

constexpr int kStreamTile = 1024;  // lookups per tile

struct alignas(16) ReqDev {
  const double* E;
  const int32_t* mat;
  void* out;
  int64_t n;
  int64_t tile_begin;  // first tile of the request in the batch
  int64_t begin;       // first position in the batch's concatenated order
  uint64_t tag;        // the batch's tag (request streams; 0 otherwise)
  int64_t reserved;
};
static_assert(sizeof(ReqDev) == 64, "ReqDev layout");

__host__ __device__ inline int64_t tiles_of(int64_t n) {
  return (n + kStreamTile - 1) / kStreamTile;
}

// Largest r in [0, count) with reqs[r].tile_begin <= g, or 0 when there is
// none.  Only descriptors 1 .. count - 1 are read, at most
// ceil(log2(count)) of them, whatever they hold: the result is always a
// valid index and the loop always ends.
__host__ __device__ inline int request_of(const ReqDev* reqs, int count,
                                          int64_t g) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (reqs[mid].tile_begin <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Whether descriptor R, found for tile g of a batch, may be used: it carries
// the batch's tag, its size lies in [1, max_n] (max_n: the largest request
// the host submitted) and g is one of its tiles.  A descriptor that was not
// written for this batch fails the tag test, so its pointers are never
// dereferenced.
__host__ __device__ inline bool descriptor_ok(const ReqDev& R, int64_t g,
                                              uint64_t tag, int64_t max_n) {
  if (R.tag != tag || R.n < 1 || R.n > max_n) return false;
  if (R.tile_begin < 0 || g < R.tile_begin) return false;
  return g - R.tile_begin < tiles_of(R.n);
}

}  // namespace xs
