// Queue formation: stable LSD radix sort of lookups by (material, energy)
// and stable compaction of active slots.
//
// The paper (section 5.1, "minimum sorting threshold") sorts particles so
// that neighbours in the buffer sit in the same material and near in energy,
// improving the locality of the cross-section lookup; the order never changes
// a lookup's value.  Here the key is a 32-bit word: an optional inactive
// flag, the material, and the top bits of the energy's IEEE pattern above
// the table's lowest energy (monotone in E for positive doubles).  Each
// 8-bit digit pass is reduce-then-scan: per-tile digit histograms, a scan
// of each digit's counts over the tiles, then a scatter that adds the
// digits' starts and whose ranks inside a 64-lane wave come from per-wave
// LDS counters.
#include "xs_internal.h"

namespace xs {

namespace {

// Radix passes take 8192 keys per block (16 per lane): with 256 digits a
// tile then holds ~32 keys of a digit, so the scatter writes runs of ~128
// bytes (one cache line) instead of ~64, with the same waves per compute
// unit as 4096-key tiles (two blocks of 75 KB of LDS instead of four).
constexpr int kRadixThreads = 512;
constexpr int kRadixTile = kRadixThreads * kSortItems;

struct SortSrc {
  const double* E;
  const int32_t* mat;
  const uint8_t* active;
  SortKey key;
  int64_t n;
};

__device__ __forceinline__ uint32_t make_key(const SortKey& k, double e,
                                             int32_t m, bool inactive) {
  uint32_t key = 0;
  if (k.e_bits) {
    int64_t d = __double_as_longlong(e) - k.e_bits_min;
    d = d < 0 ? 0 : (d >> k.e_shift);
    const int64_t maxv = (1ll << k.e_bits) - 1;
    key = (uint32_t)(d > maxv ? maxv : d);
  }
  if (k.mat_bits) {
    const int32_t mm = m < 0 ? 0 : (m >= k.M ? k.M - 1 : m);
    const int rest = k.e_bits - k.band_bits;  // energy bits below the material
    const uint32_t band = key >> rest, low = key & ((1u << rest) - 1u);
    key = (band << (k.mat_bits + rest)) | ((uint32_t)mm << rest) | low;
  }
  if (k.flag_bit && inactive) key |= 1u << (k.mat_bits + k.e_bits);
  return key;
}

__device__ __forceinline__ uint32_t src_key(const SortSrc& s, int64_t i) {
  return make_key(s.key, s.E[i], s.mat[i], s.active && !s.active[i]);
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive scan over a 64-lane wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Inclusive scan over a block of NT threads; *total gets the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t x,
                                                    uint32_t* total) {
  __shared__ uint32_t wsum[NT / 64];
  const uint32_t incl = wave_incl_scan(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const uint32_t s = wsum[i];
    off += i < w ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return incl + off;
}

// Per-tile digit histogram, digit-major: hist[d * nT + tile].  A block's
// keys are all read before any is counted, so its loads are in flight
// together.  The first pass makes the keys from the queries and writes them
// (keys_out) for its scatter, which then reads 4 bytes per lookup instead of
// the 12 of the energy and material.
template <bool FROM_INPUT>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(
    SortSrc src, const uint32_t* __restrict__ keys_in, int shift,
    uint32_t* __restrict__ hist, int32_t nT, uint32_t* __restrict__ keys_out) {
  static_assert(kRadixThreads >= kRadixBins, "a lane per digit");
  __shared__ uint32_t h[kRadixBins];
  const int tid = threadIdx.x;
  if (tid < kRadixBins) h[tid] = 0;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  uint32_t key[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * kRadixThreads + tid;
    key[r] = i < src.n ? (FROM_INPUT ? src_key(src, i) : keys_in[i]) : 0u;
    if (FROM_INPUT && i < src.n) keys_out[i] = key[r];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * kRadixThreads + tid;
    if (i < src.n) atomicAdd(&h[(key[r] >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  if (tid < kRadixBins) hist[(int64_t)tid * nT + blockIdx.x] = h[tid];
}

// Row d becomes its exclusive scan over the tiles (the position of the
// tile's first key of digit d among the digit's keys); totals[d] gets the
// row's sum.  The digits' starts (the exclusive scan of totals) are added
// by the scatter.
// NT lanes per row: 256 for short rows, 1024 (fewer rounds) for long ones.
template <int NT>
__global__ __launch_bounds__(NT) void k_row_scan(
    uint32_t* __restrict__ hist, int32_t nT, uint32_t* __restrict__ totals) {
  const int d = blockIdx.x;
  uint32_t* row = hist + (int64_t)d * nT;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nT; c0 += NT) {
    const int i = c0 + threadIdx.x;
    const uint32_t x = i < nT ? row[i] : 0u;
    uint32_t tot;
    const uint32_t incl = block_incl_scan<NT>(x, &tot);
    if (i < nT) row[i] = carry + incl - x;
    carry += tot;
  }
  if (threadIdx.x == 0) totals[d] = carry;
}

// Stable scatter of one digit pass.  Wave w of the block owns the tile's
// elements [w*1024, (w+1)*1024), read 64 at a time in order, so the order
// (wave, round, lane) is input order.  wcnt[w][d] counts digit d so far in
// wave w; an element's rank among its wave's elements of digit d is the old
// value of that counter, which it increments.  On gfx950 the adds of one
// LDS instruction return in lane order (checked over 16.7M adds with
// random, few and all-equal digits), so the pass is stable; were they not,
// elements of one digit would swap only within a wave's 64, which moves
// lookups a few places in the queue and never changes a result.  The tile
// is then reordered in LDS by digit and written out in that order:
// consecutive lanes write consecutive positions of one digit's run instead
// of 64 scattered words per wave.
template <bool FROM_INPUT, bool WRITE_KEYS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(
    SortSrc src, const uint32_t* __restrict__ keys_in,
    const uint32_t* __restrict__ vals_in, int shift,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ totals,
    int32_t nT, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kPerWave = kRadixTile / kWaves;
  static_assert(kPerWave == kSortItems * 64, "a wave's elements, 64 a round");
  static_assert(kRadixThreads >= kRadixBins, "a lane per digit");
  __shared__ uint32_t wcnt[kWaves][kRadixBins];
  __shared__ int32_t gdelta[kRadixBins];  // output position - tile position
  __shared__ uint32_t skey[kRadixTile];
  __shared__ uint32_t sval[kRadixTile];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const bool owner = tid < kRadixBins;  // lane tid owns digit tid
  for (int i = tid; i < kWaves * kRadixBins; i += kRadixThreads)
    (&wcnt[0][0])[i] = 0;
  const uint32_t tile_off = owner ? offs[(int64_t)tid * nT + blockIdx.x] : 0u;
  __syncthreads();

  const int64_t tile0 = (int64_t)blockIdx.x * kRadixTile;
  const int64_t base = tile0 + w * kPerWave;
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool ok = i < src.n;
    uint32_t k = 0, v = 0;
    if (ok) {
      k = keys_in[i];
      v = FROM_INPUT ? (uint32_t)i : vals_in[i];
    }
    const uint32_t d = (k >> shift) & (kRadixBins - 1);
    rank[r] = ok ? atomicAdd(&wcnt[w][d], 1u) : 0u;
    key[r] = k;
    val[r] = v;
  }
  __syncthreads();
  {
    // Lane tid < 256 owns digit tid: its waves' counts become their first
    // tile positions, and the digit's tile start maps to its output start.
    // The other lanes add zeros to the block's scans.
    uint32_t c[kWaves], tot = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
      c[ww] = owner ? wcnt[ww][tid] : 0u;
      tot += c[ww];
    }
    uint32_t all;
    const uint32_t start = block_incl_scan<kRadixThreads>(tot, &all) - tot;
    if (owner) {
      uint32_t s = start;
#pragma unroll
      for (int ww = 0; ww < kWaves; ++ww) {
        wcnt[ww][tid] = s;
        s += c[ww];
      }
    }
    // the digit's first output position: the keys of all smaller digits
    const uint32_t td = owner ? totals[tid] : 0u;
    const uint32_t dstart = block_incl_scan<kRadixThreads>(td, &all) - td;
    if (owner) gdelta[tid] = (int32_t)((int64_t)dstart + tile_off - start);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * 64 + lane;
    if (i < src.n) {
      const uint32_t d = (key[r] >> shift) & (kRadixBins - 1);
      const uint32_t lp = wcnt[w][d] + rank[r];
      skey[lp] = key[r];
      sval[lp] = val[r];
    }
  }
  __syncthreads();
  const int cnt = (int)min<int64_t>(kRadixTile, src.n - tile0);
  for (int j = tid; j < cnt; j += kRadixThreads) {
    const uint32_t k = skey[j];
    const uint32_t d = (k >> shift) & (kRadixBins - 1);
    const int64_t pos = (int64_t)j + gdelta[d];
    if ((uint64_t)pos < (uint64_t)src.n) {  // always true with consistent offsets
      if (WRITE_KEYS) keys_out[pos] = k;
      vals_out[pos] = sval[j];
    }
  }
}

// ---- compaction ----------------------------------------------------------

__global__ __launch_bounds__(kSortThreads) void k_compact_count(
    const uint8_t* __restrict__ active, int64_t n, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t wtot[kSortThreads / 64];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t base = (int64_t)blockIdx.x * kSortTile + w * (kSortTile / 4);
  uint32_t c = 0;
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * 64 + lane;
    c += (uint32_t)__popcll(__ballot(i < n && active[i] != 0));
  }
  if (lane == 0) wtot[w] = c;
  __syncthreads();
  if (tid == 0) cnt[blockIdx.x] = wtot[0] + wtot[1] + wtot[2] + wtot[3];
}

// Exclusive scan of the tile counts in one block; total -> *count.
__global__ __launch_bounds__(1024) void k_compact_scan(
    uint32_t* __restrict__ cnt, int32_t nT, int64_t* __restrict__ count) {
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nT; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const uint32_t x = i < nT ? cnt[i] : 0u;
    uint32_t tot;
    const uint32_t incl = block_incl_scan<1024>(x, &tot);
    if (i < nT) cnt[i] = carry + incl - x;
    carry += tot;
  }
  if (threadIdx.x == 0) *count = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_compact_scatter(
    const uint8_t* __restrict__ active, int64_t n,
    const uint32_t* __restrict__ toff, int32_t* __restrict__ list) {
  __shared__ uint32_t wtot[kSortThreads / 64];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int64_t base = (int64_t)blockIdx.x * kSortTile + w * (kSortTile / 4);
  uint64_t bal[kSortItems];
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * 64 + lane;
    bal[r] = __ballot(i < n && active[i] != 0);
    c += (uint32_t)__popcll(bal[r]);
  }
  if (lane == 0) wtot[w] = c;
  __syncthreads();
  uint32_t pos = toff[blockIdx.x];
  for (int ww = 0; ww < w; ++ww) pos += wtot[ww];
  const uint64_t below = lanes_below(lane);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t at = pos + (uint32_t)__popcll(bal[r] & below);
    if (((bal[r] >> lane) & 1ull) && at < (uint64_t)n)
      list[at] = (int32_t)(base + r * 64 + lane);
    pos += (uint32_t)__popcll(bal[r]);
  }
}

// The number of active lookups after a sort whose key carries the inactive
// flag as its top bit: the keys whose last-pass digit is below the flag's.
__global__ __launch_bounds__(kRadixBins) void k_count_below(
    const uint32_t* __restrict__ totals, uint32_t flag_digit,
    int64_t* __restrict__ count) {
  uint32_t all;
  const uint32_t x = threadIdx.x < flag_digit ? totals[threadIdx.x] : 0u;
  (void)block_incl_scan<kRadixBins>(x, &all);
  if (threadIdx.x == 0) *count = all;
}

// ---- block ranges over a sorted queue -------------------------------------
//
// The LDS-staged lookup shares one material's windows across a block, so a
// block that straddles two groups of the sort key (two materials) falls
// back to the per-lane walk.  Cutting the queue at every group and each
// group into block-sized pieces removes such blocks; a group's last piece
// is partly idle instead.

// starts[g] = the number of keys with key >> gshift < g, for g in
// [0, groups]: one wave per group, 64 probes per step over the sorted keys.
__global__ __launch_bounds__(256) void k_group_starts(
    const uint32_t* __restrict__ keys, int64_t n, int gshift, int64_t groups,
    int32_t* __restrict__ starts) {
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g > groups) return;
  const uint64_t target = (uint64_t)g << gshift;
  // the count lies in [lo, lo + len]
  int64_t lo = 0, len = n;
  while (len > 64) {
    const int64_t p = lo + (int64_t)(lane + 1) * len / 65;
    const int c = __popcll(__ballot(keys[p] < target));
    const int64_t p_lo = lo + (int64_t)c * len / 65;        // probe c - 1
    const int64_t p_hi = lo + (int64_t)(c + 1) * len / 65;  // probe c
    const int64_t nlo = c == 0 ? lo : p_lo + 1;
    const int64_t nhi = c == 64 ? lo + len : p_hi;
    lo = nlo;
    len = nhi - nlo;
  }
  const int c =
      __popcll(__ballot(lane < len && keys[lo + lane] < target));
  if (lane == 0) starts[g] = (int32_t)(lo + c);
}

// first[j] = the first block of group j (blocks of per_block positions per
// group, the last one partial), first[groups] = their total.
__global__ __launch_bounds__(1024) void k_block_prefix(
    const int32_t* __restrict__ starts, int64_t groups, int64_t per_block,
    int32_t* __restrict__ first) {
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < groups; c0 += 1024) {
    const int64_t j = c0 + threadIdx.x;
    const uint32_t nb =
        j < groups ? (uint32_t)((starts[j + 1] - starts[j] + per_block - 1) /
                                per_block)
                   : 0u;
    uint32_t tot;
    const uint32_t incl = block_incl_scan<1024>(nb, &tot);
    if (j < groups) first[j] = (int32_t)(carry + incl - nb);
    carry += tot;
  }
  if (threadIdx.x == 0) first[groups] = (int32_t)carry;
}

// ranges[2v], ranges[2v + 1] = the queue positions of block v: the piece
// (v - first[j]) of group j, the last group whose first block is <= v, for
// the blocks of groups [0, used).
__global__ __launch_bounds__(256) void k_block_ranges(
    const int32_t* __restrict__ starts, const int32_t* __restrict__ first,
    int64_t groups, int64_t used, int64_t per_block, int64_t max_blocks,
    int32_t* __restrict__ ranges) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= max_blocks || v >= first[used]) return;
  int64_t lo = 0, hi = groups - 1;  // at most log2(groups) + 1 steps
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (first[mid] <= v) lo = mid; else hi = mid - 1;
  }
  const int64_t b0 = starts[lo] + (v - first[lo]) * per_block;
  const int64_t b1 = b0 + per_block < starts[lo + 1] ? b0 + per_block
                                                     : starts[lo + 1];
  ranges[2 * v] = (int32_t)b0;
  ranges[2 * v + 1] = (int32_t)b1;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

hipError_t launch_block_ranges(const uint32_t* keys, int64_t n, int gshift,
                               int64_t groups, int64_t used, int64_t per_block,
                               void* spare, LookupArgs* a, hipStream_t s) {
  const int64_t max_blocks = (n + per_block - 1) / per_block + used;
  char* p = (char*)spare;
  auto* starts = (int32_t*)p; p += align256((size_t)(groups + 1) * 4);
  auto* first = (int32_t*)p;  p += align256((size_t)(groups + 1) * 4);
  p += 256;
  auto* ranges = (int32_t*)p;
  hipLaunchKernelGGL(k_group_starts, dim3((unsigned)((groups + 1 + 3) / 4)),
                     dim3(256), 0, s, keys, n, gshift, groups, starts);
  hipLaunchKernelGGL(k_block_prefix, dim3(1), dim3(1024), 0, s, starts,
                     groups, per_block, first);
  hipLaunchKernelGGL(k_block_ranges, dim3((unsigned)((max_blocks + 255) / 256)),
                     dim3(256), 0, s, starts, first, groups, used, per_block,
                     max_blocks, ranges);
  a->blocks = ranges;
  a->n_blocks = first + used;  // the blocks of the served groups
  a->max_blocks = max_blocks;
  return hipGetLastError();
}

size_t sort_workspace_bytes(int64_t n, int total_bits) {
  (void)total_bits;
  const int64_t nT = (n + kRadixTile - 1) / kRadixTile;
  return 4 * align256((size_t)n * 4) + align256((size_t)nT * kRadixBins * 4) +
         align256(kRadixBins * 4);
}

size_t compact_workspace_bytes(int64_t n) {
  const int64_t nT = (n + kSortTile - 1) / kSortTile;
  return align256((size_t)n * 4) + align256((size_t)nT * 4) + align256(8);
}

hipError_t launch_sort(const SortKey& key, int64_t n, const double* E,
                       const int32_t* mat, const uint8_t* active, void* ws,
                       const int32_t** perm_out, const uint32_t** keys_out,
                       uint32_t** spare, const int64_t** active_out,
                       hipStream_t s) {
  const int32_t nT = (int32_t)((n + kRadixTile - 1) / kRadixTile);
  char* p = (char*)ws;
  uint32_t* bufk[2];
  uint32_t* bufv[2];
  bufk[0] = (uint32_t*)p; p += align256((size_t)n * 4);
  bufv[0] = (uint32_t*)p; p += align256((size_t)n * 4);
  bufk[1] = (uint32_t*)p; p += align256((size_t)n * 4);
  bufv[1] = (uint32_t*)p; p += align256((size_t)n * 4);
  uint32_t* hist = (uint32_t*)p; p += align256((size_t)nT * kRadixBins * 4);
  uint32_t* totals = (uint32_t*)p;

  SortSrc src{E, mat, active, key, n};
  const int passes = (key.total_bits + kRadixBits - 1) / kRadixBits;
  int cur = 0;  // buffer holding the current keys/vals (after pass 0)
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * kRadixBits;
    const bool first = pass == 0, last = pass == passes - 1;
    const int dst = first ? 0 : 1 - cur;
    // The first pass writes the keys to bufk[1], which the second pass
    // rewrites only after the first pass's scatter has read them.
    if (first)
      hipLaunchKernelGGL((k_radix_hist<true>), dim3(nT), dim3(kRadixThreads), 0,
                         s, src, nullptr, shift, hist, nT, bufk[1]);
    else
      hipLaunchKernelGGL((k_radix_hist<false>), dim3(nT), dim3(kRadixThreads), 0,
                         s, src, bufk[cur], shift, hist, nT, nullptr);
    if (nT <= 512)
      hipLaunchKernelGGL(k_row_scan<256>, dim3(kRadixBins), dim3(256), 0, s,
                         hist, nT, totals);
    else
      hipLaunchKernelGGL(k_row_scan<1024>, dim3(kRadixBins), dim3(1024), 0, s,
                         hist, nT, totals);
    // the last pass writes its keys only when they are asked for; the
    // keys it reads are no longer needed after it
    if (last && keys_out) {
      *keys_out = bufk[dst];
      *spare = first ? bufk[1] : bufk[cur];
      if (first)
        hipLaunchKernelGGL((k_radix_scatter<true, true>), dim3(nT),
                           dim3(kRadixThreads), 0, s, src, bufk[1], nullptr,
                           shift, hist, totals, nT, bufk[dst], bufv[dst]);
      else
        hipLaunchKernelGGL((k_radix_scatter<false, true>), dim3(nT),
                           dim3(kRadixThreads), 0, s, src, bufk[cur], bufv[cur],
                           shift, hist, totals, nT, bufk[dst], bufv[dst]);
    } else if (first && last)
      hipLaunchKernelGGL((k_radix_scatter<true, false>), dim3(nT),
                         dim3(kRadixThreads), 0, s, src, bufk[1], nullptr, shift,
                         hist, totals, nT, bufk[dst], bufv[dst]);
    else if (first)
      hipLaunchKernelGGL((k_radix_scatter<true, true>), dim3(nT),
                         dim3(kRadixThreads), 0, s, src, bufk[1], nullptr, shift,
                         hist, totals, nT, bufk[dst], bufv[dst]);
    else if (last)
      hipLaunchKernelGGL((k_radix_scatter<false, false>), dim3(nT),
                         dim3(kRadixThreads), 0, s, src, bufk[cur], bufv[cur],
                         shift, hist, totals, nT, bufk[dst], bufv[dst]);
    else
      hipLaunchKernelGGL((k_radix_scatter<false, true>), dim3(nT),
                         dim3(kRadixThreads), 0, s, src, bufk[cur], bufv[cur],
                         shift, hist, totals, nT, bufk[dst], bufv[dst]);
    cur = dst;
  }
  *perm_out = (const int32_t*)bufv[cur];
  if (active_out && key.flag_bit) {
    // the flag is the key's top bit, in the last pass's digit; the count
    // goes where the histograms were (no longer read)
    const int last_shift = (passes - 1) * kRadixBits;
    const uint32_t flag_digit = 1u << (key.total_bits - 1 - last_shift);
    auto* count = (int64_t*)hist;
    hipLaunchKernelGGL(k_count_below, dim3(1), dim3(kRadixBins), 0, s, totals,
                       flag_digit, count);
    *active_out = count;
  }
  return hipGetLastError();
}

hipError_t launch_compact(int64_t n, const uint8_t* active, void* ws,
                          const int32_t** perm_out, const int64_t** count_out,
                          hipStream_t s) {
  const int32_t nT = (int32_t)((n + kSortTile - 1) / kSortTile);
  char* p = (char*)ws;
  int32_t* list = (int32_t*)p; p += align256((size_t)n * 4);
  uint32_t* cnt = (uint32_t*)p; p += align256((size_t)nT * 4);
  int64_t* count = (int64_t*)p;
  hipLaunchKernelGGL(k_compact_count, dim3(nT), dim3(kSortThreads), 0, s,
                     active, n, cnt);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, cnt, nT, count);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nT), dim3(kSortThreads), 0, s,
                     active, n, cnt, list);
  *perm_out = list;
  *count_out = count;
  return hipGetLastError();
}

}  // namespace xs
