// Many uneven lookup requests served together: xs_lookup_requests (one
// call per batch of requests) and the request streams xs_stream_* (a
// persistent kernel replayed from a HIP graph).
//
// The paper's particle buffer is refilled after every kernel call and the
// host launches one event kernel per queue (section 5.1, "maximum number of
// particles in-flight" and "queuing logic"); with short kernels the launch
// and the count transfer to the host leave bubbles.  Here a batch of
// requests is described once in device memory and drained by one launch
// (or, batch-sorted, by one gather, one sorted lookup and one scatter).  The
// request kernels work in tiles of 1024 lookups: a block sorts its tile in
// LDS by (material, energy) so that waves hold one material, runs the lookup
// walk of the main kernel and stamps the request's first and last tile times
// with the device wall clock.  Every loop bound is a kernel argument
// computed on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <limits>
#include <vector>

#include "xs_lookup_impl.h"
#include "xs_stream_tiles.h"

namespace xs {
namespace {

constexpr int kStreamThreads = 256;
constexpr int kPerLane = kStreamTile / kStreamThreads;

// Tile sort key: material in the high 16 bits, then the top 16 bits of the
// energy key; lanes without a lookup sort last.
__device__ __forceinline__ uint32_t tile_key(double e, int m, int M,
                                             int64_t ebits_min, int eshift) {
  int64_t d = __double_as_longlong(e) - ebits_min;
  d = d < 0 ? 0 : (d >> eshift);
  const uint32_t ek = (uint32_t)(d > 0xffff ? 0xffff : d);
  const uint32_t mm = (uint32_t)(m < 0 ? 0 : (m >= M ? M - 1 : m));
  return (mm << 16) | ek;
}

// Sorts the tile's lookups in LDS by (material, energy) and looks them up:
// lane tid takes sorted positions tid, tid + 256, ...  Called by all 256
// lanes of the block; the caller synchronises before reusing skey/sidx.
template <int GRID, int PREC, int U>
__device__ __forceinline__ void process_tile(const DevTables& t,
                                             const ReqDev& R, int64_t base,
                                             uint32_t* skey, uint16_t* sidx,
                                             int64_t ebits_min, int eshift) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int p = 0; p < kPerLane; ++p) {
    const int pos = tid + p * kStreamThreads;
    const int64_t q = base + pos;
    uint32_t key = 0xffffffffu;
    if (q < R.n) key = tile_key(R.E[q], R.mat[q], t.M, ebits_min, eshift);
    skey[pos] = key;
    sidx[pos] = (uint16_t)pos;
  }
  __syncthreads();
  // Bitonic network over the 1024 (key, position) pairs.
  for (int k = 2; k <= kStreamTile; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int p = 0; p < kPerLane / 2; ++p) {
        const int i = tid + p * kStreamThreads;  // pair (a, a + j), bit j of a clear
        const int a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const int b = a | j;
        const bool up = (a & k) == 0;
        const uint32_t ka = skey[a], kb = skey[b];
        if ((ka > kb) == up) {
          skey[a] = kb;
          skey[b] = ka;
          const uint16_t t2 = sidx[a];
          sidx[a] = sidx[b];
          sidx[b] = t2;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll 1
  for (int p = 0; p < kPerLane; ++p) {
    const int pos = tid + p * kStreamThreads;
    const int64_t q = base + sidx[pos];
    const bool act = q < R.n;
    double e = 1.0;
    int m = -1;
    if (act) {
      e = R.E[q];
      m = R.mat[q];
    }
    const bool ok = act && valid_query(e, m, t.M);
    if (act && !ok) Acc<PREC>::store_nan(R.out, q);
    const int mu = __builtin_amdgcn_readfirstlane(m);
    const bool wave_uniform = __all(ok && m == mu);
    if (ok) {
      const double e1[1] = {e};
      Locator<GRID> loc[1];
      Acc<PREC> acc[1];
      loc[0].init(t, e, m);
      acc[0].zero();
      if (wave_uniform)
        walk_material<GRID, PREC, 1, U>(t, mu, e1, loc, acc);
      else
        walk_material<GRID, PREC, 1, U>(t, m, e1, loc, acc);
      acc[0].store(R.out, q);
    }
  }
}

// Persistent form for request streams: a fixed grid (a few blocks per
// compute unit) strides over the batch's tiles.  Nothing read from device
// memory bounds a loop: the tile count, the request count, the batch's tag
// and the largest request size are kernel arguments, rewritten in the
// instantiated graph before every launch, so every block leaves after at
// most ceil(tiles / gridDim) tiles whatever the descriptors hold.  A tile
// whose descriptor fails descriptor_ok (not written for this batch) is
// skipped without touching the descriptor's pointers and counted in
// stamps[2 * count + 1], which the host turns into an error.
template <int GRID, int PREC, int U>
__global__ __launch_bounds__(kStreamThreads) void k_stream(
    const DevTables t, const ReqDev* __restrict__ reqs, int count,
    int64_t tiles, uint64_t tag, int64_t max_n, unsigned long long* stamps,
    int64_t ebits_min, int eshift) {
  __shared__ uint32_t skey[kStreamTile];
  __shared__ uint16_t sidx[kStreamTile];
  __shared__ int s_req;
  __shared__ int s_ok;
  for (int64_t g = blockIdx.x; g < tiles; g += gridDim.x) {
    const unsigned long long t0 = wall_clock64();
    // One lane picks and checks the descriptor; the block follows its
    // verdict, so the barriers inside process_tile are met by every lane.
    if (threadIdx.x == 0) {
      const int r = request_of(reqs, count, g);
      s_req = r;
      s_ok = descriptor_ok(reqs[r], g, tag, max_n) ? 1 : 0;
    }
    __syncthreads();
    const int r = s_req;
    const bool ok = s_ok != 0;
    if (ok) {
      const ReqDev R = reqs[r];
      process_tile<GRID, PREC, U>(t, R, (g - R.tile_begin) * kStreamTile,
                                  skey, sidx, ebits_min, eshift);
    }
    __syncthreads();  // LDS and s_req / s_ok are rewritten for the next tile
    if (threadIdx.x == 0) {
      if (ok) {
        const unsigned long long t1 = wall_clock64();
        atomicMin(&stamps[2 * r], t0);
        atomicMax(&stamps[2 * r + 1], t1);
        atomicMin(&stamps[2 * count], t0);
      } else {
        atomicAdd(&stamps[2 * count + 1], 1ull);
      }
    }
  }
}

// One launch for a batch of requests: block b processes global tile b (the
// grid is exactly the batch's tile count, computed on the host), so no block
// waits on or loops over anything read from device memory.
template <int GRID, int PREC, int U>
__global__ __launch_bounds__(kStreamThreads) void k_requests(
    const DevTables t, const ReqDev* __restrict__ reqs, int count,
    unsigned long long* stamps, int64_t ebits_min, int eshift) {
  __shared__ uint32_t skey[kStreamTile];
  __shared__ uint16_t sidx[kStreamTile];
  const int64_t g = blockIdx.x;
  const unsigned long long t0 = wall_clock64();
  const int r = request_of(reqs, count, g);
  const ReqDev R = reqs[r];
  process_tile<GRID, PREC, U>(t, R, (g - R.tile_begin) * kStreamTile, skey,
                              sidx, ebits_min, eshift);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t1 = wall_clock64();
    atomicMin(&stamps[2 * r], t0);
    atomicMax(&stamps[2 * r + 1], t1);
    atomicMin(&stamps[2 * count], t0);
  }
}

// stamps[2r] = first start (init: max), stamps[2r+1] = last end (init: 0),
// stamps[2*count] = batch start, stamps[2*count+1] = tiles skipped because
// their descriptor was not the batch's (request streams).
__global__ void k_requests_init(unsigned long long* stamps, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    stamps[2 * i] = ~0ull;
    stamps[2 * i + 1] = 0;
  }
  if (i == 0) {
    stamps[2 * count] = ~0ull;
    stamps[2 * count + 1] = 0;
  }
}

// Batch-sorted mode, step 1: block b copies tile b of its request into the
// concatenated (E, material) arrays and stamps the request's start.
__global__ __launch_bounds__(kStreamThreads) void k_requests_gather(
    const ReqDev* __restrict__ reqs, int count, double* __restrict__ E_all,
    int32_t* __restrict__ m_all, unsigned long long* stamps) {
  const int64_t g = blockIdx.x;
  const unsigned long long t0 = wall_clock64();
  const int r = request_of(reqs, count, g);
  const ReqDev R = reqs[r];
  const int64_t base = (g - R.tile_begin) * kStreamTile;
#pragma unroll
  for (int p = 0; p < kPerLane; ++p) {
    const int64_t q = base + threadIdx.x + p * kStreamThreads;
    if (q < R.n) {
      E_all[R.begin + q] = R.E[q];
      m_all[R.begin + q] = R.mat[q];
    }
  }
  if (threadIdx.x == 0) {
    atomicMin(&stamps[2 * r], t0);
    atomicMin(&stamps[2 * count], t0);
  }
}

// Batch-sorted mode, step 3: block b copies tile b of its request's results
// from the concatenated output and stamps the request's end.
template <class T>
__global__ __launch_bounds__(kStreamThreads) void k_requests_scatter(
    const ReqDev* __restrict__ reqs, int count, const T* __restrict__ out_all,
    unsigned long long* stamps) {
  const int64_t g = blockIdx.x;
  const int r = request_of(reqs, count, g);
  const ReqDev R = reqs[r];
  const int64_t base = (g - R.tile_begin) * kStreamTile * XS_CHANNELS;
  const int64_t len = R.n * XS_CHANNELS;
  T* out = (T*)R.out;
  const T* src = out_all + R.begin * XS_CHANNELS;
  for (int k = threadIdx.x; k < kStreamTile * XS_CHANNELS; k += kStreamThreads) {
    const int64_t q = base + k;
    if (q < len) out[q] = src[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&stamps[2 * r + 1], wall_clock64());
}

}  // namespace
}  // namespace xs


// ---- one launch for a batch of requests ------------------------------------

namespace xs {
namespace {

size_t align256b(size_t b) { return (b + 255) & ~size_t(255); }

template <int GRID, int PREC, int U>
hipError_t launch_requests_kernel(const DevTables& t, const ReqDev* reqs,
                                  int count, unsigned long long* stamps,
                                  int64_t tiles, int64_t bmin, int shift,
                                  hipStream_t s) {
  hipLaunchKernelGGL((k_requests<GRID, PREC, U>), dim3((unsigned)tiles),
                     dim3(kStreamThreads), 0, s, t, reqs, count, stamps, bmin,
                     shift);
  return hipGetLastError();
}

template <int GRID, int PREC>
hipError_t launch_requests_u(const xs_params& p, const DevTables& t,
                             const ReqDev* reqs, int count,
                             unsigned long long* stamps, int64_t tiles,
                             int64_t bmin, int shift, hipStream_t s) {
  switch (p.unroll) {
    case 1: return launch_requests_kernel<GRID, PREC, 1>(t, reqs, count, stamps, tiles, bmin, shift, s);
    case 2: return launch_requests_kernel<GRID, PREC, 2>(t, reqs, count, stamps, tiles, bmin, shift, s);
    default: return launch_requests_kernel<GRID, PREC, 4>(t, reqs, count, stamps, tiles, bmin, shift, s);
  }
}

template <int GRID>
hipError_t launch_requests_p(const xs_params& p, const DevTables& t,
                             const ReqDev* reqs, int count,
                             unsigned long long* stamps, int64_t tiles,
                             int64_t bmin, int shift, hipStream_t s) {
  return p.precision == XS_FP64
             ? launch_requests_u<GRID, XS_FP64>(p, t, reqs, count, stamps, tiles, bmin, shift, s)
             : launch_requests_u<GRID, XS_FP32>(p, t, reqs, count, stamps, tiles, bmin, shift, s);
}

void energy_key_shift(const xs_tables_s* h, int64_t* bmin, int* shift) {
  int64_t lo, hi;
  std::memcpy(&lo, &h->info.e_min, 8);
  std::memcpy(&hi, &h->info.e_max, 8);
  int sh = 0;
  while (((hi - lo) >> sh) > 0xffff) ++sh;
  *bmin = lo;
  *shift = sh;
}

// Batch-sorted serving (after the stamps are reset): one gather kernel
// copies every request into one queue, the queue is sorted and looked up as
// one batch, and one scatter kernel writes each request's results back.
// `lookup` runs the sorted lookup of the gathered queue on the stream.
template <class Lookup>
xs_status enqueue_batch_sorted(const ReqDev* reqs_dev, int count, int64_t tiles,
                               int precision, unsigned long long* stamps,
                               double* E_all, int32_t* m_all, void* out_all,
                               hipStream_t s, Lookup lookup) {
  const dim3 grid((unsigned)tiles), block(kStreamThreads);
  hipLaunchKernelGGL(k_requests_gather, grid, block, 0, s, reqs_dev, count,
                     E_all, m_all, stamps);
  XS_HIP(hipGetLastError());
  if (xs_status st = lookup()) return st;
  if (precision == XS_FP64)
    hipLaunchKernelGGL(k_requests_scatter<double>, grid, block, 0, s, reqs_dev,
                       count, (const double*)out_all, stamps);
  else
    hipLaunchKernelGGL(k_requests_scatter<float>, grid, block, 0, s, reqs_dev,
                       count, (const float*)out_all, stamps);
  XS_HIP(hipGetLastError());
  return XS_OK;
}

// Validation, parameters and workspace layout of one xs_lookup_requests call.
struct RequestPlan {
  xs_params p{};
  int64_t total = 0;   // lookups in the batch
  int64_t tiles = 0;   // 1024-lookup tiles (each request starts a tile)
  bool batch_sorted = false;
  size_t off_stamps = 0, off_E = 0, off_mat = 0, off_out = 0,
         off_lookup_ws = 0, lookup_ws_bytes = 0, ws_bytes = 0;
};

xs_status plan_requests(xs_tables_t h, const xs_request* reqs, int32_t count,
                        const xs_params* params, RequestPlan* plan) {
  if (!h) return fail(XS_EINVAL, "table handle is NULL");
  if (count < 1 || count > (1 << 24) || !reqs)
    return fail(XS_EINVAL, "count must be in [1, 2^24] and reqs not NULL");
  RequestPlan q;
  for (int i = 0; i < count; ++i) {
    const xs_request& r = reqs[i];
    if (r.n < 0 || r.n > 0x7fffffffLL)
      return fail(XS_EINVAL, "request %d: n out of range", i);
    if (r.n > 0 && (!r.d_E || !r.d_mat || !r.d_out))
      return fail(XS_EINVAL, "request %d: a pointer is NULL", i);
    q.total += r.n;
    q.tiles += (r.n + kStreamTile - 1) / kStreamTile;
  }
  if (q.tiles > 0x7fffffffLL || q.total > 0x7fffffffLL)
    return fail(XS_EINVAL, "batch too large (at most 2^31 - 1 lookups)");
  // Parameters as for one batch of the whole size.
  if (xs_status st = xs_resolve_params(h, std::max<int64_t>(q.total, 1), params,
                                       &q.p))
    return st;
  q.batch_sorted = q.p.sort != XS_SORT_NONE && q.total >= q.p.sort_threshold &&
                   q.total > 0;
  size_t off = align256b(sizeof(ReqDev) * (size_t)count);
  q.off_stamps = off;
  off += align256b(8 * (2 * (size_t)count + 1));
  if (q.batch_sorted) {
    const size_t esz = q.p.precision == XS_FP64 ? 8 : 4;
    q.off_E = off;
    off += align256b(8 * (size_t)q.total);
    q.off_mat = off;
    off += align256b(4 * (size_t)q.total);
    q.off_out = off;
    off += align256b(esz * XS_CHANNELS * (size_t)q.total);
    if (xs_status st = xs_workspace_size(h, q.total, &q.p, &q.lookup_ws_bytes))
      return st;
    q.off_lookup_ws = off;
    off += align256b(q.lookup_ws_bytes);
  }
  q.ws_bytes = off;
  *plan = q;
  return XS_OK;
}

}  // namespace
}  // namespace xs

using namespace xs;

extern "C" {

xs_status xs_requests_workspace_size(xs_tables_t h, const xs_request* reqs,
                                     int32_t count, const xs_params* params,
                                     size_t* bytes) {
  clear_error();
  if (!bytes) return fail(XS_EINVAL, "bytes is NULL");
  RequestPlan plan;
  if (xs_status st = plan_requests(h, reqs, count, params, &plan)) return st;
  *bytes = plan.ws_bytes;
  return XS_OK;
}

xs_status xs_lookup_requests(xs_tables_t h, const xs_request* reqs,
                             int32_t count, const xs_params* params,
                             void* d_ws, size_t ws_bytes, void* stream) {
  clear_error();
  RequestPlan plan;
  if (xs_status st = plan_requests(h, reqs, count, params, &plan)) return st;
  if (!d_ws || ws_bytes < plan.ws_bytes || (uintptr_t)d_ws % 256)
    return fail(XS_EWORKSPACE, "a 256-byte aligned workspace of %zu bytes is "
                "needed", plan.ws_bytes);
  int dev = -1;
  XS_HIP(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(XS_EINVAL, "current device %d is not the tables' device %d",
                dev, h->device);
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)d_ws;
  ReqDev* reqs_dev = (ReqDev*)ws;
  auto* stamps = (unsigned long long*)(ws + plan.off_stamps);
  {
    std::lock_guard<std::mutex> lk(h->mu);
    const size_t bytes = sizeof(ReqDev) * (size_t)count;
    if (h->req_event) XS_HIP(hipEventSynchronize(h->req_event));
    if (h->req_stage_bytes < bytes) {
      if (h->req_stage) XS_HIP(hipHostFree(h->req_stage));
      h->req_stage = nullptr;
      h->req_stage_bytes = 0;
      XS_HIP(hipHostMalloc(&h->req_stage, bytes));
      h->req_stage_bytes = bytes;
    }
    if (!h->req_event) XS_HIP(hipEventCreateWithFlags(&h->req_event,
                                                      hipEventDisableTiming));
    auto* rd = (ReqDev*)h->req_stage;
    int64_t tiles = 0, begin = 0;
    for (int i = 0; i < count; ++i) {
      const xs_request& r = reqs[i];
      rd[i] = ReqDev{r.d_E, r.d_mat, r.d_out, r.n, tiles, begin};
      tiles += (r.n + kStreamTile - 1) / kStreamTile;
      begin += r.n;
    }
    XS_HIP(hipMemcpyAsync(reqs_dev, rd, bytes, hipMemcpyHostToDevice, s));
    XS_HIP(hipEventRecord(h->req_event, s));
  }
  hipLaunchKernelGGL(k_requests_init, dim3((count + 1 + 255) / 256), dim3(256),
                     0, s, stamps, count);
  XS_HIP(hipGetLastError());
  if (plan.tiles == 0) return XS_OK;
  const xs_params& p = plan.p;

  if (plan.batch_sorted) {
    auto* E_all = (double*)(ws + plan.off_E);
    auto* m_all = (int32_t*)(ws + plan.off_mat);
    void* out_all = ws + plan.off_out;
    return enqueue_batch_sorted(
        reqs_dev, count, plan.tiles, p.precision, stamps, E_all, m_all,
        out_all, s, [&] {
          return xs_lookup_batch(h, plan.total, E_all, m_all, out_all, &p,
                                 ws + plan.off_lookup_ws, plan.lookup_ws_bytes,
                                 stream);
        });
  }

  int64_t bmin;
  int shift;
  energy_key_shift(h, &bmin, &shift);
  hipError_t e;
  switch (p.grid) {
    case XS_GRID_NUCLIDE:
      e = launch_requests_p<XS_GRID_NUCLIDE>(p, tables_for(h, p), reqs_dev, count, stamps, plan.tiles, bmin, shift, s);
      break;
    case XS_GRID_HASH:
      e = launch_requests_p<XS_GRID_HASH>(p, tables_for(h, p), reqs_dev, count, stamps, plan.tiles, bmin, shift, s);
      break;
    default:
      e = launch_requests_p<XS_GRID_UNIONIZED>(p, tables_for(h, p), reqs_dev, count, stamps, plan.tiles, bmin, shift, s);
      break;
  }
  if (e != hipSuccess)
    return fail(XS_EHIP, "request kernel launch failed: %s", hipGetErrorString(e));
  return XS_OK;
}

xs_status xs_requests_stats(const void* d_ws, int32_t count, void* stream,
                            xs_request_stats* stats, double* makespan_us) {
  clear_error();
  if (!d_ws || count < 1) return fail(XS_EINVAL, "workspace and count needed");
  hipStream_t s = (hipStream_t)stream;
  XS_HIP(s ? hipStreamSynchronize(s) : hipDeviceSynchronize());
  std::vector<ReqDev> rd(count);
  std::vector<unsigned long long> st(2 * (size_t)count + 1);
  XS_HIP(hipMemcpy(rd.data(), d_ws, sizeof(ReqDev) * (size_t)count,
                   hipMemcpyDeviceToHost));
  XS_HIP(hipMemcpy(st.data(),
                   (const char*)d_ws + align256b(sizeof(ReqDev) * (size_t)count),
                   8 * st.size(), hipMemcpyDeviceToHost));
  int dev = 0, khz = 0;
  XS_HIP(hipGetDevice(&dev));
  XS_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  const double us_per_tick = 1000.0 / (khz > 0 ? khz : 100000);
  const unsigned long long t0 = st[2 * (size_t)count];
  unsigned long long tmax = t0;
  for (int i = 0; i < count; ++i)
    if (st[2 * i] != ~0ull) tmax = std::max(tmax, st[2 * i + 1]);
  if (makespan_us) *makespan_us = t0 == ~0ull ? 0.0 : (tmax - t0) * us_per_tick;
  if (stats) {
    for (int i = 0; i < count; ++i) {
      xs_request_stats& r = stats[i];
      r.n = rd[i].n;
      if (st[2 * i] == ~0ull) {
        r.start_us = r.end_us = r.latency_us = 0.0;
        continue;
      }
      r.start_us = (st[2 * i] - t0) * us_per_tick;
      r.end_us = (st[2 * i + 1] - t0) * us_per_tick;
      r.latency_us = r.end_us - r.start_us;
    }
  }
  return XS_OK;
}

}  // extern "C"

// ---- request streams: a reusable graph per batch ----------------------------
//
// Two modes, chosen per batch from the parameters resolved for its total
// size.  Tile mode (no sort, or fewer lookups than the sort threshold): the
// graph [reset stamps] -> [persistent kernel], built once; each submit
// rewrites the two nodes' arguments.  Sorted mode: the batch-sorted
// pipeline of xs_lookup_requests (gather, sort, staged lookup, scatter) is
// captured from a private stream and the stream's second executable graph
// is updated in place (re-instantiated only when the kernels differ from
// the previous sorted batch's); its buffers grow with the largest batch.
//
// Ordering of a submit: the descriptors are written to pinned host memory,
// copied to the device on the stream object's own upload stream, and the
// host waits for that copy to complete before it rewrites or captures the
// graph and launches it on the caller's stream.  No kernel therefore starts
// before its descriptors are in device memory, whatever the runtime does to
// order a copy against a graph launch on one stream; and in tile mode each
// descriptor carries the batch's tag, which the kernel checks before it
// uses the descriptor.

struct xs_stream_s {
  xs_tables_t tables = nullptr;
  xs_params params{};
  xs_params user{};        // as given at creation (resolved per batch)
  bool has_user = false;
  hipStream_t capture = nullptr;   // sorted mode: captures the pipeline
  hipGraphExec_t sexec = nullptr;  // sorted mode: the pipeline's graph
  void* sorted_ws = nullptr;       // queue, results and sort workspace
  size_t sorted_ws_bytes = 0;
  bool last_sorted = false;        // mode of the batch in flight
  hipStream_t stream = nullptr;  // the caller's stream (graph launches)
  hipStream_t upload = nullptr;  // descriptor copies (host waits for them)
  int32_t max_requests = 0;
  int32_t pending = 0;  // requests of the batch in flight (0 = idle)
  uint64_t batches = 0; // submitted batches (tag source)
  xs::ReqDev* reqs_dev = nullptr;
  unsigned long long* stamps_dev = nullptr;  // 2 * max_requests + 2
  xs::ReqDev* host = nullptr;                // pinned staging of descriptors
  std::vector<int64_t> sizes;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t init_node = nullptr, run_node = nullptr;
  hipEvent_t done = nullptr;
  int blocks = 0;
  double clock_khz = 0;
  // kernel arguments of the two graph nodes (rewritten before each launch)
  xs::DevTables a_t{};
  const xs::ReqDev* a_reqs = nullptr;
  unsigned long long* a_stamps = nullptr;
  int a_count = 0;
  int64_t a_tiles = 0;
  uint64_t a_tag = 0;
  int64_t a_max_n = 0;
  int64_t a_bmin = 0;
  int a_shift = 0;
  void* run_args[9] = {};
  void* init_args[2] = {};
  const void* run_func = nullptr;
};

namespace xs {
namespace {

void stream_release(xs_stream_s* s) {
  if (s->sexec) (void)hipGraphExecDestroy(s->sexec);
  if (s->capture) (void)hipStreamDestroy(s->capture);
  if (s->sorted_ws) (void)hipFree(s->sorted_ws);
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->done) (void)hipEventDestroy(s->done);
  if (s->upload) (void)hipStreamDestroy(s->upload);
  if (s->reqs_dev) (void)hipFree(s->reqs_dev);
  if (s->stamps_dev) (void)hipFree(s->stamps_dev);
  if (s->host) (void)hipHostFree(s->host);
  delete s;
}

template <int GRID, int PREC>
const void* stream_func_p(int unroll) {
  switch (unroll) {
    case 1: return (const void*)&k_stream<GRID, PREC, 1>;
    case 2: return (const void*)&k_stream<GRID, PREC, 2>;
    default: return (const void*)&k_stream<GRID, PREC, 4>;
  }
}

const void* stream_func(const xs_params& p) {
  switch (p.grid) {
    case XS_GRID_NUCLIDE:
      return p.precision == XS_FP64 ? stream_func_p<XS_GRID_NUCLIDE, XS_FP64>(p.unroll)
                                    : stream_func_p<XS_GRID_NUCLIDE, XS_FP32>(p.unroll);
    case XS_GRID_HASH:
      return p.precision == XS_FP64 ? stream_func_p<XS_GRID_HASH, XS_FP64>(p.unroll)
                                    : stream_func_p<XS_GRID_HASH, XS_FP32>(p.unroll);
    default:
      return p.precision == XS_FP64 ? stream_func_p<XS_GRID_UNIONIZED, XS_FP64>(p.unroll)
                                    : stream_func_p<XS_GRID_UNIONIZED, XS_FP32>(p.unroll);
  }
}

hipKernelNodeParams init_params(xs_stream_s* s) {
  hipKernelNodeParams kp{};
  kp.func = (void*)&k_requests_init;
  kp.gridDim = dim3((s->max_requests + 1 + 255) / 256);
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  kp.kernelParams = s->init_args;
  kp.extra = nullptr;
  return kp;
}

hipKernelNodeParams run_params(xs_stream_s* s) {
  hipKernelNodeParams kp{};
  kp.func = (void*)s->run_func;
  kp.gridDim = dim3(s->blocks);
  kp.blockDim = dim3(kStreamThreads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = s->run_args;
  kp.extra = nullptr;
  return kp;
}

// Captures the batch-sorted pipeline for `count` requests (descriptors
// already in device memory) and launches it on the caller's stream.
xs_status submit_sorted(xs_stream_s* s, int count, int64_t tiles,
                        int64_t total, const xs_params& ps) {
  xs_tables_t h = s->tables;
  const size_t esz = ps.precision == XS_FP64 ? 8 : 4;
  size_t lws = 0;
  if (xs_status st = xs_workspace_size(h, total, &ps, &lws)) return st;
  const size_t off_mat = align256b(8 * (size_t)total);
  const size_t off_out = off_mat + align256b(4 * (size_t)total);
  const size_t off_ws = off_out + align256b(esz * XS_CHANNELS * (size_t)total);
  const size_t need = off_ws + align256b(lws);
  if (need > s->sorted_ws_bytes) {
    // No batch is in flight (a submit needs the previous one waited for).
    if (s->sorted_ws) XS_HIP(hipFree(s->sorted_ws));
    s->sorted_ws = nullptr;
    s->sorted_ws_bytes = 0;
    XS_HIP(hipMalloc(&s->sorted_ws, need));
    s->sorted_ws_bytes = need;
  }
  char* ws = (char*)s->sorted_ws;
  auto* E_all = (double*)ws;
  auto* m_all = (int32_t*)(ws + off_mat);
  void* out_all = ws + off_out;
  hipStream_t cap = s->capture;
  XS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_requests_init, dim3((count + 1 + 255) / 256), dim3(256),
                     0, cap, s->stamps_dev, count);
  xs_status st = enqueue_batch_sorted(
      s->reqs_dev, count, tiles, ps.precision, s->stamps_dev, E_all, m_all,
      out_all, cap, [&] {
        return lookup_batch_into(h, total, E_all, m_all, out_all, &ps,
                                 ws + off_ws, lws, cap);
      });
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(cap, &g);
  if (st == XS_OK && ce != hipSuccess)
    st = fail(XS_EHIP, "capturing the sorted batch failed: %s",
              hipGetErrorString(ce));
  if (st == XS_OK && s->sexec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult r = hipGraphExecUpdateSuccess;
    if (hipGraphExecUpdate(s->sexec, g, &bad, &r) != hipSuccess ||
        r != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(s->sexec);
      s->sexec = nullptr;
    }
  }
  if (st == XS_OK && !s->sexec) {
    const hipError_t ie = hipGraphInstantiate(&s->sexec, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      s->sexec = nullptr;
      st = fail(XS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    }
  }
  if (g) (void)hipGraphDestroy(g);
  if (st != XS_OK) return st;
  XS_HIP(hipGraphLaunch(s->sexec, s->stream));
  XS_HIP(hipEventRecord(s->done, s->stream));
  return XS_OK;
}

}  // namespace
}  // namespace xs

extern "C" {

xs_status xs_stream_create(xs_tables_t h, const xs_params* params,
                           int32_t max_requests, void* stream,
                           xs_stream_t* out) {
  clear_error();
  if (!h || !out) return fail(XS_EINVAL, "tables and out must not be NULL");
  if (max_requests < 1 || max_requests > (1 << 20))
    return fail(XS_EINVAL, "max_requests must be in [1, 2^20]");
  xs_params p;
  // Resolved like a large batch; sort, block size, lookups per lane and the
  // threshold do not apply (tiles are sorted in LDS, blocks are 256 lanes).
  if (xs_status st = xs_resolve_params(h, 1 << 20, params, &p)) return st;
  auto* s = new (std::nothrow) xs_stream_s();
  if (!s) return fail(XS_ENOMEM, "host allocation failed");
  s->tables = h;
  s->params = p;
  if (params) {
    s->user = *params;
    s->has_user = true;
  }
  s->stream = (hipStream_t)stream;
  s->max_requests = max_requests;
  auto bail = [&](xs_status st) {
    stream_release(s);
    return st;
  };
  auto hip = [&](hipError_t e, const char* what) -> xs_status {
    if (e == hipSuccess) return XS_OK;
    return fail(e == hipErrorOutOfMemory ? XS_ENOMEM : XS_EHIP, "%s: %s", what,
                hipGetErrorString(e));
  };
  xs_status st;
  const size_t req_bytes = sizeof(ReqDev) * (size_t)max_requests;
  if ((st = hip(hipMalloc(&s->reqs_dev, req_bytes), "hipMalloc")) ||
      (st = hip(hipMalloc(&s->stamps_dev, 8 * (2 * (size_t)max_requests + 2)),
                "hipMalloc")) ||
      (st = hip(hipHostMalloc(&s->host, req_bytes), "hipHostMalloc")) ||
      (st = hip(hipEventCreateWithFlags(&s->done, hipEventDisableTiming),
                "hipEventCreate")) ||
      (st = hip(hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking),
                "hipStreamCreateWithFlags")) ||
      (st = hip(hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking),
                "hipStreamCreateWithFlags")))
    return bail(st);
  int dev = 0, cus = 0, khz = 0;
  if ((st = hip(hipGetDevice(&dev), "hipGetDevice")) ||
      (st = hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                      dev), "hipDeviceGetAttribute")) ||
      (st = hip(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev),
                "hipDeviceGetAttribute")))
    return bail(st);
  if (dev != h->device)
    return bail(fail(XS_EINVAL, "current device %d is not the tables' device %d",
                     dev, h->device));
  s->blocks = std::max(1, cus) * 4;
  s->clock_khz = khz > 0 ? khz : 100000.0;

  // Kernel arguments live in the handle; the nodes point at them.  Until the
  // first submit the run node has no tiles and matches no descriptor.
  s->a_t = tables_for(h, p);
  s->a_reqs = s->reqs_dev;
  s->a_stamps = s->stamps_dev;
  s->a_count = 1;
  s->a_tiles = 0;
  s->a_tag = 0;
  s->a_max_n = 0;
  energy_key_shift(h, &s->a_bmin, &s->a_shift);
  s->run_args[0] = &s->a_t;
  s->run_args[1] = &s->a_reqs;
  s->run_args[2] = &s->a_count;
  s->run_args[3] = &s->a_tiles;
  s->run_args[4] = &s->a_tag;
  s->run_args[5] = &s->a_max_n;
  s->run_args[6] = &s->a_stamps;
  s->run_args[7] = &s->a_bmin;
  s->run_args[8] = &s->a_shift;
  s->init_args[0] = &s->a_stamps;
  s->init_args[1] = &s->a_count;
  s->run_func = stream_func(p);

  // The graph [reset stamps] -> [persistent kernel], built node by node.
  const hipKernelNodeParams ip = init_params(s), rp = run_params(s);
  if ((st = hip(hipGraphCreate(&s->graph, 0), "hipGraphCreate")) ||
      (st = hip(hipGraphAddKernelNode(&s->init_node, s->graph, nullptr, 0, &ip),
                "hipGraphAddKernelNode")) ||
      (st = hip(hipGraphAddKernelNode(&s->run_node, s->graph, &s->init_node, 1,
                                      &rp), "hipGraphAddKernelNode")) ||
      (st = hip(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0),
                "hipGraphInstantiate")))
    return bail(st);
  *out = s;
  return XS_OK;
}

xs_status xs_stream_submit(xs_stream_t s, const xs_request* reqs,
                           int32_t count) {
  clear_error();
  if (!s) return fail(XS_EINVAL, "stream is NULL");
  if (s->pending) return fail(XS_EINVAL, "a batch is still in flight; call "
                              "xs_stream_wait first");
  if (count < 1 || count > s->max_requests)
    return fail(XS_EINVAL, "count must be in [1, %d]", s->max_requests);
  if (!reqs) return fail(XS_EINVAL, "reqs is NULL");
  int64_t tiles = 0, begin = 0, max_n = 0;
  for (int i = 0; i < count; ++i) {
    const xs_request& r = reqs[i];
    if (r.n < 0 || r.n > 0x7fffffffLL)
      return fail(XS_EINVAL, "request %d: n out of range", i);
    if (r.n > 0 && (!r.d_E || !r.d_mat || !r.d_out))
      return fail(XS_EINVAL, "request %d: a pointer is NULL", i);
    tiles += tiles_of(r.n);
    begin += r.n;
    max_n = std::max<int64_t>(max_n, r.n);
  }
  if (tiles > 0x7fffffffLL) return fail(XS_EINVAL, "batch too large");
  // A tag no earlier batch of any stream object in the process used.
  static std::atomic<uint64_t> batches_in_process{0};
  const uint64_t tag = 0x9e3779b97f4a7c15ull * (++batches_in_process);
  ++s->batches;
  // The previous batch has been waited for, so the staging buffer and the
  // device descriptors are free.
  s->sizes.assign(count, 0);
  tiles = 0;
  begin = 0;
  for (int i = 0; i < count; ++i) {
    const xs_request& r = reqs[i];
    s->host[i] = ReqDev{r.d_E, r.d_mat, r.d_out, r.n, tiles, begin, tag, 0};
    tiles += tiles_of(r.n);
    begin += r.n;
    s->sizes[i] = r.n;
  }
  XS_HIP(hipMemcpyAsync(s->reqs_dev, s->host, sizeof(ReqDev) * count,
                        hipMemcpyHostToDevice, s->upload));
  XS_HIP(hipStreamSynchronize(s->upload));

  // Sorted mode when the parameters for this batch's size sort it (debug
  // mode synchronises inside the lookup, which a capture cannot hold).
  const int64_t total = begin;
  if (total > 0 && total <= 0x7fffffffLL && !s->tables->d.dbg) {
    xs_params ps;
    if (xs_status st = xs_resolve_params(s->tables, total,
                                         s->has_user ? &s->user : nullptr, &ps))
      return st;
    if (ps.sort != XS_SORT_NONE && total >= ps.sort_threshold) {
      if (xs_status st = submit_sorted(s, count, tiles, total, ps)) return st;
      s->last_sorted = true;
      s->pending = count;
      return XS_OK;
    }
  }
  s->last_sorted = false;
  s->a_count = count;
  s->a_tiles = tiles;
  s->a_tag = tag;
  s->a_max_n = max_n;
  const hipKernelNodeParams ip = init_params(s), rp = run_params(s);
  XS_HIP(hipGraphExecKernelNodeSetParams(s->exec, s->init_node, &ip));
  XS_HIP(hipGraphExecKernelNodeSetParams(s->exec, s->run_node, &rp));
  XS_HIP(hipGraphLaunch(s->exec, s->stream));
  XS_HIP(hipEventRecord(s->done, s->stream));
  s->pending = count;
  return XS_OK;
}

xs_status xs_stream_wait(xs_stream_t s, xs_request_stats* stats,
                         double* makespan_us) {
  clear_error();
  if (!s) return fail(XS_EINVAL, "stream is NULL");
  if (!s->pending) return fail(XS_EINVAL, "no batch in flight");
  XS_HIP(hipEventSynchronize(s->done));
  const int count = s->pending;
  s->pending = 0;
  std::vector<unsigned long long> st(2 * (size_t)count + 2);
  XS_HIP(hipMemcpy(st.data(), s->stamps_dev, 8 * st.size(),
                   hipMemcpyDeviceToHost));
  if (st[2 * (size_t)count + 1] != 0)
    return fail(XS_EHIP, "%llu tiles of the batch met request descriptors "
                "that were not this batch's and were skipped (their outputs "
                "are not written)", st[2 * (size_t)count + 1]);
  const double us_per_tick = 1000.0 / s->clock_khz;
  const unsigned long long t0 = st[2 * (size_t)count];
  unsigned long long tmax = t0;
  for (int i = 0; i < count; ++i)
    if (st[2 * i] != ~0ull) tmax = std::max(tmax, st[2 * i + 1]);
  if (makespan_us) *makespan_us = t0 == ~0ull ? 0.0 : (tmax - t0) * us_per_tick;
  if (stats) {
    for (int i = 0; i < count; ++i) {
      xs_request_stats& r = stats[i];
      r.n = s->sizes[i];
      if (st[2 * i] == ~0ull) {
        r.start_us = r.end_us = r.latency_us = 0.0;
        continue;
      }
      r.start_us = (st[2 * i] - t0) * us_per_tick;
      r.end_us = (st[2 * i + 1] - t0) * us_per_tick;
      r.latency_us = r.end_us - r.start_us;
    }
  }
  return XS_OK;
}

xs_status xs_stream_params(xs_stream_t s, xs_params* out) {
  clear_error();
  if (!s || !out) return fail(XS_EINVAL, "stream and out must not be NULL");
  *out = s->params;
  return XS_OK;
}

xs_status xs_stream_destroy(xs_stream_t s) {
  clear_error();
  if (!s) return XS_OK;
  if (s->pending) (void)hipEventSynchronize(s->done);
  stream_release(s);
  return XS_OK;
}

}  // extern "C"
