// A toy event loop around the lookup (xs_event_run).
//
// The paper's application keeps a buffer of particles in flight and runs one
// kernel per event over it; particles that finish are replaced from the
// source until every history has run (section 5.1: particles in flight,
// queued versus queueless event logic, the sorting threshold).  This loop
// reproduces that shape with the lookup as its one real event: each
// iteration looks up the macroscopic values of the live slots
// (xs_lookup_active, so the queue mode and sort policy apply), then one
// kernel collides every live particle and refills dead slots with new
// histories.
//
// The collision is deliberately simple and uses only +, -, *, and compares
// in FP64, so its results are exactly reproducible:
//   absorbed             if u0 * (S0 + S1) < 0.25 * S1
//   else E' = E * (0.2 + 0.8 * u1); the history ends if E' < e_cut
//   else the particle may enter another material: if u2 < 0.2,
//        m' = min(floor((u2 * 5) * M), M - 1)
// with S0, S1 the first two looked-up channels (FP32 values widened) and
// u0..u2 uniform numbers that depend only on (seed, history, collision):
// SplitMix64 (Steele, Lea & Flood 2014) evaluated at counter
// history * 2^20 + collision * 4 + draw.  A history's outcome therefore does
// not depend on which slot or iteration ran it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kEventThreads = 256;
constexpr int64_t kCollisionLimit = (1 << 18) - 1;  // counter field width

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// Draw `i` of collision `c` of history `h`, uniform on [0, 1).
__device__ __forceinline__ double draw(uint64_t seed, int64_t h, int64_t c,
                                       int i) {
  const uint64_t ctr = ((uint64_t)h << 20) + ((uint64_t)c << 2) + (uint64_t)i;
  const uint64_t x = mix64(seed + (ctr + 1) * 0x9E3779B97F4A7C15ull);
  return (double)(x >> 11) * 0x1.0p-53;
}

struct EventDev {
  int64_t n_slots, n_hist;
  uint64_t seed;
  double e_cut;
  int32_t M;
  double* E;
  int32_t* mat;
  uint8_t* alive;
  int64_t* hist;
  int32_t* ncoll;
  const void* sigma;
  // [0] next history to start, [1] histories finished, [2] lookups run
  unsigned long long* counters;
  int32_t* t_coll;
  double* t_energy;
  uint8_t* t_fate;
};

__device__ __forceinline__ void source(const EventDev& d, int64_t slot,
                                       int64_t h) {
  const double u0 = draw(d.seed, h, 0, 0), u1 = draw(d.seed, h, 0, 1);
  d.E[slot] = 0.01 + 0.99 * u0;
  d.mat[slot] = min((int)(u1 * (double)d.M), d.M - 1);
  d.hist[slot] = h;
  d.ncoll[slot] = 0;
  d.alive[slot] = 1;
}

__global__ __launch_bounds__(kEventThreads) void k_event_start(EventDev d) {
  const int64_t i = (int64_t)blockIdx.x * kEventThreads + threadIdx.x;
  if (i == 0) {
    d.counters[0] = (unsigned long long)min(d.n_slots, d.n_hist);
    d.counters[1] = 0;
    d.counters[2] = 0;
  }
  if (i >= d.n_slots) return;
  if (i < d.n_hist) source(d, i, i);
  else d.alive[i] = 0;
}

template <class T>
__global__ __launch_bounds__(kEventThreads) void k_event_advance(EventDev d) {
  const int64_t i = (int64_t)blockIdx.x * kEventThreads + threadIdx.x;
  const bool in = i < d.n_slots;
  bool was_alive = in && d.alive[i];
  bool finished = false;
  if (was_alive) {
    const T* sg = (const T*)d.sigma + i * XS_CHANNELS;
    const double s0 = (double)sg[0], s1 = (double)sg[1];
    const int64_t h = d.hist[i];
    const int64_t c = (int64_t)d.ncoll[i] + 1;
    const double u0 = draw(d.seed, h, c, 0), u1 = draw(d.seed, h, c, 1),
                 u2 = draw(d.seed, h, c, 2);
    const double e = d.E[i];
    int fate = 0;
    double e_out = e;
    if (u0 * (s0 + s1) < 0.25 * s1) {
      fate = 1;  // absorbed
    } else {
      e_out = e * (0.2 + 0.8 * u1);
      if (e_out < d.e_cut) fate = 2;           // below the energy cut-off
      else if (c >= kCollisionLimit) fate = 3;  // collision limit
    }
    if (fate) {
      d.t_coll[h] = (int32_t)c;
      d.t_energy[h] = e_out;
      d.t_fate[h] = (uint8_t)fate;
      d.alive[i] = 0;
      finished = true;
    } else {
      d.E[i] = e_out;
      if (u2 < 0.2) d.mat[i] = min((int)((u2 * 5.0) * (double)d.M), d.M - 1);
      d.ncoll[i] = (int32_t)c;
    }
  }
  // Wave-aggregated counts: lookups run this iteration, histories finished.
  const uint64_t looked = __ballot(was_alive), done = __ballot(finished);
  if ((threadIdx.x & 63) == 0) {
    if (looked) atomicAdd(&d.counters[2], (unsigned long long)__popcll(looked));
    if (done) atomicAdd(&d.counters[1], (unsigned long long)__popcll(done));
  }
  // Refill: a dead slot claims the next history while any is left.
  if (in && !d.alive[i] &&
      __hip_atomic_load(&d.counters[0], __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_AGENT) < (unsigned long long)d.n_hist) {
    const unsigned long long h = atomicAdd(&d.counters[0], 1ull);
    if (h < (unsigned long long)d.n_hist) source(d, i, (int64_t)h);
  }
}

}  // namespace
}  // namespace xs

using namespace xs;

extern "C" {

xs_status xs_event_workspace_size(xs_tables_t h, const xs_event_config* cfg,
                                  const xs_params* params, size_t* bytes) {
  clear_error();
  if (!h || !cfg || !bytes) return fail(XS_EINVAL, "a pointer is NULL");
  if (cfg->n_slots < 1) return fail(XS_EINVAL, "n_slots must be >= 1");
  return xs_workspace_size(h, cfg->n_slots, params, bytes);
}

xs_status xs_event_run(xs_tables_t h, const xs_event_config* cfg,
                       const xs_event_buffers* b, const xs_params* params,
                       void* d_ws, size_t ws_bytes, void* stream,
                       xs_event_result* result) {
  clear_error();
  if (!h || !cfg || !b || !result)
    return fail(XS_EINVAL, "tables, config, buffers and result are needed");
  if (cfg->n_slots < 1 || cfg->n_slots > 0x7fffffffLL)
    return fail(XS_EINVAL, "n_slots must be in [1, 2^31)");
  if (cfg->n_histories < 0 || cfg->n_histories > (int64_t(1) << 40))
    return fail(XS_EINVAL, "n_histories must be in [0, 2^40]");
  if (!(cfg->e_cut > 0.0)) return fail(XS_EINVAL, "e_cut must be > 0");
  if (cfg->check_every < 1 || cfg->max_iterations < 1)
    return fail(XS_EINVAL, "check_every and max_iterations must be >= 1");
  if (!b->E || !b->mat || !b->alive || !b->hist || !b->ncoll || !b->sigma ||
      !b->counters || (cfg->n_histories > 0 &&
                       (!b->t_collisions || !b->t_energy || !b->t_fate)))
    return fail(XS_EINVAL, "a buffer is NULL");
  xs_params p;
  // resolved as xs_lookup_active (which runs the lookups) resolves them
  if (xs_status st = resolve_for(h, cfg->n_slots, 1, params, &p)) return st;
  hipStream_t s = (hipStream_t)stream;

  EventDev d{};
  d.n_slots = cfg->n_slots;
  d.n_hist = cfg->n_histories;
  d.seed = cfg->seed;
  d.e_cut = cfg->e_cut;
  d.M = h->d.M;
  d.E = b->E;
  d.mat = b->mat;
  d.alive = b->alive;
  d.hist = b->hist;
  d.ncoll = b->ncoll;
  d.sigma = b->sigma;
  d.counters = (unsigned long long*)b->counters;
  d.t_coll = b->t_collisions;
  d.t_energy = b->t_energy;
  d.t_fate = b->t_fate;
  const dim3 grid((unsigned)((cfg->n_slots + kEventThreads - 1) / kEventThreads));
  const dim3 block(kEventThreads);

  hipLaunchKernelGGL(k_event_start, grid, block, 0, s, d);
  XS_HIP(hipGetLastError());
  int64_t it = 0;
  unsigned long long cnt[3] = {0, 0, 0};
  bool complete = cfg->n_histories == 0;
  while (!complete && it < cfg->max_iterations) {
    if (xs_status st = xs_lookup_active(h, cfg->n_slots, b->E, b->mat, b->alive,
                                        b->sigma, &p, d_ws, ws_bytes, stream))
      return st;
    if (p.precision == XS_FP64)
      hipLaunchKernelGGL(k_event_advance<double>, grid, block, 0, s, d);
    else
      hipLaunchKernelGGL(k_event_advance<float>, grid, block, 0, s, d);
    XS_HIP(hipGetLastError());
    ++it;
    if (it % cfg->check_every == 0 || it == cfg->max_iterations) {
      XS_HIP(hipMemcpyAsync(cnt, d.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
      XS_HIP(hipStreamSynchronize(s));
      complete = (int64_t)cnt[1] >= cfg->n_histories;
    }
  }
  XS_HIP(hipMemcpyAsync(cnt, d.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  XS_HIP(hipStreamSynchronize(s));
  result->iterations = it;
  result->histories = (int64_t)cnt[1];
  result->lookups = (int64_t)cnt[2];
  if ((int64_t)cnt[1] < cfg->n_histories)
    return fail(XS_ETIMEOUT, "%lld of %lld histories finished after %lld "
                "iterations", (long long)cnt[1], (long long)cfg->n_histories,
                (long long)it);
  return XS_OK;
}

}  // extern "C"
