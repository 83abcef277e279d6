// C entry points of libxs: argument and table validation, table packing and
// upload, parameter resolution, the lookup pipeline (optional sort or
// compaction, then the lookup kernel) and per-stage event timing.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>

#include "xs_internal.h"

namespace xs {

namespace {
thread_local char g_error[512] = "";
}

xs_status fail(xs_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_error[0] = '\0'; }

namespace {

int ceil_log2(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

int64_t double_bits(double x) {
  int64_t b;
  std::memcpy(&b, &x, sizeof(b));
  return b;
}

// 64-bit digest of a table description: every array, the build flags and
// the hash-bin counts, in 8-byte words (a multiply-rotate mix per word, then
// a final avalanche; Stafford's variant 13 of the MurmurHash3 finaliser).
struct Digest {
  uint64_t h = 0x243F6A8885A308D3ull;
  void word(uint64_t w) {
    h ^= w * 0x9E3779B97F4A7C15ull;
    h = (h << 27 | h >> 37) * 0xC2B2AE3D27D4EB4Full + 0x165667B19E3779F9ull;
  }
  void bytes(const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
      uint64_t w;
      std::memcpy(&w, c + i, 8);
      word(w);
    }
    uint64_t w = 0;
    std::memcpy(&w, c + i, n - i);
    word(w ^ ((uint64_t)(n - i) << 56));
    word(n);
  }
  uint64_t done() const {
    uint64_t z = h;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

uint64_t table_checksum(const xs_table_desc* d) {
  Digest g;
  const int K = d->n_nuclides, M = d->n_materials;
  const int64_t P = d->grid_offsets[K];
  const int32_t L = d->mat_offsets[M];
  g.word((uint64_t)K);
  g.word((uint64_t)M);
  g.bytes(d->grid_offsets, sizeof(int64_t) * (K + 1));
  g.bytes(d->energy, sizeof(double) * P);
  g.bytes(d->xs, sizeof(double) * P * XS_CHANNELS);
  g.bytes(d->mat_offsets, sizeof(int32_t) * (M + 1));
  g.bytes(d->mat_nuclides, sizeof(int32_t) * L);
  g.bytes(d->mat_density, sizeof(double) * L);
  g.word(d->build_flags);
  if (d->build_flags & XS_BUILD_HASH) {
    g.word((uint64_t)d->n_hash_bins);
    for (int i = 0; i < d->n_extra_hash_grids; ++i)
      g.word((uint64_t)d->extra_hash_bins[i]);
  }
  return g.done();
}

// Frees what a partially built handle holds.
void release(xs_tables_s* h) {
  for (void* p : h->allocations) (void)hipFree(p);
  h->allocations.clear();
  for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
  h->event_pool.clear();
  for (auto& c : h->prof)
    for (hipEvent_t e : c.ev) (void)hipEventDestroy(e);
  h->prof.clear();
  if (h->req_event) {
    (void)hipEventSynchronize(h->req_event);
    (void)hipEventDestroy(h->req_event);
    h->req_event = nullptr;
  }
  if (h->req_stage) (void)hipHostFree(h->req_stage);
  h->req_stage = nullptr;
}

template <class T>
xs_status upload(xs_tables_s* h, const T* src, size_t count, T** dst,
                 hipStream_t s) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(T), 1);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess)
    return fail(XS_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes,
                hipGetErrorString(e));
  h->allocations.push_back(p);
  if (count) XS_HIP(hipMemcpyAsync(p, src, count * sizeof(T),
                                   hipMemcpyHostToDevice, s));
  *dst = (T*)p;
  return XS_OK;
}

xs_status alloc_dev(xs_tables_s* h, size_t bytes, void** dst) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 1));
  if (e != hipSuccess)
    return fail(XS_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes,
                hipGetErrorString(e));
  h->allocations.push_back(p);
  *dst = p;
  return XS_OK;
}

// The FP32 form keeps a relative error bound only while every channel value
// and density is zero or rounds to a normal, finite FP32 number: larger ones
// would become infinite, smaller ones subnormal or zero.
bool fp32_normal_or_zero(double x) {
  if (x == 0.0) return true;
  const float f = (float)x;
  return std::isfinite(f) && std::fabs(f) >= FLT_MIN;
}

// Host-only checks of a table description (no HIP call).
xs_status validate_desc(const xs_table_desc* d) {
  if (!d) return fail(XS_EINVAL, "desc is NULL");
  if (d->n_nuclides < 1) return fail(XS_ETABLE, "n_nuclides must be >= 1");
  if (d->n_channels != XS_CHANNELS)
    return fail(XS_ETABLE, "n_channels must be %d", XS_CHANNELS);
  if (!d->grid_offsets || !d->energy || !d->xs)
    return fail(XS_EINVAL, "grid arrays must not be NULL");
  if (d->n_materials < 1 || d->n_materials > 65536)
    return fail(XS_ETABLE, "n_materials must be in [1, 65536]");
  if (!d->mat_offsets || !d->mat_nuclides || !d->mat_density)
    return fail(XS_EINVAL, "material arrays must not be NULL");
  if (d->build_flags & ~(XS_BUILD_FP32 | XS_BUILD_HASH | XS_BUILD_UNIONIZED |
                         XS_BUILD_UNION_BY_MATERIAL | XS_BUILD_FP32_PAIRS))
    return fail(XS_EINVAL, "unknown build flag bits 0x%x", d->build_flags);
  if ((d->build_flags & XS_BUILD_UNION_BY_MATERIAL) &&
      !(d->build_flags & XS_BUILD_UNIONIZED))
    return fail(XS_EINVAL, "XS_BUILD_UNION_BY_MATERIAL needs XS_BUILD_UNIONIZED");
  if ((d->build_flags & XS_BUILD_FP32_PAIRS) && !(d->build_flags & XS_BUILD_FP32))
    return fail(XS_EINVAL, "XS_BUILD_FP32_PAIRS needs XS_BUILD_FP32");
  if ((d->build_flags & XS_BUILD_HASH) &&
      (d->n_hash_bins < 1 || d->n_hash_bins > 100000))
    return fail(XS_EINVAL, "n_hash_bins must be in [1, 100000]");
  if (d->n_extra_hash_grids != 0) {
    if (!(d->build_flags & XS_BUILD_HASH))
      return fail(XS_EINVAL, "extra hash grids need XS_BUILD_HASH");
    if (d->n_extra_hash_grids < 0 ||
        d->n_extra_hash_grids > XS_MAX_HASH_GRIDS - 1)
      return fail(XS_EINVAL, "n_extra_hash_grids must be in [0, %d]",
                  XS_MAX_HASH_GRIDS - 1);
    if (!d->extra_hash_bins)
      return fail(XS_EINVAL, "extra_hash_bins is NULL");
    for (int i = 0; i < d->n_extra_hash_grids; ++i) {
      const int32_t b = d->extra_hash_bins[i];
      if (b < 1 || b > 100000)
        return fail(XS_EINVAL, "extra_hash_bins[%d] = %d not in [1, 100000]",
                    i, b);
      if (b == d->n_hash_bins)
        return fail(XS_EINVAL, "extra_hash_bins[%d] repeats n_hash_bins", i);
      for (int j = 0; j < i; ++j)
        if (d->extra_hash_bins[j] == b)
          return fail(XS_EINVAL, "extra_hash_bins lists %d twice", b);
    }
  }

  const int K = d->n_nuclides;
  const bool fp32 = (d->build_flags & XS_BUILD_FP32) != 0;
  if (d->grid_offsets[0] != 0) return fail(XS_ETABLE, "grid_offsets[0] != 0");
  for (int k = 0; k < K; ++k) {
    const int64_t a = d->grid_offsets[k], b = d->grid_offsets[k + 1];
    if (b - a < 2)
      return fail(XS_ETABLE, "nuclide %d has %lld grid points (needs >= 2)", k,
                  (long long)(b - a));
    if (b >= (int64_t)0x7fffffff)
      return fail(XS_ETABLE, "more than 2^31-2 grid points in total");
    for (int64_t p = a; p < b; ++p) {
      const double e = d->energy[p];
      // [2^-400, 2^400] keeps every bracket's fraction inside the range the
      // kernels' division handles without rescaling.
      if (!(e >= 0x1p-400 && e <= 0x1p400))
        return fail(XS_ETABLE, "nuclide %d point %lld: energy %g outside "
                    "[2^-400, 2^400]", k, (long long)(p - a), e);
      if (p > a && !(d->energy[p - 1] < e))
        return fail(XS_ETABLE, "nuclide %d: energies not strictly increasing "
                    "at point %lld", k, (long long)(p - a));
      if (fp32 && p > a && !fp32_normal_or_zero(1.0 / (e - d->energy[p - 1])))
        return fail(XS_ETABLE, "nuclide %d point %lld: the spacing %g of its "
                    "energies has no normal FP32 reciprocal (XS_BUILD_FP32 "
                    "needs spacings between about 3e-39 and 8e37)", k,
                    (long long)(p - a), e - d->energy[p - 1]);
      for (int c = 0; c < XS_CHANNELS; ++c) {
        const double x = d->xs[p * XS_CHANNELS + c];
        if (!std::isfinite(x) || x < 0.0)
          return fail(XS_ETABLE, "nuclide %d point %lld channel %d: value %g "
                      "not finite and >= 0", k, (long long)(p - a), c, x);
        if (fp32 && !fp32_normal_or_zero(x))
          return fail(XS_ETABLE, "nuclide %d point %lld channel %d: value %g "
                      "does not round to a normal FP32 number or zero "
                      "(XS_BUILD_FP32)", k, (long long)(p - a), c, x);
      }
    }
  }
  const int M = d->n_materials;
  if (d->mat_offsets[0] != 0) return fail(XS_ETABLE, "mat_offsets[0] != 0");
  std::vector<int32_t> seen(K, -1);
  for (int m = 0; m < M; ++m) {
    const int32_t a = d->mat_offsets[m], b = d->mat_offsets[m + 1];
    if (b - a < 1) return fail(XS_ETABLE, "material %d is empty", m);
    for (int32_t j = a; j < b; ++j) {
      const int32_t k = d->mat_nuclides[j];
      if (k < 0 || k >= K)
        return fail(XS_ETABLE, "material %d: nuclide id %d out of range", m, k);
      if (seen[k] == m)
        return fail(XS_ETABLE, "material %d lists nuclide %d twice", m, k);
      seen[k] = m;
      const double r = d->mat_density[j];
      if (!std::isfinite(r) || !(r > 0.0))
        return fail(XS_ETABLE, "material %d: density %g not finite and > 0", m,
                    r);
      if (fp32 && !fp32_normal_or_zero(r))
        return fail(XS_ETABLE, "material %d: density %g does not round to a "
                    "normal FP32 number (XS_BUILD_FP32)", m, r);
    }
  }
  return XS_OK;
}

xs_status check_handle(xs_tables_t h) {
  if (!h) return fail(XS_EINVAL, "table handle is NULL");
  return XS_OK;
}

const xs_params* nearest_tuned(const xs_tables_s* h, int active, int prec,
                               int64_t n) {
  const int want = size_class(n);
  int best = -1, dist = 1 << 30;
  for (int b = 0; b < kBuckets; ++b) {
    if (!h->tuned_valid[active][prec][b]) continue;
    const int dd = std::abs(b - want);
    if (dd < dist) {
      dist = dd;
      best = b;
    }
  }
  return best < 0 ? nullptr : &h->tuned[active][prec][best];
}

bool hash_built(const xs_tables_s* h, int32_t bins) {
  for (const HashGrid& g : h->hash)
    if (g.B == bins) return true;
  return false;
}

xs_status resolve(xs_tables_s* h, int64_t n, const xs_params* in,
                  xs_params* out, int active = 0) {
  xs_params p;
  if (in) {
    p = *in;
  } else {
    xs_params_default(&p, XS_FP64);
  }
  if (p.precision != XS_FP64 && p.precision != XS_FP32)
    return fail(XS_EINVAL, "precision must be XS_FP64 or XS_FP32");
  if (p.precision == XS_FP32 && !h->d.rec32)
    return fail(XS_ENOTBUILT, "FP32 tables were not built (XS_BUILD_FP32)");

  xs_params t;
  bool have_tuned = false;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    const xs_params* tp = nearest_tuned(h, active, p.precision, n);
    if (tp) {
      t = *tp;
      have_tuned = true;
    }
  }
  if (!have_tuned) untuned_defaults(h, n, p.precision, &t);
  if (p.grid == XS_AUTO) p.grid = t.grid;
  if (p.sort == XS_AUTO) p.sort = t.sort;
  if (p.block_size == 0 || p.block_size == XS_AUTO) p.block_size = t.block_size;
  if (p.lookups_per_thread == 0 || p.lookups_per_thread == XS_AUTO)
    p.lookups_per_thread = t.lookups_per_thread;
  if (p.lds_stage == XS_AUTO) {
    // only where the fields set explicitly allow it
    const bool fits = p.lookups_per_thread <= 2 &&
                      (p.unroll == 0 || p.unroll == XS_AUTO || p.unroll == 1) &&
                      p.block_size <= 1024 / p.lookups_per_thread &&
                      p.wave_per_lookup != 1;
    p.lds_stage = fits ? t.lds_stage : 0;
  }
  if (p.wave_per_lookup == XS_AUTO) {
    // only where the fields set explicitly allow it
    const bool fits = p.lookups_per_thread == 1 && p.lds_stage == 0 &&
                      (p.unroll == 0 || p.unroll == XS_AUTO || p.unroll == 1) &&
                      p.block_size <= 256;
    p.wave_per_lookup = fits ? t.wave_per_lookup : 0;
  }
  if (p.sort_threshold < 0) p.sort_threshold = t.sort_threshold;
  if (p.queue == XS_AUTO) p.queue = t.queue;
  if (p.unroll == 0 || p.unroll == XS_AUTO) {
    // the tuned depth when it applies and the block leaves room for it
    const int u = (p.lookups_per_thread <= 2 && p.lds_stage == 0 &&
                   p.wave_per_lookup != 1) ? t.unroll : 1;
    const int w = p.lookups_per_thread * u;
    const int max_block = w <= 1 ? 1024 : (w <= 4 ? 512 : 256);
    p.unroll = p.block_size <= max_block ? u : 1;
  }

  if (p.grid < 0 || p.grid > 2) return fail(XS_EINVAL, "unknown grid %d", p.grid);
  if (p.grid == XS_GRID_HASH && h->d.B == 0)
    return fail(XS_ENOTBUILT, "hash grid was not built (XS_BUILD_HASH)");
  // hash_bins is conditional on the hash grid: automatic means the tuned
  // grid when the tuned entry searches a hash grid that was built, else the
  // default one; other grid methods carry 0.
  if (p.grid != XS_GRID_HASH) {
    p.hash_bins = 0;
  } else {
    if (p.hash_bins == 0 || p.hash_bins == XS_AUTO)
      p.hash_bins = (t.grid == XS_GRID_HASH && hash_built(h, t.hash_bins))
                        ? t.hash_bins : h->d.B;
    if (!hash_built(h, p.hash_bins))
      return fail(XS_ENOTBUILT, "no hash grid of %d bins was built",
                  p.hash_bins);
  }
  if (p.grid == XS_GRID_UNIONIZED && h->d.U == 0)
    return fail(XS_ENOTBUILT, "unionized grid was not built (XS_BUILD_UNIONIZED)");
  if (p.sort < 0 || p.sort > 4) return fail(XS_EINVAL, "unknown sort %d", p.sort);
  if (p.block_size < 64 || p.block_size > 1024 || p.block_size % 64)
    return fail(XS_EINVAL, "block_size %d not in 64..1024 step 64", p.block_size);
  if (p.lookups_per_thread < 1 || p.lookups_per_thread > 8)
    return fail(XS_EINVAL, "lookups_per_thread %d not in 1..8",
                p.lookups_per_thread);
  if (p.lds_stage < 0 || p.lds_stage > 3)
    return fail(XS_EINVAL, "lds_stage must be 0 (off) or a stage shape 1..3");
  if (p.lds_stage > 0 && (p.lookups_per_thread > 2 || p.unroll != 1))
    return fail(XS_EINVAL, "lds_stage > 0 runs one or two lookups per lane "
                "with one nuclide in flight (lookups_per_thread <= 2, "
                "unroll = 1)");
  if (p.wave_per_lookup != 0 && p.wave_per_lookup != 1)
    return fail(XS_EINVAL, "wave_per_lookup must be 0 or 1");
  if (p.wave_per_lookup == 1 &&
      (p.lookups_per_thread != 1 || p.unroll != 1 || p.lds_stage != 0 ||
       p.block_size > 256))
    return fail(XS_EINVAL, "wave_per_lookup = 1 needs lookups_per_thread = "
                "unroll = 1, lds_stage = 0 and block_size <= 256");
  if (p.queue != XS_QUEUE_COMPACT && p.queue != XS_QUEUE_PREDICATED)
    return fail(XS_EINVAL, "unknown queue mode %d", p.queue);
  if (p.unroll != 1 && p.unroll != 2 && p.unroll != 4)
    return fail(XS_EINVAL, "unroll %d not 1, 2 or 4", p.unroll);
  if (p.unroll > 1 && p.lookups_per_thread > 2)
    return fail(XS_EINVAL, "unroll %d needs lookups_per_thread <= 2",
                p.unroll);
  {
    const int w = p.lookups_per_thread * p.unroll;
    const int max_block = p.lds_stage > 0
                              ? 1024 / p.lookups_per_thread
                              : (w <= 1 ? 1024 : (w <= 4 ? 512 : 256));
    if (p.block_size > max_block)
      return fail(XS_EINVAL, "block_size %d too large for %d lookups per lane "
                  "x %d nuclides in flight (max %d)", p.block_size,
                  p.lookups_per_thread, p.unroll, max_block);
  }
  *out = p;
  return XS_OK;
}

SortKey make_sort_key(const xs_tables_s* h, int sort, bool flag, int64_t n) {
  SortKey k{};
  k.M = h->d.M;
  k.flag_bit = flag ? 1 : 0;
  const int mb = ceil_log2(h->d.M);
  switch (sort) {
    case XS_SORT_BAND_MATERIAL: {
      // About 4096 to 8192 lookups per (band, material) group: whole blocks
      // stay in one material (a block that straddles two groups takes the
      // slower per-lane walk), and the bands are still fine enough that the
      // lookups in flight on an XCD span a narrow energy range.  Measured
      // against groups of ~1024: 4-7 % faster sorted lookups from 1e6 to
      // 1e7 lookups; against ~16384: faster below 1e7.
      int bb = 0;
      while (bb < 12 && (n >> (bb + 1)) >= (int64_t)h->d.M * 4096) ++bb;
      k.band_bits = bb;
      k.mat_bits = mb;
      k.e_bits = 24 - mb - k.flag_bit;
      if (k.e_bits < bb + 1) k.e_bits = 32 - mb - k.flag_bit;
      break;
    }
    case XS_SORT_MATERIAL:
      k.mat_bits = std::max(mb, 1);
      k.e_bits = 0;
      break;
    case XS_SORT_ENERGY:
      k.mat_bits = 0;
      k.e_bits = 16 - k.flag_bit;
      break;
    default: {
      k.mat_bits = mb;
      const int target = mb + k.flag_bit + 8 <= 16 ? 16 : 32;
      k.e_bits = target - mb - k.flag_bit;
      break;
    }
  }
  k.e_bits_min = double_bits(h->info.e_min);
  if (k.e_bits > 0) {
    const int64_t span = double_bits(h->info.e_max) - k.e_bits_min;
    int s = 0;
    while ((span >> s) >= (int64_t(1) << k.e_bits)) ++s;
    k.e_shift = s;
  }
  k.total_bits = k.mat_bits + k.e_bits + k.flag_bit;
  return k;
}

hipEvent_t take_event(xs_tables_s* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Debug mode: counts the call's invalid queries, waits for the stream and
// fails with their number and the first position.
xs_status debug_check(xs_tables_s* h, int64_t n, const double* E,
                      const int32_t* mat, const uint8_t* active,
                      hipStream_t s) {
  XS_HIP(launch_debug_count(n, E, mat, active, h->d.M, h->dbg_dev, s));
  unsigned long long c[kDbgWords];
  XS_HIP(hipMemcpyAsync(c, h->dbg_dev, sizeof(c), hipMemcpyDeviceToHost, s));
  XS_HIP(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> lk(h->mu);
    ++h->dbg_calls;
  }
  if (c[kDbgCallInvalid])
    return fail(XS_EINVAL, "%llu of %lld queries are invalid (first at %llu): "
                "energies must be finite and > 0, materials in [0, %d)",
                c[kDbgCallInvalid], (long long)n, c[kDbgCallFirst], h->d.M);
  return XS_OK;
}

xs_status lookup_common(xs_tables_t h, int64_t n, const double* E,
                        const int32_t* mat, const uint8_t* active, bool masked,
                        void* out, const xs_params* params, void* ws,
                        size_t ws_bytes, void* stream, bool no_alloc = false) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (n < 0) return fail(XS_EINVAL, "n must be >= 0");
  if (n > 0x7fffffffLL) return fail(XS_EINVAL, "n must be < 2^31");
  xs_params p;
  if (xs_status st = resolve(h, n, params, &p, masked ? 1 : 0)) return st;
  if (n == 0) return XS_OK;
  if (!E || !mat || !out) return fail(XS_EINVAL, "query or output pointer is NULL");
  if (masked && !active) return fail(XS_EINVAL, "active mask is NULL");
  int dev = -1;
  XS_HIP(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(XS_EINVAL, "current device %d is not the tables' device %d",
                dev, h->device);

  const bool do_sort = p.sort != XS_SORT_NONE && n >= p.sort_threshold;
  const bool compact = masked && !do_sort && p.queue == XS_QUEUE_COMPACT;
  const SortKey key = do_sort ? make_sort_key(h, p.sort, masked, n) : SortKey{};
  const size_t need = do_sort   ? sort_workspace_bytes(n, key.total_bits)
                      : compact ? compact_workspace_bytes(n)
                                : 0;
  if (need > 0) {
    if (!ws || ws_bytes < need)
      return fail(XS_EWORKSPACE, "workspace of %zu bytes needed, %zu given",
                  need, ws ? ws_bytes : (size_t)0);
    if ((uintptr_t)ws % 256)
      return fail(XS_EWORKSPACE, "workspace must be 256-byte aligned");
  }
  hipStream_t s = (hipStream_t)stream;

  ProfCall pc{};
  // Profiling takes (and may create) HIP events, so calls that must not
  // allocate are not recorded.
  const bool prof = h->profiling && !no_alloc;
  if (prof) {
    std::lock_guard<std::mutex> lk(h->mu);
    for (auto& e : pc.ev) {
      e = take_event(h);
      if (!e) return fail(XS_EHIP, "hipEventCreate failed");
    }
    pc.sorted = do_sort || compact;
    pc.n = n;
  }
  if (prof) XS_HIP(hipEventRecord(pc.ev[0], s));

  LookupArgs a{n, E, mat, nullptr, nullptr, masked ? active : nullptr, out};
  if (do_sort) {
    // The LDS-staged kernel over a key with the material in it gets block
    // ranges cut at every group of the key (bits above the energy rest), so
    // no block holds two materials; when the key has few enough groups
    // (at most one per four blocks) and the batch is not tiny.  Only for
    // the narrow-window stage shapes (1, 2; dense batches): with the wide
    // windows of shape 3 the per-lane walk of the few straddling blocks
    // costs less than finding the groups (measured from 5e5 to 2e6).
    const int rest = key.e_bits - key.band_bits;
    const int group_bits = key.total_bits - rest;
    const int64_t per_block = (int64_t)p.block_size * p.lookups_per_thread;
    const int64_t nb = (n + per_block - 1) / per_block;
    const bool cut = p.lds_stage > 0 && p.lds_stage <= 2 && key.mat_bits > 0 &&
                     p.sort != XS_SORT_ENERGY && n >= 4096 &&
                     group_bits < 31 &&
                     ((int64_t)1 << group_bits) <= std::max<int64_t>(1, nb / 4);
    // With a mask the inactive lookups sort last (the key's top bit): the
    // kernels serve only the active head of the queue, as blocks cut from
    // the groups without the flag or as a device-side count.
    const uint32_t* keys = nullptr;
    uint32_t* spare = nullptr;
    const int64_t groups = (int64_t)1 << group_bits;
    XS_HIP(launch_sort(key, n, E, mat, masked ? active : nullptr, ws, &a.perm,
                       cut ? &keys : nullptr, &spare,
                       masked && !cut ? &a.count_dev : nullptr, s));
    if (cut)
      XS_HIP(launch_block_ranges(keys, n, rest, groups,
                                 key.flag_bit ? groups >> 1 : groups,
                                 per_block, spare, &a, s));
  } else if (compact) {
    XS_HIP(launch_compact(n, active, ws, &a.perm, &a.count_dev, s));
    a.active = nullptr;
  }
  if (prof) XS_HIP(hipEventRecord(pc.ev[1], s));
  hipError_t e;
  const DevTables d = tables_for(h, p);
  switch (p.grid) {
    case XS_GRID_NUCLIDE: e = launch_lookup_nuclide(d, p, a, s); break;
    case XS_GRID_HASH: e = launch_lookup_hash(d, p, a, s); break;
    default: e = launch_lookup_union(d, p, a, s); break;
  }
  if (e != hipSuccess)
    return fail(XS_EHIP, "lookup kernel launch failed: %s", hipGetErrorString(e));
  if (prof) {
    XS_HIP(hipEventRecord(pc.ev[2], s));
    std::lock_guard<std::mutex> lk(h->mu);
    h->prof.push_back(pc);
  }
  if (h->d.dbg)
    return debug_check(h, n, E, mat, masked ? active : nullptr, s);
  return XS_OK;
}

}  // namespace

int size_class(int64_t n) {
  return n > 1 ? 63 - __builtin_clzll((unsigned long long)n) : 0;
}

xs_status resolve_for(xs_tables_s* h, int64_t n, int active,
                      const xs_params* in, xs_params* out) {
  return resolve(h, n, in, out, active);
}

DevTables tables_for(const xs_tables_s* h, const xs_params& p) {
  DevTables d = h->d;
  if (p.grid == XS_GRID_HASH)
    for (const HashGrid& g : h->hash)
      if (g.B == p.hash_bins) {
        d.B = g.B;
        d.inv_dln = g.inv_dln;
        d.H = g.H;
      }
  return d;
}

xs_status lookup_batch_into(xs_tables_t h, int64_t n, const double* E,
                            const int32_t* mat, void* out,
                            const xs_params* params, void* ws, size_t ws_bytes,
                            void* stream) {
  return lookup_common(h, n, E, mat, nullptr, false, out, params, ws, ws_bytes,
                       stream, true);
}

// Untuned batches smaller than one query per lane of the chip (256 compute
// units x 1024 lanes) default to one wave per query.
constexpr int64_t kWaveDefaultBelow = 256 * 1024;

void untuned_defaults(const xs_tables_s* h, int64_t n, int precision,
                      xs_params* out) {
  // The shapes the tuner picks on the full-size workload: the union grid
  // (else the hash grid, else bisection), the banded sort at the paper's
  // threshold, 128-lane blocks staging windows in LDS, with wider windows
  // for sparser batches (shape 3 below 1.5M lookups, 2 below 3M, 1 above).
  xs_params t{};
  t.precision = precision;
  t.grid = h->d.U > 0 ? XS_GRID_UNIONIZED
                      : (h->d.B > 0 ? XS_GRID_HASH : XS_GRID_NUCLIDE);
  t.sort = XS_SORT_BAND_MATERIAL;
  t.block_size = 128;
  t.lookups_per_thread = 1;
  t.lds_stage = n < 1500000 ? 3 : (n < 3000000 ? 2 : 1);
  t.sort_threshold = 20000;
  t.queue = XS_QUEUE_COMPACT;
  t.unroll = 1;
  t.wave_per_lookup = 0;
  t.hash_bins = t.grid == XS_GRID_HASH ? h->d.B : 0;
  if (n < kWaveDefaultBelow) {
    // Too few queries to give every lane of the chip one: a wave per
    // query, unsorted.
    t.sort = XS_SORT_NONE;
    t.lds_stage = 0;
    t.wave_per_lookup = 1;
  }
  *out = t;
}

}  // namespace xs

using namespace xs;

extern "C" {

xs_status xs_create_tables(const xs_table_desc* desc, void* stream,
                           xs_tables_t* out) {
  clear_error();
  if (!out) return fail(XS_EINVAL, "out is NULL");
  if (xs_status st = validate_desc(desc)) return st;
  const int K = desc->n_nuclides, M = desc->n_materials;
  const int64_t P = desc->grid_offsets[K];
  const int32_t L = desc->mat_offsets[M];
  hipStream_t s = (hipStream_t)stream;

  auto* h = new (std::nothrow) xs_tables_s();
  if (!h) return fail(XS_ENOMEM, "host allocation failed");
  auto cleanup = [&](xs_status st) {
    if (s) (void)hipStreamSynchronize(s); else (void)hipDeviceSynchronize();
    release(h);
    delete h;
    return st;
  };
  if (hipGetDevice(&h->device) != hipSuccess)
    return cleanup(fail(XS_EHIP, "no HIP device available"));

  // Host packing.
  std::vector<Rec64> rec64(P);
  std::vector<Rec32> rec32((desc->build_flags & XS_BUILD_FP32) ? P : 0);
  double e_min = std::numeric_limits<double>::infinity(), e_max = 0.0;
  std::vector<int32_t> goff(K + 1);
  for (int k = 0; k <= K; ++k) goff[k] = (int32_t)desc->grid_offsets[k];
  for (int k = 0; k < K; ++k) {
    e_min = std::min(e_min, desc->energy[goff[k]]);
    e_max = std::max(e_max, desc->energy[goff[k + 1] - 1]);
  }
  for (int64_t p = 0; p < P; ++p) {
    for (int c = 0; c < XS_CHANNELS; ++c) rec64[p].x[c] = desc->xs[p * 5 + c];
    rec64[p].e = desc->energy[p];
    if (!rec32.empty()) {
      for (int c = 0; c < XS_CHANNELS; ++c)
        rec32[p].x[c] = (float)desc->xs[p * 5 + c];
      rec32[p].rcp = 0.0f;
      rec32[p].e = desc->energy[p];
    }
  }
  // Each FP32 record carries RN32(1 / d) of the interval it starts, d being
  // the FP64 difference the kernels form (the seed of their division).
  if (!rec32.empty())
    for (int k = 0; k < K; ++k)
      for (int64_t p = goff[k]; p + 1 < goff[k + 1]; ++p)
        rec32[p].rcp = (float)(1.0 / (desc->energy[p + 1] - desc->energy[p]));
  std::vector<MatRec> mrec(L);
  int max_L = 0;
  for (int m = 0; m < M; ++m) {
    max_L = std::max(max_L, desc->mat_offsets[m + 1] - desc->mat_offsets[m]);
    for (int32_t j = desc->mat_offsets[m]; j < desc->mat_offsets[m + 1]; ++j) {
      const int k = desc->mat_nuclides[j];
      mrec[j].base = goff[k];
      mrec[j].n = goff[k + 1] - goff[k];
      mrec[j].k = k;
      mrec[j].rho32 = (float)desc->mat_density[j];
    }
  }

  DevTables& d = h->d;
  d.K = K;
  d.M = M;
  double* E_dev;
  Rec64* r64;
  int32_t *moff, *goff_dev;
  MatRec* mr;
  double* rho;
  xs_status st;
  if ((st = upload(h, desc->energy, (size_t)P, &E_dev, s))) return cleanup(st);
  if ((st = upload(h, rec64.data(), rec64.size(), &r64, s))) return cleanup(st);
  if ((st = upload(h, desc->mat_offsets, (size_t)M + 1, &moff, s))) return cleanup(st);
  if ((st = upload(h, mrec.data(), mrec.size(), &mr, s))) return cleanup(st);
  if ((st = upload(h, desc->mat_density, (size_t)L, &rho, s))) return cleanup(st);
  if ((st = upload(h, goff.data(), goff.size(), &goff_dev, s))) return cleanup(st);
  d.E = E_dev;
  d.rec64 = r64;
  d.moff = moff;
  d.mrec = mr;
  d.rho64 = rho;
  if (!rec32.empty()) {
    Rec32* r32;
    if ((st = upload(h, rec32.data(), rec32.size(), &r32, s))) return cleanup(st);
    d.rec32 = r32;
  }
  // kept until the function returns, like the other host arrays whose
  // copies are in flight
  std::vector<Rec32> pairs;
  size_t pair_bytes = 0;
  if (!rec32.empty() && (desc->build_flags & XS_BUILD_FP32_PAIRS)) {
    pairs.resize(2 * (size_t)P);
    for (int k = 0; k < K; ++k)
      for (int64_t p = goff[k]; p < goff[k + 1]; ++p) {
        pairs[2 * p] = rec32[p];
        pairs[2 * p + 1] = rec32[p + 1 < goff[k + 1] ? p + 1 : p];
      }
    Rec32* pr;
    if ((st = upload(h, pairs.data(), pairs.size(), &pr, s))) return cleanup(st);
    d.pair32 = pr;
    pair_bytes = pairs.size() * sizeof(Rec32);
  }

  xs_table_info_t& info = h->info;
  info.n_nuclides = K;
  info.n_materials = M;
  info.max_material_size = max_L;
  info.n_points = P;
  info.build_flags = desc->build_flags;
  info.e_min = e_min;
  info.e_max = e_max;
  info.bytes_grid = (size_t)P * 8;
  info.bytes_fp64 = (size_t)P * sizeof(Rec64);
  info.bytes_fp32 = rec32.size() * sizeof(Rec32) + pair_bytes;
  info.bytes_materials = (size_t)(M + 1) * 4 + (size_t)L * (sizeof(MatRec) + 8);

  if (desc->build_flags & XS_BUILD_HASH) {
    // The default grid first, then the extra ones; every grid spans the same
    // [e_min, e_max] in ln E.
    d.ln_emin = std::log(e_min);
    const double span = std::log(e_max) - d.ln_emin;
    for (int g = 0; g <= desc->n_extra_hash_grids; ++g) {
      const int B = g == 0 ? desc->n_hash_bins : desc->extra_hash_bins[g - 1];
      void* H;
      const size_t bytes = (size_t)(B + 1) * K * 4;
      if ((st = alloc_dev(h, bytes, &H))) return cleanup(st);
      DevTables db = d;
      db.B = B;
      db.inv_dln = (double)B / span;
      db.H = (const int32_t*)H;
      hipError_t e = launch_hash_build(db, goff_dev, span / B, (int32_t*)H, s);
      if (e != hipSuccess)
        return cleanup(fail(XS_EHIP, "hash build launch failed: %s",
                            hipGetErrorString(e)));
      h->hash.push_back(HashGrid{B, db.inv_dln, db.H});
      info.hash_bins[g] = B;
      info.bytes_hash += bytes;
    }
    d.B = h->hash[0].B;
    d.inv_dln = h->hash[0].inv_dln;
    d.H = h->hash[0].H;
    info.n_hash_bins = d.B;
    info.n_hash_grids = (int32_t)h->hash.size();
  }
  info.checksum = table_checksum(desc);
  if (desc->build_flags & XS_BUILD_UNIONIZED) {
    std::vector<double> u(desc->energy, desc->energy + P);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    const int64_t U = (int64_t)u.size();
    double* u_dev;
    if ((st = upload(h, u.data(), u.size(), &u_dev, s))) return cleanup(st);
    void* uidx;
    const bool by_mat = (desc->build_flags & XS_BUILD_UNION_BY_MATERIAL) != 0;
    const size_t bytes = (size_t)U * (by_mat ? (size_t)L : (size_t)K) * 4;
    if ((st = alloc_dev(h, bytes, &uidx))) return cleanup(st);
    d.U = U;
    d.u = u_dev;
    d.uidx = (const int32_t*)uidx;
    d.union_by_material = by_mat ? 1 : 0;
    hipError_t e = by_mat
        ? launch_union_index_by_material(d, L, (int32_t*)uidx, s)
        : launch_union_index(d, goff_dev, (int32_t*)uidx, s);
    if (e != hipSuccess)
      return cleanup(fail(XS_EHIP, "union index launch failed: %s",
                          hipGetErrorString(e)));
    info.union_size = U;
    info.bytes_union = (size_t)U * 8 + bytes;

    // Logarithmic bins over the union grid (about 32 points per bin): the
    // union bracket of each bin's lower edge.  Lookups verify the bracket
    // they find, so the rounding of log and exp never changes a result.
    const int UB = (int)std::max<int64_t>(1, std::min<int64_t>(U / 32, 1 << 20));
    const double uln = std::log(u.front());
    const double uspan = std::log(u.back()) - uln;
    std::vector<int32_t> uh((size_t)UB + 1);
    for (int b = 0; b < UB; ++b) {
      const double edge = std::exp(uln + (double)b * (uspan / UB));
      const int64_t c = std::upper_bound(u.begin(), u.end(), edge) - u.begin();
      uh[b] = (int32_t)std::max<int64_t>(c - 1, 0);
    }
    uh[UB] = (int32_t)(U - 1);
    int32_t* uh_dev;
    if ((st = upload(h, uh.data(), uh.size(), &uh_dev, s))) return cleanup(st);
    d.UB = UB;
    d.u_ln_min = uln;
    d.u_inv_dln = (double)UB / uspan;
    d.uh = uh_dev;
  }
  hipError_t e = s ? hipStreamSynchronize(s) : hipDeviceSynchronize();
  if (e != hipSuccess)
    return cleanup(fail(XS_EHIP, "table build failed: %s", hipGetErrorString(e)));
  // Locate this device's fixed scratch array once (xs_lookup_batch_noalloc);
  // a failure is reported by that entry point, not here.
  (void)scratch_setup(h->device);
  clear_error();
  *out = h;
  return XS_OK;
}

xs_status xs_destroy_tables(xs_tables_t h) {
  clear_error();
  if (!h) return XS_OK;
  release(h);
  delete h;
  return XS_OK;
}

xs_status xs_table_info(xs_tables_t h, xs_table_info_t* info) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (!info) return fail(XS_EINVAL, "info is NULL");
  *info = h->info;
  return XS_OK;
}

xs_status xs_params_default(xs_params* p, int32_t precision) {
  clear_error();
  if (!p) return fail(XS_EINVAL, "params is NULL");
  if (precision != XS_FP64 && precision != XS_FP32)
    return fail(XS_EINVAL, "precision must be XS_FP64 or XS_FP32");
  p->precision = precision;
  p->grid = XS_AUTO;
  p->sort = XS_AUTO;
  p->block_size = 0;
  p->lookups_per_thread = 0;
  p->wave_per_lookup = XS_AUTO;
  p->lds_stage = XS_AUTO;
  p->sort_threshold = -1;
  p->queue = XS_AUTO;
  p->unroll = 0;
  p->hash_bins = XS_AUTO;
  return XS_OK;
}

xs_status xs_resolve_params(xs_tables_t h, int64_t n, const xs_params* in,
                            xs_params* out) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (!out) return fail(XS_EINVAL, "out is NULL");
  if (n < 0) return fail(XS_EINVAL, "n must be >= 0");
  return resolve(h, n, in, out);
}

xs_status xs_workspace_size(xs_tables_t h, int64_t n, const xs_params* params,
                            size_t* bytes) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (!bytes) return fail(XS_EINVAL, "bytes is NULL");
  if (n < 0 || n > 0x7fffffffLL) return fail(XS_EINVAL, "n out of range");
  size_t b = 0;
  // Enough for either entry point, each resolving automatic fields from its
  // own tuned entries: a sort (with or without the active flag) or a
  // compaction.
  for (int active = 0; active < 2; ++active) {
    xs_params p;
    if (xs_status st = resolve(h, n, params, &p, active)) return st;
    if (n > 0) {
      if (p.sort != XS_SORT_NONE && n >= p.sort_threshold)
        b = std::max(b, sort_workspace_bytes(n, 32));
      else
        b = std::max(b, compact_workspace_bytes(n));
    }
  }
  *bytes = b;
  return XS_OK;
}

xs_status xs_lookup_batch(xs_tables_t h, int64_t n, const double* d_E,
                          const int32_t* d_mat, void* d_out,
                          const xs_params* params, void* d_ws, size_t ws_bytes,
                          void* stream) {
  return lookup_common(h, n, d_E, d_mat, nullptr, false, d_out, params, d_ws,
                       ws_bytes, stream);
}

xs_status xs_lookup_active(xs_tables_t h, int64_t n, const double* d_E,
                           const int32_t* d_mat, const uint8_t* d_active,
                           void* d_out, const xs_params* params, void* d_ws,
                           size_t ws_bytes, void* stream) {
  return lookup_common(h, n, d_E, d_mat, d_active, true, d_out, params, d_ws,
                       ws_bytes, stream);
}

xs_status xs_lookup_indices(xs_tables_t h, int64_t n, const double* d_E,
                            const int32_t* d_mat, const int64_t* d_idx_offsets,
                            int32_t* d_idx, int32_t grid, void* stream) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (n < 0 || n > 0x7fffffffLL) return fail(XS_EINVAL, "n out of range");
  if (grid < 0 || grid > 2) return fail(XS_EINVAL, "unknown grid %d", grid);
  if (grid == XS_GRID_HASH && h->d.B == 0)
    return fail(XS_ENOTBUILT, "hash grid was not built");
  if (grid == XS_GRID_UNIONIZED && h->d.U == 0)
    return fail(XS_ENOTBUILT, "unionized grid was not built");
  if (n == 0) return XS_OK;
  if (!d_E || !d_mat || !d_idx_offsets || !d_idx)
    return fail(XS_EINVAL, "a pointer is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  switch (grid) {
    case XS_GRID_NUCLIDE:
      e = launch_indices_nuclide(h->d, n, d_E, d_mat, d_idx_offsets, d_idx, s);
      break;
    case XS_GRID_HASH:
      e = launch_indices_hash(h->d, n, d_E, d_mat, d_idx_offsets, d_idx, s);
      break;
    default:
      e = launch_indices_union(h->d, n, d_E, d_mat, d_idx_offsets, d_idx, s);
      break;
  }
  if (e != hipSuccess)
    return fail(XS_EHIP, "index kernel launch failed: %s", hipGetErrorString(e));
  if (h->d.dbg) return debug_check(h, n, d_E, d_mat, nullptr, s);
  return XS_OK;
}

xs_status xs_set_debug(xs_tables_t h, int32_t on) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (on != 0 && on != 1) return fail(XS_EINVAL, "on must be 0 or 1");
  int dev = -1;
  XS_HIP(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(XS_EINVAL, "current device %d is not the tables' device %d",
                dev, h->device);
  if (on && !h->dbg_dev) {
    void* p = nullptr;
    if (xs_status st = alloc_dev(h, kDbgWords * sizeof(unsigned long long), &p))
      return st;
    h->dbg_dev = (unsigned long long*)p;
  }
  if (on) {
    XS_HIP(hipDeviceSynchronize());
    XS_HIP(hipMemset(h->dbg_dev, 0, kDbgWords * sizeof(unsigned long long)));
    XS_HIP(hipDeviceSynchronize());
  }
  std::lock_guard<std::mutex> lk(h->mu);
  h->d.dbg = on ? h->dbg_dev : nullptr;
  h->dbg_calls = 0;
  return XS_OK;
}

xs_status xs_debug_counters(xs_tables_t h, xs_debug_info* out) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (!out) return fail(XS_EINVAL, "out is NULL");
  xs_debug_info r{};
  if (h->d.dbg) {
    unsigned long long c[kDbgWords];
    XS_HIP(hipDeviceSynchronize());
    XS_HIP(hipMemcpy(c, h->dbg_dev, sizeof(c), hipMemcpyDeviceToHost));
    r.invalid_queries = (int64_t)c[kDbgInvalid];
    r.hash_bin_scans = (int64_t)c[kDbgHashScans];
    r.hash_full_searches = (int64_t)c[kDbgHashFull];
    std::lock_guard<std::mutex> lk(h->mu);
    r.calls = h->dbg_calls;
    r.on = 1;
  }
  *out = r;
  return XS_OK;
}

xs_status xs_profile_begin(xs_tables_t h) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  std::lock_guard<std::mutex> lk(h->mu);
  for (auto& c : h->prof)
    for (hipEvent_t e : c.ev) h->event_pool.push_back(e);
  h->prof.clear();
  h->profiling = true;
  return XS_OK;
}

xs_status xs_profile_end(xs_tables_t h, xs_profile_t* out) {
  clear_error();
  if (xs_status st = check_handle(h)) return st;
  if (!out) return fail(XS_EINVAL, "out is NULL");
  std::lock_guard<std::mutex> lk(h->mu);
  h->profiling = false;
  xs_profile_t r{};
  for (auto& c : h->prof) {
    XS_HIP(hipEventSynchronize(c.ev[2]));
    float a = 0, b = 0, t = 0;
    XS_HIP(hipEventElapsedTime(&a, c.ev[0], c.ev[1]));
    XS_HIP(hipEventElapsedTime(&b, c.ev[1], c.ev[2]));
    XS_HIP(hipEventElapsedTime(&t, c.ev[0], c.ev[2]));
    r.ms_sort += a;
    r.ms_lookup += b;
    r.ms_total += t;
    r.calls += 1;
    r.sorted_calls += c.sorted ? 1 : 0;
    r.lookups += c.n;
  }
  for (auto& c : h->prof)
    for (hipEvent_t e : c.ev) h->event_pool.push_back(e);
  h->prof.clear();
  *out = r;
  return XS_OK;
}

const char* xs_status_string(xs_status st) {
  switch (st) {
    case XS_OK: return "XS_OK";
    case XS_EINVAL: return "XS_EINVAL: invalid argument";
    case XS_ETABLE: return "XS_ETABLE: table data rejected";
    case XS_ENOTBUILT: return "XS_ENOTBUILT: structure not built";
    case XS_EWORKSPACE: return "XS_EWORKSPACE: workspace missing or too small";
    case XS_ENOMEM: return "XS_ENOMEM: allocation failed";
    case XS_EHIP: return "XS_EHIP: HIP runtime error";
    case XS_ETIMEOUT: return "XS_ETIMEOUT: time limit reached";
    default: return "unknown xs_status";
  }
}

const char* xs_last_error(void) { return g_error; }

}  // extern "C"
