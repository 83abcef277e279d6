// Internal declarations of libxs: device table layout, kernels' launch
// helpers and the host-side handle.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "xs.h"

namespace xs {

// ---- device table layout -------------------------------------------------
//
// Search grid: every nuclide's energies back to back (FP64), dense so that
// bisection probes share cache lines.  Interpolation reads a record pair
// (point i and i+1) that carries both energies and the five channels, so a
// bracket costs one contiguous 96-byte (FP64) or 64-byte (FP32) read.

struct alignas(16) Rec64 {  // 48 bytes
  double x[XS_CHANNELS];
  double e;
};
struct alignas(16) Rec32 {  // 32 bytes
  float x[XS_CHANNELS];
  float rcp;  // RN32(1 / (E[p+1] - E[p])): the seed of the fraction's
              // division for the interval this point starts (0 at a
              // nuclide's last point)
  double e;
};
static_assert(sizeof(Rec64) == 48, "Rec64 layout");
static_assert(sizeof(Rec32) == 32, "Rec32 layout");

// One entry of a material list: where the nuclide's grid starts, its length,
// its id (row of the hash and union index tables) and its FP32 density.
struct alignas(16) MatRec {
  int32_t base;
  int32_t n;
  int32_t k;
  float rho32;
};

struct DevTables {
  int32_t K;                 // nuclides
  int32_t M;                 // materials
  const double* E;           // [P] search grid
  const Rec64* rec64;        // [P]
  const Rec32* rec32;        // [P] (null unless built)
  // [2P]: pair32[2p], pair32[2p + 1] = records p and p + 1 of a nuclide
  // (the last point of a nuclide repeats itself); null unless built
  const Rec32* pair32;
  const int32_t* moff;       // [M+1]
  const MatRec* mrec;        // [sum L]
  const double* rho64;       // [sum L]
  // logarithmic hash bins
  int32_t B;                 // bins (0 = not built)
  double ln_emin;            // ln of the lowest grid energy
  double inv_dln;            // B / (ln e_max - ln e_min)
  const int32_t* H;          // [(B+1) * K]: bracket of each bin's lower edge
  // unionized grid
  int64_t U;                 // union points (0 = not built)
  const double* u;           // [U]
  const int32_t* uidx;       // [U][K], or per material m a block [U][L_m]
                             // at U * moff[m] (union_by_material)
  int32_t union_by_material;
  // logarithmic bins over the union grid: row uh[b] is the union bracket of
  // bin b's lower edge (uh[UB] = U - 1), so a lookup searches one bin
  int32_t UB;                // bins (0 = not built)
  double u_ln_min;           // ln u[0]
  double u_inv_dln;          // UB / (ln u[U-1] - ln u[0])
  const int32_t* uh;         // [UB + 1]
  // debug counters, null unless the handle is in debug mode:
  // [kDbgHashScans] hash searches that left the fast two-interval window,
  // [kDbgHashFull] of those, searches that fell back to full bisection
  unsigned long long* dbg;
};

// Device debug counters (8 words): the two above, then the invalid queries
// of all debug calls, of the current call, and the lowest invalid position
// of the current call.
enum : int {
  kDbgHashScans = 0,
  kDbgHashFull = 1,
  kDbgInvalid = 2,
  kDbgCallInvalid = 3,
  kDbgCallFirst = 4,
  kDbgWords = 8
};

// ---- sort key ------------------------------------------------------------
// Layout, high to low: [inactive flag][energy band][material][energy rest].
// Without a band (band_bits = 0) the material sits above all energy bits.
struct SortKey {
  int32_t mat_bits;   // bits of the material field (0 = not in the key)
  int32_t e_bits;     // bits of the energy key (0 = not in the key)
  int32_t band_bits;  // top bits of the energy key placed above the material
  int32_t e_shift;    // right shift applied to (bits(E) - bits(e_min))
  int32_t flag_bit;   // 1: an "inactive" flag sits above the other fields
  int64_t e_bits_min; // IEEE bit pattern of e_min
  int32_t M;
  int32_t total_bits;
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per block
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;

// ---- host handle ---------------------------------------------------------

constexpr int kBuckets = 48;  // tuned parameters per floor(log2(n))

// One logarithmic hash grid of a handle (the default first).
struct HashGrid {
  int32_t B;
  double inv_dln;
  const int32_t* H;
};

struct ProfCall {
  hipEvent_t ev[3];  // before sort, after sort, after lookup
  bool sorted;
  int64_t n;
};

}  // namespace xs

struct xs_tables_s {
  int device = 0;
  xs::DevTables d{};
  xs_table_info_t info{};
  std::vector<void*> allocations;
  // every hash grid built (d's B, inv_dln and H are those of the first)
  std::vector<xs::HashGrid> hash;
  // tuned parameters per entry point (0 xs_lookup_batch, 1
  // xs_lookup_active), precision and batch-size class
  bool tuned_valid[2][2][xs::kBuckets] = {};
  xs_params tuned[2][2][xs::kBuckets] = {};
  std::mutex mu;
  bool profiling = false;
  std::vector<xs::ProfCall> prof;
  std::vector<hipEvent_t> event_pool;
  // pinned staging of request descriptors (xs_lookup_requests); the event
  // marks the end of the last copy out of it
  void* req_stage = nullptr;
  size_t req_stage_bytes = 0;
  hipEvent_t req_event = nullptr;
  // debug mode (xs_set_debug): device counters and calls checked since on
  unsigned long long* dbg_dev = nullptr;
  int64_t dbg_calls = 0;
};

namespace xs {

// Error reporting: records a message for xs_last_error() and returns st.
xs_status fail(xs_status st, const char* fmt, ...);
void clear_error();

#define XS_HIP(call)                                                      \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess)                                                 \
      return ::xs::fail(e_ == hipErrorOutOfMemory ? XS_ENOMEM : XS_EHIP,  \
                        "%s failed: %s", #call, hipGetErrorString(e_));   \
  } while (0)

// The library's parameters for a batch of n lookups when none were tuned
// (every field set; xs_api.hip).
void untuned_defaults(const xs_tables_s* h, int64_t n, int precision,
                      xs_params* out);

// Resolves automatic fields for entry point `active` (0 xs_lookup_batch, 1
// xs_lookup_active) and checks the result; xs_api.hip.
xs_status resolve_for(xs_tables_s* h, int64_t n, int active,
                      const xs_params* in, xs_params* out);

// The device tables a call with resolved parameters p runs on: the handle's,
// with the hash grid p.hash_bins names when p.grid is HASH.
DevTables tables_for(const xs_tables_s* h, const xs_params& p);

// Batch-size class of n: floor(log2 n), 0 for n <= 1.
int size_class(int64_t n);

// xs_lookup_batch's pipeline on a caller-chosen workspace, without the
// profiling events (which may allocate); xs_api.hip.
xs_status lookup_batch_into(xs_tables_t h, int64_t n, const double* E,
                            const int32_t* mat, void* out,
                            const xs_params* params, void* ws, size_t ws_bytes,
                            void* stream);

// The fixed device-side scratch array of xs_lookup_batch_noalloc
// (xs_noalloc.hip): finds its address on `device` (which must be current)
// once per device and caches it.  XS_OK or XS_EHIP.
xs_status scratch_setup(int device);

// Debug mode (xs_debug.hip): resets the current call's words of `counters`
// and counts the invalid queries among the first n (active ones only when
// `active` is not null).
hipError_t launch_debug_count(int64_t n, const double* E, const int32_t* mat,
                              const uint8_t* active, int M,
                              unsigned long long* counters, hipStream_t s);

// Table builders (xs_build.hip).
hipError_t launch_hash_build(const DevTables& t, const int32_t* goff_dev,
                             double dln, int32_t* H, hipStream_t s);
hipError_t launch_union_index(const DevTables& t, const int32_t* goff_dev,
                              int32_t* uidx, hipStream_t s);
hipError_t launch_union_index_by_material(const DevTables& t, int32_t Ltot,
                                          int32_t* uidx, hipStream_t s);

// Lookup kernels (xs_lookup_*.hip).  count_dev, when not null, holds the
// number of valid entries of perm (device-side queue length); the kernels
// then deal the blocks that hold queue entries evenly over the XCDs and the
// rest of the grid (sized for n) leaves at once.
struct LookupArgs {
  int64_t n;
  const double* E;
  const int32_t* mat;
  const int32_t* perm;     // null = identity
  const int64_t* count_dev;
  const uint8_t* active;   // null = all active
  void* out;
  // LDS-staged kernel over a sorted queue: block v covers the queue
  // positions [blocks[2v], blocks[2v + 1]), each range inside one group of
  // the sort key, for v < *n_blocks (launched as max_blocks blocks); null:
  // block v covers the next block_size * lookups-per-lane positions
  const int32_t* blocks = nullptr;
  const int32_t* n_blocks = nullptr;
  int64_t max_blocks = 0;
};
hipError_t launch_lookup_nuclide(const DevTables& t, const xs_params& p,
                                 const LookupArgs& a, hipStream_t s);
hipError_t launch_lookup_hash(const DevTables& t, const xs_params& p,
                              const LookupArgs& a, hipStream_t s);
hipError_t launch_lookup_union(const DevTables& t, const xs_params& p,
                               const LookupArgs& a, hipStream_t s);
hipError_t launch_indices_nuclide(const DevTables& t, int64_t n,
                                  const double* E, const int32_t* mat,
                                  const int64_t* off, int32_t* idx,
                                  hipStream_t s);
hipError_t launch_indices_hash(const DevTables& t, int64_t n, const double* E,
                               const int32_t* mat, const int64_t* off,
                               int32_t* idx, hipStream_t s);
hipError_t launch_indices_union(const DevTables& t, int64_t n, const double* E,
                                const int32_t* mat, const int64_t* off,
                                int32_t* idx, hipStream_t s);

// Sort and compaction (xs_sort.hip).
size_t sort_workspace_bytes(int64_t n, int total_bits);
size_t compact_workspace_bytes(int64_t n);
// Sorts lookups by `key`; on return *perm_out points into ws at the
// permutation (sorted position -> input index).  With keys_out, the sorted
// keys are written too (*keys_out), and *spare points at n words of ws the
// sort no longer needs.  With active_out and a key with the inactive flag,
// *active_out points into ws at the number of active lookups (device
// int64), which lead the sorted order.
hipError_t launch_sort(const SortKey& key, int64_t n, const double* E,
                       const int32_t* mat, const uint8_t* active, void* ws,
                       const int32_t** perm_out, const uint32_t** keys_out,
                       uint32_t** spare, const int64_t** active_out,
                       hipStream_t s);
// Block ranges of the LDS-staged kernel over sorted keys: the queue is cut
// at every change of key >> gshift (groups of one material) and each group
// into pieces of per_block positions.  groups = the number of possible
// values of key >> gshift; only the ranges of groups [0, used) are served
// (used = groups / 2 when the top group bit is the inactive flag).  The
// ranges and the starts use 8 * (2 * groups + 2 + n / per_block) + 256
// bytes of `spare`.  Sets a->blocks, a->n_blocks and a->max_blocks (an
// upper bound of the count).
hipError_t launch_block_ranges(const uint32_t* keys, int64_t n, int gshift,
                               int64_t groups, int64_t used, int64_t per_block,
                               void* spare, LookupArgs* a, hipStream_t s);
// Stable compaction of active slots: perm (in ws) lists them in input
// order, *count_out (device) their number.
hipError_t launch_compact(int64_t n, const uint8_t* active, void* ws,
                          const int32_t** perm_out,
                          const int64_t** count_out, hipStream_t s);

}  // namespace xs
