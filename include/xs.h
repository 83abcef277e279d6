/*
 * xs.h: C interface of the MI355X (gfx950) batched macroscopic
 * cross-section lookup library, libxs.so.
 *
 * The operation (paper section 5.1, the paragraph on logarithmic hash-grid
 * bins that follows Table 1): a particle at energy E inside material m needs
 * the macroscopic cross sections of m at E.  Every nuclide k of m is searched
 * for the interval of its energy grid that holds E, its tabulated channels
 * are interpolated linearly in E, and the nuclides' values are summed
 * weighted by their densities in m:
 *
 *   i_k   = clamp(#{p : E_k[p] <= E} - 1, 0, n_k - 2)
 *   Eh    = min(max(E, E_k[0]), E_k[n_k - 1])
 *   f     = (Eh - E_k[i]) / (E_k[i+1] - E_k[i]),   g = 1 - f
 *   s_k,c = g * X_k[i][c] + f * X_k[i+1][c]
 *   S_c   = sum over the material list, in list order, of rho_j * s_kj,c
 *
 * The paper gives the particle count in flight (1e5 to ~8e6, Table 1), the
 * number of logarithmic hash bins (100 to 100k, default 4,000), queued versus
 * queueless control flow and a minimum sorting threshold (default 20,000) as
 * the tunables of this kernel; they appear here as the batch size n, the
 * hash-grid bin count, xs_lookup_active's queue mode and sort_threshold.
 *
 * Conventions for every entry point:
 *  - Return value: XS_OK (0) or a negative xs_status.  No C++ exception and
 *    no abort crosses this interface.  On error, out-parameters are left
 *    untouched and xs_last_error() describes the failure (per thread).
 *  - "DEVICE" pointers are HIP device memory on the current device, owned by
 *    the caller, and must stay valid until the stream has completed the
 *    call.  "HOST" pointers are read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Lookups are asynchronous: a fault inside a kernel surfaces at the next
 *    synchronisation of that stream, not as a return value here.
 *  - A table handle is immutable after creation (xs_tune only records tuned
 *    parameters in it) and may be used from several streams at once, each
 *    call with its own workspace.
 */
#ifndef XS_H
#define XS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xs_status;
#define XS_OK 0
#define XS_EINVAL (-1)     /* an argument is NULL, out of range or unsupported */
#define XS_ETABLE (-2)     /* table data rejected by xs_create_tables */
#define XS_ENOTBUILT (-3)  /* grid type or precision not built into the handle */
#define XS_EWORKSPACE (-4) /* workspace missing, too small or misaligned */
#define XS_ENOMEM (-5)     /* a device or host allocation failed */
#define XS_EHIP (-6)       /* a HIP runtime call failed */
#define XS_ETIMEOUT (-7)   /* a bounded wait ran out (tuner cut-off, stream) */

#define XS_AUTO (-1)       /* "choose for me" in xs_params fields */
#define XS_CHANNELS 5      /* reaction channels per grid point */

/* Grid search methods.  All three return the same brackets i_k. */
#define XS_GRID_NUCLIDE 0    /* bisection of each nuclide's grid */
#define XS_GRID_HASH 1       /* logarithmic hash bins narrow each search */
#define XS_GRID_UNIONIZED 2  /* one search of the union grid + index table */

#define XS_FP64 0  /* FP64 tables, arithmetic and output */
#define XS_FP32 1  /* FP32 channels and densities, FP64 search and fraction,
                      FP32 interpolation, Kahan-compensated FP32 sum, FP32
                      output */

/* Reordering of lookups before the lookup kernel (never changes values).
 * Paper section 5.1 ("minimum sorting threshold"): sorting puts neighbouring
 * particles in the same material and close in energy.  BAND_MATERIAL orders
 * by a coarse energy band first, then material, then energy inside the band:
 * lookups in flight together then cover a narrow energy range of every
 * nuclide (a small cache footprint) while each wave still holds a single
 * material. */
#define XS_SORT_NONE 0
#define XS_SORT_MATERIAL 1
#define XS_SORT_ENERGY 2
#define XS_SORT_MATERIAL_ENERGY 3
#define XS_SORT_BAND_MATERIAL 4

/* xs_lookup_active: how inactive slots are skipped. */
#define XS_QUEUE_COMPACT 0     /* queued: compact active lookups, then look up */
#define XS_QUEUE_PREDICATED 1  /* queueless: every slot's lane checks its flag */

/* Optional structures built by xs_create_tables. */
#define XS_BUILD_FP32 1u
#define XS_BUILD_HASH 2u
#define XS_BUILD_UNIONIZED 4u
/* With XS_BUILD_UNIONIZED: store the union index per material, a block
 * [U][L_m] of the brackets of material m's list, instead of [U][K].  A lookup
 * then reads L_m contiguous indices instead of a K-wide row; memory is
 * U * sum(L_m) * 4 bytes instead of U * K * 4. */
#define XS_BUILD_UNION_BY_MATERIAL 8u
/* With XS_BUILD_FP32: also store each grid interval's two FP32 records side
 * by side in a 64-byte aligned block (64 more bytes per grid point).  A
 * lookup that reads its bracket of each nuclide from global memory (the
 * one-wave-per-lookup kernel, union or bisection grid) then touches one
 * aligned 64-byte block per nuclide instead of two neighbouring 32-byte
 * records, which cross a 128-byte line for one interval in four.  Results
 * are unchanged. */
#define XS_BUILD_FP32_PAIRS 16u

typedef struct xs_tables_s* xs_tables_t;

/* Table description: all pointers HOST, read during xs_create_tables only.
 * Requirements (else XS_ETABLE):
 *  - 1 <= n_nuclides; n_channels == 5;
 *  - grid_offsets[0] == 0, n_k = grid_offsets[k+1] - grid_offsets[k] >= 2,
 *    total points < 2^31;
 *  - energy: within [2^-400, 2^400] (about 3.9e-121 to 2.6e120; any unit
 *    of energy in use fits) and strictly increasing within each nuclide;
 *  - xs: [total points][5] point-major, finite and >= 0;
 *  - 1 <= n_materials <= 65536; mat_offsets[0] == 0, sizes L_m >= 1;
 *  - mat_nuclides: ids in [0, n_nuclides), no id twice within a material,
 *    any order (the sum follows this list order);
 *  - mat_density: finite and > 0;
 *  - with XS_BUILD_FP32, every nonzero channel value and every density must
 *    round to a normal finite FP32 number (about 1.2e-38 to 3.4e38), since
 *    the FP32 form's relative error bound holds only there, and so must the
 *    reciprocal of every spacing of neighbouring grid energies (spacings of
 *    about 3e-39 to 8e37; the FP32 records carry it);
 *  - n_hash_bins in [1, 100000] when XS_BUILD_HASH is set (the paper's range
 *    is 100 to 100k; 1 bin makes every search a full bisection);
 *  - with XS_BUILD_HASH, n_extra_hash_grids in [0, XS_MAX_HASH_GRIDS - 1]
 *    further hash grids of extra_hash_bins[i] bins each, every count in
 *    [1, 100000] and all counts (n_hash_bins included) distinct; without
 *    XS_BUILD_HASH it must be 0.  Grid HASH then searches the grid that
 *    xs_params.hash_bins names (paper Table 1: the bin count is a tunable
 *    that trades memory for search length); n_hash_bins is the default. */
#define XS_MAX_HASH_GRIDS 8
typedef struct {
  int32_t n_nuclides;
  int32_t n_channels;
  const int64_t* grid_offsets; /* [n_nuclides + 1] */
  const double* energy;        /* [grid_offsets[n_nuclides]] */
  const double* xs;            /* [grid_offsets[n_nuclides] * 5] */
  int32_t n_materials;
  const int32_t* mat_offsets;  /* [n_materials + 1] */
  const int32_t* mat_nuclides; /* [mat_offsets[n_materials]] */
  const double* mat_density;   /* [mat_offsets[n_materials]] */
  uint32_t build_flags;        /* XS_BUILD_* bits */
  int32_t n_hash_bins;         /* bins of the default hash grid */
  int32_t n_extra_hash_grids;  /* further hash grids (0 = none) */
  const int32_t* extra_hash_bins; /* [n_extra_hash_grids] bin counts */
} xs_table_desc;

/* Launch and method parameters of one lookup call.  Every field except
 * `precision` may be XS_AUTO (or 0 for block_size / lookups_per_thread), in
 * which case the value recorded by xs_tune for this precision and batch size
 * is used, else the library default: grid UNIONIZED if built, else HASH if
 * built, else NUCLIDE; block 128, 1 lookup per thread, 1 nuclide in flight;
 * for n >= 262,144 (one query per lane of the chip) sort BAND_MATERIAL at
 * n >= 20,000 and LDS stage shape 3 below 1.5M lookups, 2 below 3M, 1
 * above; for smaller n one wave per lookup, unsorted.  An XS_AUTO
 * wave_per_lookup or lds_stage becomes 0 wherever the fields set explicitly
 * exclude it.  The
 * choice never changes the results: every combination returns the same
 * indices and, within one precision, bit-identical sums. */
typedef struct {
  int32_t precision;          /* XS_FP64 or XS_FP32 (output element type) */
  int32_t grid;               /* XS_GRID_* */
  int32_t sort;               /* XS_SORT_* */
  int32_t block_size;         /* 64..1024, multiple of 64; with
                                 w = lookups_per_thread * unroll, at most 512
                                 when w > 1 and 256 when w > 4; with
                                 lds_stage > 0 at most 1024 /
                                 lookups_per_thread */
  int32_t lookups_per_thread; /* 1..8 */
  int32_t lds_stage;          /* 0: off; 1, 2, 3: blocks whose lookups share
                                 a material stage each nuclide's bracket
                                 window in LDS, 32 nuclides with windows of
                                 up to 8 records (6 in FP64) per round, 16
                                 with 16 (12), or 8 with 32 (24): wider
                                 windows suit sparser batches.  Needs
                                 lookups_per_thread <= 2 and unroll = 1 */
  int64_t sort_threshold;     /* sort only when n >= sort_threshold
                                 (0 = always, INT64_MAX = never) */
  int32_t queue;              /* xs_lookup_active only: XS_QUEUE_* */
  int32_t unroll;             /* nuclides in flight per lane: 1, 2 or 4
                                 (2 and 4 need lookups_per_thread <= 2) */
  int32_t wave_per_lookup;    /* 1: the 64 lanes of a wave share one lookup,
                                 each taking every 64th nuclide of its
                                 material (small batches); needs
                                 lookups_per_thread = unroll = 1, lds_stage
                                 = 0 and block_size <= 256 */
  int32_t hash_bins;          /* grid HASH only: bin count of the built hash
                                 grid to search (XS_ENOTBUILT if none has
                                 it); 0 or XS_AUTO: the tuned one, else the
                                 default grid.  Resolves to 0 for the other
                                 grid methods (a conditional parameter) */
} xs_params;

/* Sizes of a built handle. */
typedef struct {
  int32_t n_nuclides, n_materials, max_material_size, n_hash_bins;
  int64_t n_points;          /* total grid points over all nuclides */
  int64_t union_size;        /* points of the union grid (0 if not built) */
  uint32_t build_flags;
  uint32_t reserved;
  double e_min, e_max;       /* smallest first and largest last grid energy */
  int32_t n_hash_grids;      /* hash grids built (0 without XS_BUILD_HASH) */
  int32_t hash_bins[XS_MAX_HASH_GRIDS]; /* their bin counts, default first */
  int32_t reserved2;
  uint64_t checksum;         /* 64-bit digest of every array of the table
                                description, the build flags and the hash-bin
                                counts: the key of tuned-parameter caches */
  size_t bytes_grid;         /* search grid (FP64 energies) */
  size_t bytes_fp64;         /* FP64 interpolation records */
  size_t bytes_fp32;         /* FP32 interpolation records (and pairs) */
  size_t bytes_materials;    /* material lists */
  size_t bytes_hash;         /* hash-bin index table */
  size_t bytes_union;        /* union grid + its index table */
} xs_table_info_t;

/* Per-stage device time of lookup calls made between xs_profile_begin and
 * xs_profile_end on the handle (HIP events on each call's stream). */
typedef struct {
  double ms_sort;      /* key build + radix passes (+ compaction) */
  double ms_lookup;    /* the lookup kernel itself */
  double ms_total;     /* first to last event of each call, summed */
  int64_t calls;       /* lookup calls recorded */
  int64_t sorted_calls;/* calls that sorted */
  int64_t lookups;     /* lookups processed by the recorded calls */
} xs_profile_t;

/* ---- tables ------------------------------------------------------------ */

/* Validates `desc`, copies every array to device memory, builds the optional
 * FP32 records, hash-bin table (paper section 5.1: "logarithmic hash grid
 * bins") and unionized grid, and returns a handle.  Synchronises `stream`
 * before returning; the host arrays may be freed afterwards.
 * Errors: XS_EINVAL (NULL), XS_ETABLE (data), XS_ENOMEM, XS_EHIP. */
xs_status xs_create_tables(const xs_table_desc* desc, void* stream,
                           xs_tables_t* out);

/* Frees every device allocation of the handle.  The caller must have
 * completed all work that uses it.  NULL is accepted (no-op). */
xs_status xs_destroy_tables(xs_tables_t tables);

/* Sizes and byte counts of the handle. */
xs_status xs_table_info(xs_tables_t tables, xs_table_info_t* info);

/* ---- parameters ---------------------------------------------------------- */

/* Fills *p with XS_AUTO everywhere (0 for block_size, lookups_per_thread
 * and unroll, -1 for sort_threshold) and the given precision. */
xs_status xs_params_default(xs_params* p, int32_t precision);

/* Resolves XS_AUTO fields for a batch of n lookups exactly as
 * xs_lookup_batch would, and checks the result (XS_EINVAL for out-of-range
 * values, XS_ENOTBUILT for a grid or precision the handle lacks).  `in` may
 * be NULL (all automatic, FP64). */
xs_status xs_resolve_params(xs_tables_t tables, int64_t n,
                            const xs_params* in, xs_params* out);

/* Bytes of device workspace xs_lookup_batch / xs_lookup_active need for n
 * lookups with these parameters (0 when no sort or compaction runs). */
xs_status xs_workspace_size(xs_tables_t tables, int64_t n,
                            const xs_params* params, size_t* bytes);

/* ---- lookups ------------------------------------------------------------- */

/* n lookups: out[q][c] = S_c(d_E[q], d_mat[q]) for q < n, c < 5.
 *  d_E   DEVICE double [n];  d_mat DEVICE int32 [n];
 *  d_out DEVICE [n][5] double (XS_FP64) or float (XS_FP32);
 *  params may be NULL (all automatic, FP64);
 *  d_ws  DEVICE, 256-byte aligned, ws_bytes >= xs_workspace_size(...).
 * A lookup with E not finite and > 0, or m outside [0, n_materials), gets
 * NaN in all five channels.  n == 0 is a no-op.  Output order is input order
 * whatever the sort policy. */
xs_status xs_lookup_batch(xs_tables_t tables, int64_t n, const double* d_E,
                          const int32_t* d_mat, void* d_out,
                          const xs_params* params, void* d_ws, size_t ws_bytes,
                          void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * lookup, parameters, results and errors as xs_lookup_batch, but the sort's
 * scratch comes from a fixed array inside the library instead of a caller
 * workspace, so the call allocates nothing (no hipMalloc, no event; calls
 * are not recorded by xs_profile_begin).  The caller still passes the
 * queries and the output.
 *  - Every GPU the library runs on holds one such array of
 *    XS_NOALLOC_SCRATCH_BYTES (128 MiB) from the library's load until the
 *    process ends; its address is found once per device by
 *    xs_create_tables.
 *  - A sorted batch (sort != XS_SORT_NONE and n >= sort_threshold) may hold
 *    at most XS_NOALLOC_MAX_SORTED lookups (8,323,456: the paper's 1e5 to
 *    8e6 particles in flight fit); larger sorted batches return
 *    XS_EWORKSPACE before anything is enqueued.  Unsorted batches use no
 *    scratch and take any n xs_lookup_batch takes.
 *  - All calls on one GPU share that GPU's array, and it keeps the last
 *    call's contents: calls that overlap in time on one GPU (other host
 *    threads, or other streams not ordered after this one) race and may
 *    return wrong results.  Calls on one stream are ordered and safe. */
#define XS_NOALLOC_SCRATCH_BYTES (128u << 20)
#define XS_NOALLOC_MAX_SORTED 8323456
xs_status xs_lookup_batch_noalloc(xs_tables_t tables, int64_t n,
                                  const double* d_E, const int32_t* d_mat,
                                  void* d_out, const xs_params* params,
                                  void* stream);

/* As xs_lookup_batch for the slots whose d_active[q] != 0 (DEVICE uint8
 * [n]); the outputs of other slots are not written.  params->queue picks
 * compaction of the active slots (queued) or a predicated pass over all
 * slots (queueless), paper section 5.1 "queuing logic". */
xs_status xs_lookup_active(xs_tables_t tables, int64_t n, const double* d_E,
                           const int32_t* d_mat, const uint8_t* d_active,
                           void* d_out, const xs_params* params, void* d_ws,
                           size_t ws_bytes, void* stream);

/* Validation path: writes the bracket i_k of every (lookup, nuclide) pair
 * found with the given grid method.  d_idx_offsets DEVICE int64 [n+1] is the
 * prefix sum of the material sizes of the lookups; lookup q writes
 * d_idx[d_idx_offsets[q] + j] for its j-th nuclide (list order).  A lookup
 * with invalid E writes -1; one with an invalid material writes nothing. */
xs_status xs_lookup_indices(xs_tables_t tables, int64_t n, const double* d_E,
                            const int32_t* d_mat, const int64_t* d_idx_offsets,
                            int32_t* d_idx, int32_t grid, void* stream);

/* ---- tuning ---------------------------------------------------------------- */

/* Search strategies.  FOREST is the paper's method (section 2.1): Bayesian
 * optimisation with a random-forest surrogate of log(runtime) and the
 * lower-confidence-bound acquisition a(x) = mu(x) - kappa sigma(x) (Eq. 1),
 * sigma being the spread of the trees' predictions. */
#define XS_TUNE_EXHAUSTIVE 0
#define XS_TUNE_FOREST 1

/* The space (paper section 5.2 builds its space the same way, with
 * conditional parameters):
 *   grid method (built and in grid_mask)
 *     hash_bins      one of the hash grids on offer   | grid == HASH
 *   sort policy (in sort_mask)
 *     sort_threshold 0 (always sort), 20,000 (the    | sort != NONE
 *                    paper's default) or INT64_MAX
 *                    (never), paper Table 1
 *   queue mode       COMPACT or PREDICATED            | active == 1
 *   block size 64..1024 x (lookups per lane, nuclides in flight, LDS stage
 *   shape, wave per lookup), invalid combinations excluded.
 * An inactive parameter holds a fixed value (hash_bins 0, sort_threshold
 * INT64_MAX, queue COMPACT) and is never varied. */
typedef struct {
  int32_t precision;      /* XS_FP64 or XS_FP32 */
  int32_t strategy;       /* XS_TUNE_* */
  int32_t max_evals;      /* FOREST: evaluations including the baseline and
                             the initial random ones (<= 0: whole space) */
  int32_t init_samples;   /* FOREST: random configurations before the first
                             surrogate fit */
  int32_t batch;          /* FOREST: configurations proposed per fit (the
                             paper's workers per batch); >= 1 */
  int32_t reps;           /* timed runs per configuration, best kept (the
                             paper reports the best of 5) */
  int32_t warmup;         /* untimed runs per configuration */
  int32_t active;         /* 0: tune xs_lookup_batch; 1: xs_lookup_active
                             (the queue mode joins the space) */
  double timeout_factor;  /* a configuration whose first timed run exceeds
                             factor x the baseline's time is stopped and
                             scored at that time-out (paper: 1.5); <= 0
                             disables */
  double kappa;           /* LCB weight, >= 0 (paper default 1.96) */
  uint64_t seed;          /* random initial samples and bootstrap draws */
  uint32_t grid_mask;     /* bit g: consider grid method g (0 = all built) */
  uint32_t sort_mask;     /* bit s: consider sort policy s (0 = all) */
  int32_t n_hash_grids;   /* xs_tune_search only: the hash grids on offer
                             (0: one grid, hash_bins 0); xs_tune offers
                             every hash grid of the handle */
  int32_t hash_bins[XS_MAX_HASH_GRIDS];
  int32_t confirm;        /* finalists re-timed after the search (< 2: none).
                             The search scores each configuration on one
                             evaluation, so among near-equal configurations
                             the winner is often the one that drew the
                             luckier run.  The `confirm` best configurations
                             and the baseline are evaluated again, round-
                             robin, three times, and the lowest median wins;
                             best_ms and baseline_ms are then those medians.
                             These runs are not counted in `evaluated`. */
} xs_tune_config;

typedef struct {
  xs_params best;         /* fully resolved, no XS_AUTO fields */
  double best_ms;
  xs_params baseline;     /* the library default, evaluated first */
  double baseline_ms;
  int32_t evaluated;      /* configurations run, baseline included (0 when
                             the entry came from a cache) */
  int32_t cut;            /* of which stopped at the time-out */
  int32_t space_size;     /* valid configurations in the space */
  int32_t best_eval;      /* 1-based evaluation at which `best` was found */
  int64_t n;              /* xs_tune: the batch size tuned */
  int32_t from_cache;     /* xs_tune: 1 if read from the cache file */
  int32_t measured;       /* xs_tune: evaluations that ran on the device (a
                             configuration that launches the same kernels
                             at this n as one already timed reuses its
                             time) */
} xs_tune_result;

/* Evaluator used by xs_tune_search: run configuration *p and store its time
 * in *ms (milliseconds).  It may stop early once the time exceeds cutoff_ms
 * (infinity until the baseline is known) and report any value above it.
 * Returns XS_OK or an error status, which aborts the search. */
typedef xs_status (*xs_eval_fn)(const xs_params* p, double cutoff_ms,
                                double* ms, void* user);

/* Fills *c with the defaults: FOREST, 48 evaluations, 10 initial samples,
 * batch 1, best of 5 after 1 warm-up, time-out 1.5x baseline, kappa 1.96,
 * seed 1234, all grids and sorts, xs_lookup_batch, 3 finalists confirmed. */
xs_status xs_tune_config_default(xs_tune_config* c);

/* Searches the space above over the grid methods in built_grids & grid_mask
 * and the hash grids cfg lists, calling `eval` for each configuration it
 * picks; the first is the baseline (hash grid if built, banded sort at
 * threshold 20,000, block 256, two nuclides in flight).  No device call of
 * its own. */
xs_status xs_tune_search(uint32_t built_grids, const xs_tune_config* cfg,
                         xs_eval_fn eval, void* user, xs_tune_result* result);

/* A tuning request (paper section 3: ytopt proposes configurations, workers
 * run them and the results go to a performance database).  All pointers
 * DEVICE unless marked HOST. */
typedef struct {
  int32_t n_sizes;            /* batch sizes to tune, 1..64 */
  int32_t reserved;           /* must be 0 */
  const int64_t* sizes;       /* HOST [n_sizes], each in [1, 2^31 - 1]; e.g.
                                 the paper's particles in flight 1e5..8e6 */
  const double* d_E;          /* sample queries [max size]; size n tunes on
                                 the first n */
  const int32_t* d_mat;       /* [max size] */
  const uint8_t* d_active;    /* [max size] with config.active, else NULL */
  void* d_out;                /* [max size][5] of the precision's type */
  void* d_ws;                 /* 256-byte aligned, at least
                                 xs_workspace_size(max size) with a sort */
  size_t ws_bytes;
  void* stream;
  const char* cache_path;     /* HOST file of tuned parameters, or NULL */
  xs_tune_config config;
} xs_tune_request;

/* Tunes every size of the request (xs_lookup_batch, or xs_lookup_active
 * with config.active) and records each winner in the handle for the
 * batch-size class floor(log2 n): later calls whose fields are XS_AUTO use
 * the tuned value of the nearest class of the same entry point.  Each size's
 * baseline is the untuned default for it, so a result is never slower than
 * what an untuned call would run.  With a cache path, a size whose key
 * (device, table checksum, precision, entry point, class) the file holds is
 * taken from it without running anything, and each newly tuned size is
 * written to it (the file is rewritten through a temporary file and a
 * rename, so a reader never sees half a file).  results[n_sizes] (HOST)
 * receives one entry per size, in order.  Synchronises the stream.
 * Errors: XS_EINVAL (sizes, pointers, config), XS_EWORKSPACE, XS_ENOTBUILT,
 * XS_EHIP; a cache file that cannot be written is XS_EINVAL after the
 * results are recorded in the handle. */
xs_status xs_tune(xs_tables_t tables, const xs_tune_request* req,
                  xs_tune_result* results);

/* Records complete parameters (no XS_AUTO field) as tuned for the class of
 * n, for xs_lookup_batch (active 0) or xs_lookup_active (active 1); p ==
 * NULL clears every tuned entry of both. */
xs_status xs_set_tuned(xs_tables_t tables, int64_t n, int32_t active,
                       const xs_params* p);

/* Loads every entry of a tuned-parameter file whose device and table
 * checksum match this handle and device into the handle (as xs_set_tuned
 * would); entries that no longer resolve (a grid not built) are skipped.
 * *loaded (may be NULL) gets the number loaded.  A missing file loads 0. */
xs_status xs_tune_load(xs_tables_t tables, const char* cache_path,
                       int32_t* loaded);

/* The key of a tuned-parameter entry. */
typedef struct {
  char device[96];        /* device name, architecture and compute units */
  uint64_t checksum;      /* xs_table_info_t.checksum */
  int32_t precision;
  int32_t active;         /* 0 xs_lookup_batch, 1 xs_lookup_active */
  int32_t size_class;     /* floor(log2 n) */
  int32_t reserved;
} xs_tune_key;

/* The file format, for tools that read or fill a cache without a device:
 * xs_tune_cache_get finds the entry of *key in the file (XS_OK, *p and
 * *best_ms filled; XS_ENOTBUILT if the file has no such entry or does not
 * exist); xs_tune_cache_put adds or replaces it (atomic rewrite). */
xs_status xs_tune_cache_get(const char* cache_path, const xs_tune_key* key,
                            xs_params* p, double* best_ms);
xs_status xs_tune_cache_put(const char* cache_path, const xs_tune_key* key,
                            const xs_params* p, double best_ms);

/* The key of this handle, on the current device, for (precision, active,
 * n). */
xs_status xs_tune_key_of(xs_tables_t tables, int32_t precision,
                         int32_t active, int64_t n, xs_tune_key* key);

/* ---- request streams ------------------------------------------------------ */

/* Many uneven batches, each served by one launch of a HIP graph (paper
 * section 5.1: the particle buffer is refilled after each kernel call, and
 * with short kernels launches and queue-count transfers to the host leave
 * bubbles).  The stream's parameters are resolved for each batch's total
 * size, and they pick one of two graphs:
 *  - sorted (the resolved sort != XS_SORT_NONE and total >= sort_threshold,
 *    total < 2^31, debug mode off): the batch-sorted pipeline of
 *    xs_lookup_requests (gather every request into one queue, sort it, look
 *    it up with the resolved launch shape, scatter the results back) is
 *    captured for the batch and updates one instantiated graph in place; a
 *    request's time runs from the first gathered tile to its last scattered
 *    tile, so every request finishes with the batch;
 *  - otherwise the persistent kernel: the graph [reset times] ->
 *    [persistent kernel] is built once, and before each launch its kernel
 *    arguments (request and tile counts, the batch's tag, the largest
 *    request size) are rewritten.  The kernel's fixed grid strides over the
 *    batch's 1024-lookup tiles, so no loop bound comes from device memory;
 *    each block checks the tile's descriptor (the batch's tag, a size within
 *    the host's bound, the tile inside the request), sorts the tile in LDS by
 *    material and energy, looks it up, and stamps the request's first and
 *    last tile with the device wall clock.  Requests finish as their tiles
 *    do, at the throughput of unsorted lookups.
 * Results equal xs_lookup_batch's bit for bit in both. */
typedef struct xs_stream_s* xs_stream_t;

typedef struct {
  int64_t n;              /* lookups of the request, 0 <= n < 2^31 */
  const double* d_E;      /* DEVICE [n] */
  const int32_t* d_mat;   /* DEVICE [n] */
  void* d_out;            /* DEVICE [n][5] of the stream's precision */
} xs_request;

typedef struct {
  int64_t n;
  double start_us;        /* first tile start, from the batch's first start */
  double end_us;          /* last tile end, same origin */
  double latency_us;      /* end_us - start_us (0 for an empty request) */
} xs_request_stats;

/* Creates a stream for batches of up to max_requests requests on `stream`
 * (a hipStream_t as void*).  params (NULL: all automatic, FP64) fixes the
 * precision; its other fields are resolved for each batch's total (XS_AUTO
 * fields from the handle's tuned parameters, as xs_lookup_batch would), and
 * the persistent kernel takes the grid method and nuclides in flight
 * resolved here for a batch of 2^20 lookups.  Builds and instantiates the
 * persistent kernel's graph once (allocates); a sorted batch larger than
 * any before also allocates, on submit, its queue, results and sort
 * workspace (kept until the stream is destroyed). */
xs_status xs_stream_create(xs_tables_t tables, const xs_params* params,
                           int32_t max_requests, void* stream,
                           xs_stream_t* out);

/* Enqueues one batch (HOST array of count descriptors, read during the call)
 * on the stream: the descriptors are copied to the device on the stream
 * object's own upload stream and the host waits for that copy (no wait on
 * the caller's stream), then the batch's graph is launched on the caller's
 * stream.  One batch may be in flight per stream object; XS_EINVAL if the
 * previous one was not waited for. */
xs_status xs_stream_submit(xs_stream_t s, const xs_request* reqs,
                           int32_t count);

/* Waits for the batch and fills stats[count] (may be NULL) and the batch's
 * device makespan in microseconds (may be NULL).  XS_EHIP if any tile met a
 * descriptor that was not written for this batch (its outputs are then not
 * written). */
xs_status xs_stream_wait(xs_stream_t s, xs_request_stats* stats,
                         double* makespan_us);

/* The parameters the persistent kernel runs with (resolved at creation). */
xs_status xs_stream_params(xs_stream_t s, xs_params* out);

/* Waits for any batch in flight and frees the stream.  NULL is a no-op. */
xs_status xs_stream_destroy(xs_stream_t s);

/* A batch of requests served together (HOST array of count descriptors,
 * read during the call); the paper's queue of particles in flight (section
 * 5.1) fed by many callers at once.  Parameters are resolved as for one
 * batch of the total size (NULL = tuned defaults), and the sort policy picks
 * the mode:
 *  - sort != XS_SORT_NONE and total >= sort_threshold (batch-sorted): one
 *    gather kernel copies every request into one queue, the queue is sorted
 *    and looked up as in xs_lookup_batch, and one scatter kernel writes each
 *    request's results back; a request's time runs from its first gathered
 *    tile to its last scattered tile;
 *  - otherwise (tile-sorted): one launch with a 256-lane block per
 *    1024-lookup tile of each request; the block sorts its tile in LDS by
 *    material and energy and looks it up; a request's time runs from its
 *    first tile's start to its last tile's end.
 * Times come from the device wall clock.  d_ws: DEVICE, 256-byte aligned,
 * at least xs_requests_workspace_size(...) bytes for the same requests and
 * params; it holds the descriptors and times until xs_requests_stats reads
 * them.  Results equal xs_lookup_batch's on each request bit for bit.
 * Errors: XS_EINVAL (count outside [1, 2^24], a request with n < 0 or
 * n >= 2^31, NULL pointers in a non-empty request, a total of 2^31 lookups
 * or more), XS_EWORKSPACE, XS_ENOTBUILT (grid or precision not built). */
xs_status xs_lookup_requests(xs_tables_t tables, const xs_request* reqs,
                             int32_t count, const xs_params* params,
                             void* d_ws, size_t ws_bytes, void* stream);

/* Workspace bytes xs_lookup_requests needs for these requests and params. */
xs_status xs_requests_workspace_size(xs_tables_t tables, const xs_request* reqs,
                                     int32_t count, const xs_params* params,
                                     size_t* bytes);

/* Synchronises `stream` and reads the per-request times of the last
 * xs_lookup_requests call that used d_ws (stats[count] may be NULL). */
xs_status xs_requests_stats(const void* d_ws, int32_t count, void* stream,
                            xs_request_stats* stats, double* makespan_us);

/* ---- a toy event loop around the lookup ---------------------------------- */

/* The shape of the paper's event-based transport (section 5.1): a buffer of
 * n_slots particles in flight; each iteration looks up the live slots
 * (xs_lookup_active, so params' queue mode, sort policy and threshold
 * apply), then one kernel collides every live particle and refills dead
 * slots from the source until n_histories histories have run.  The
 * collision uses the first two channels S0, S1 and three uniform numbers
 * u0..u2 of (seed, history, collision) from SplitMix64 at counter
 * history * 2^20 + collision * 4 + draw:
 *   absorbed (fate 1)              if u0 * (S0 + S1) < 0.25 * S1
 *   else E' = E * (0.2 + 0.8 * u1); cut off (fate 2) if E' < e_cut;
 *   collision limit (fate 3)       at collision 2^18 - 1;
 *   else m' = min(floor((u2 * 5) * M), M - 1) when u2 < 0.2.
 * A source particle of history h has E = 0.01 + 0.99 * v0 and
 * m = min(floor(v1 * M), M - 1), v = the draws of collision 0.  All of it is
 * FP64 +, -, * and compares, so each history's outcome is exact and does
 * not depend on the slot or iteration that ran it. */
typedef struct {
  int64_t n_slots;         /* particles in flight, 1 .. 2^31 - 1 */
  int64_t n_histories;     /* histories to run, 0 .. 2^40 */
  uint64_t seed;
  double e_cut;            /* > 0 */
  int32_t check_every;     /* iterations between completion checks, >= 1 */
  int32_t max_iterations;  /* bound on iterations, >= 1 */
} xs_event_config;

typedef struct {           /* DEVICE buffers owned by the caller */
  double* E;               /* [n_slots] */
  int32_t* mat;            /* [n_slots] */
  uint8_t* alive;          /* [n_slots] */
  int64_t* hist;           /* [n_slots] history of the slot */
  int32_t* ncoll;          /* [n_slots] collisions so far */
  void* sigma;             /* [n_slots][5] of the lookup precision */
  int64_t* counters;       /* [3]: next history, finished, lookups run */
  int32_t* t_collisions;   /* [n_histories] collisions of each history */
  double* t_energy;        /* [n_histories] energy at its end */
  uint8_t* t_fate;         /* [n_histories] 1 absorbed, 2 cut off, 3 limit */
} xs_event_buffers;

typedef struct {
  int64_t iterations;      /* event iterations run */
  int64_t lookups;         /* (particle, iteration) lookups */
  int64_t histories;       /* histories finished */
} xs_event_result;

/* Workspace for xs_event_run (that of n_slots lookups with params). */
xs_status xs_event_workspace_size(xs_tables_t tables, const xs_event_config* cfg,
                                  const xs_params* params, size_t* bytes);

/* Runs the loop on `stream` until every history has finished, reading the
 * finished count to the host every check_every iterations (the paper's
 * queue-count transfer).  XS_ETIMEOUT if max_iterations pass first (the
 * tallies of finished histories are valid); XS_EINVAL for bad sizes or NULL
 * buffers. */
xs_status xs_event_run(xs_tables_t tables, const xs_event_config* cfg,
                       const xs_event_buffers* bufs, const xs_params* params,
                       void* d_ws, size_t ws_bytes, void* stream,
                       xs_event_result* result);

/* ---- measurement --------------------------------------------------------- */

/* Starts recording per-stage HIP events for subsequent lookup calls on this
 * handle (adds two events per stage per call). */
xs_status xs_profile_begin(xs_tables_t tables);

/* Synchronises the recorded events, sums them into *out and stops
 * recording. */
xs_status xs_profile_end(xs_tables_t tables, xs_profile_t* out);

/* ---- debug mode ---------------------------------------------------------- */

/* Counters of debug mode (all 0 and on = 0 while it is off). */
typedef struct {
  int32_t on;
  int32_t reserved;
  int64_t calls;              /* lookup calls checked since it was switched on */
  int64_t invalid_queries;    /* invalid queries those calls met */
  int64_t hash_bin_scans;     /* hash-grid searches whose fast two-interval
                                 window missed, so the bin was scanned */
  int64_t hash_full_searches; /* of those, searches whose verify failed (the
                                 rounding of log put E in a neighbouring bin)
                                 and that bisected the whole grid */
} xs_debug_info;

/* Switches debug mode of the handle on (1) or off (0); off at creation;
 * switching on clears the counters.  Call it while no work on the handle is
 * in flight: it synchronises the device.  While on:
 *  - xs_lookup_batch, xs_lookup_active and xs_lookup_indices (and what runs
 *    through them: xs_lookup_requests with a sort, xs_event_run) count the
 *    call's invalid queries (E not finite or <= 0, material outside
 *    [0, n_materials); inactive slots excluded), wait for the stream, and
 *    return XS_EINVAL naming their number and the first position when there
 *    are any; the results are written as usual (NaN rows, -1 indices).
 *    Debug calls cannot be captured into a graph (they synchronise);
 *  - every hash-grid search counts how often it left the fast window and how
 *    often it fell back to a full bisection (section 5.1's hash grid trades
 *    bins for search length; these counters show that trade directly). */
xs_status xs_set_debug(xs_tables_t tables, int32_t on);

/* Reads the counters (synchronises the device). */
xs_status xs_debug_counters(xs_tables_t tables, xs_debug_info* out);

/* ---- errors ------------------------------------------------------------ */

const char* xs_status_string(xs_status status);

/* Message describing the last error on the calling thread ("" if none). */
const char* xs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* XS_H */
