// Autotuner for the lookup's launch and method parameters (xs_tune,
// xs_tune_search, xs_set_tuned).
//
// The paper tunes OpenMC's particles in flight, hash-bin count, queue mode
// and sorting threshold with ytopt (section 2.1): Bayesian optimisation with
// a random-forest surrogate of the objective and the lower-confidence-bound
// acquisition a(x) = mu(x) - kappa sigma(x) (Eq. 1, kappa = 1.96 by default),
// evaluating one configuration at a time or a batch per refit (section 3,
// Steps 1-5).  An evaluation that runs longer than 1.5x the baseline
// runtime is stopped and the time-out value is recorded as its objective
// (section 3, last paragraph).  Parameters that only matter under another
// parameter's value are conditional (the paper's ConfigSpace condition, as
// in section 5.2): the hash-bin count is active only under the hash grid,
// the sort threshold only under a sort policy, the queue mode only for the
// entry point that has one (xs_lookup_active).
//
// Here the space is the lookup's own: grid method (x the hash grids built)
// x sort policy (x threshold) x block size x (lookups per lane, nuclides in
// flight, LDS staging, wave per lookup) (x queue mode), with invalid
// combinations removed.  Configurations that launch the same kernels at the
// tuned batch size (a threshold on either side of n, a queue mode behind a
// sort) share one device measurement.  The best few are timed again,
// interleaved, before the winner is chosen.  Winners go into the handle per
// batch-size class and, with a cache path, into a text file keyed by device,
// table checksum, precision, entry point and class (the paper's performance
// database, section 3), from which later runs resolve without tuning.
#include <hip/hip_runtime_api.h>

#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "xs_internal.h"

namespace xs {
namespace {

// ---- the configuration space ---------------------------------------------

constexpr int kNumFeatures = 17;
constexpr int64_t kNever = std::numeric_limits<int64_t>::max();
// Sort thresholds on offer (paper Table 1: 0 = always sort, the default
// 20,000, infinity = never).
constexpr int64_t kThresholds[] = {0, 20000, kNever};

struct Cand {
  xs_params p;
  float f[kNumFeatures];
};

int max_block(int lpt, int unroll) {
  const int w = lpt * unroll;
  return w <= 1 ? 1024 : (w <= 4 ? 512 : 256);
}

float threshold_feature(int64_t t) {
  return t >= kNever ? 20.f : std::log10((float)t + 1.f);
}

// The space, with the paper's conditional parameters (section 5.2): the
// hash-bin count only under grid HASH, the sort threshold only under a sort
// policy, the queue mode only when xs_lookup_active is tuned.  Inactive
// parameters keep one fixed value.
std::vector<Cand> enumerate_space(int precision, uint32_t grids,
                                  uint32_t sorts,
                                  const std::vector<int32_t>& hash_bins,
                                  bool active) {
  static const int kBlocks[] = {64, 128, 256, 512, 1024};
  static const int kVariants[][2] = {{1, 1}, {2, 1}, {3, 1}, {4, 1}, {5, 1},
                                     {6, 1}, {7, 1}, {8, 1}, {1, 2}, {2, 2},
                                     {1, 4}, {2, 4}};
  constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
  const std::vector<int32_t> no_hash{0};
  std::vector<Cand> out;
  for (int g = 0; g < 3; ++g) {
    if (!(grids >> g & 1u)) continue;
    for (int32_t hb : g == XS_GRID_HASH ? hash_bins : no_hash) {
      for (int s = 0; s < 5; ++s) {
        if (!(sorts >> s & 1u)) continue;
        const int n_thr = s == XS_SORT_NONE ? 1 : 3;
        for (int ti = 0; ti < n_thr; ++ti) {
          const int64_t thr = s == XS_SORT_NONE ? kNever : kThresholds[ti];
          for (int q = 0; q < (active ? 2 : 1); ++q) {
            for (int b : kBlocks) {
              for (int vi = 0; vi < kNumVariants + 7; ++vi) {
                // then LDS staging in each of the three stage shapes with
                // one or two lookups per lane (one nuclide in flight), then
                // one wave per lookup
                const bool lds = vi >= kNumVariants && vi < kNumVariants + 6;
                const bool wave = vi == kNumVariants + 6;
                const int shape = lds ? (vi - kNumVariants) / 2 + 1 : 0;
                const int v[2] = {lds ? (vi - kNumVariants) % 2 + 1
                                      : (wave ? 1 : kVariants[vi][0]),
                                  lds || wave ? 1 : kVariants[vi][1]};
                if (b > (wave ? 256
                              : (lds ? 1024 / v[0] : max_block(v[0], v[1]))))
                  continue;
                Cand c{};
                c.p.precision = precision;
                c.p.grid = g;
                c.p.sort = s;
                c.p.block_size = b;
                c.p.lookups_per_thread = v[0];
                c.p.unroll = v[1];
                c.p.lds_stage = shape;
                c.p.wave_per_lookup = wave ? 1 : 0;
                c.p.sort_threshold = thr;
                c.p.queue = q;
                c.p.hash_bins = hb;
                for (int i = 0; i < 3; ++i) c.f[i] = g == i ? 1.f : 0.f;
                for (int i = 0; i < 5; ++i) c.f[3 + i] = s == i ? 1.f : 0.f;
                c.f[8] = std::log2((float)b);
                c.f[9] = (float)v[0];
                c.f[10] = (float)v[1];
                c.f[11] = (float)(v[0] * v[1]);
                c.f[12] = (float)shape;
                c.f[13] = wave ? 1.f : 0.f;
                c.f[14] = hb > 0 ? std::log2((float)hb) : 0.f;
                c.f[15] = threshold_feature(thr);
                c.f[16] = (float)q;
                out.push_back(c);
              }
            }
          }
        }
      }
    }
  }
  return out;
}

// The value an inactive parameter holds, so that configurations differing
// only there compare equal.
xs_params canonical(xs_params p, bool active) {
  if (p.grid != XS_GRID_HASH) p.hash_bins = 0;
  if (p.sort == XS_SORT_NONE) p.sort_threshold = kNever;
  if (!active) p.queue = XS_QUEUE_COMPACT;
  return p;
}

// Categorical dimensions of a candidate for the initial design: grid, sort,
// block size, lookups per lane, nuclides in flight, LDS staging, wave per
// lookup, hash bins, sort threshold, queue mode.
constexpr int kDesignDims = 10;

int64_t design_level(const xs_params& p, int d) {
  switch (d) {
    case 0: return p.grid;
    case 1: return p.sort;
    case 2: return p.block_size;
    case 3: return p.lookups_per_thread;
    case 4: return p.unroll;
    case 5: return p.lds_stage;
    case 6: return p.wave_per_lookup;
    case 7: return p.hash_bins;
    case 8: return p.sort_threshold;
    default: return p.queue;
  }
}

std::vector<std::vector<int64_t>> design_levels(const std::vector<Cand>& space) {
  std::vector<std::vector<int64_t>> lv(kDesignDims);
  for (const Cand& c : space)
    for (int d = 0; d < kDesignDims; ++d) {
      const int64_t v = design_level(c.p, d);
      if (std::find(lv[d].begin(), lv[d].end(), v) == lv[d].end())
        lv[d].push_back(v);
    }
  for (auto& l : lv) std::sort(l.begin(), l.end());
  return lv;
}

// ---- random numbers (SplitMix64) -------------------------------------------

struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  size_t below(size_t n) { return (size_t)(next() % n); }
};

// ---- random-forest regressor ---------------------------------------------
//
// Bootstrap-sampled CART trees grown on squared error (all features tried
// at every split, nodes under 6 samples stay leaves); the forest's mean is
// the prediction.

struct Node {
  int feature = -1;  // -1: leaf
  float threshold = 0.f;
  int left = -1, right = -1;
  double value = 0.0;  // mean of the node's training targets
  double var = 0.0;    // their variance
};

struct Tree {
  std::vector<Node> nodes;
  const Node& leaf(const float* x) const {
    int i = 0;
    while (nodes[i].feature >= 0)
      i = x[nodes[i].feature] <= nodes[i].threshold ? nodes[i].left
                                                     : nodes[i].right;
    return nodes[i];
  }
};

class Forest {
 public:
  Forest(int trees, int max_features, int max_depth, uint64_t seed)
      : trees_(trees), max_features_(max_features), max_depth_(max_depth),
        rng_{seed} {}

  void fit(const std::vector<const float*>& X, const std::vector<double>& y) {
    forest_.assign(trees_, Tree{});
    const size_t n = X.size();
    for (auto& t : forest_) {
      std::vector<size_t> idx(n);
      for (auto& i : idx) i = rng_.below(n);
      grow(t, X, y, idx, 0);
    }
  }

  // Mean over trees, and the standard deviation by the law of total
  // variance: the spread of the trees' leaf means plus the variance of the
  // targets inside each leaf (Hutter et al., "Algorithm runtime prediction",
  // 2014), so that leaves pooling unlike configurations stay uncertain.
  void predict(const float* x, double* mean, double* sd) const {
    double s = 0, s2 = 0;
    for (auto& t : forest_) {
      const Node& l = t.leaf(x);
      s += l.value;
      s2 += l.var + l.value * l.value;
    }
    const double m = s / forest_.size();
    *mean = m;
    *sd = std::sqrt(std::max(0.0, s2 / forest_.size() - m * m));
  }

 private:
  int grow(Tree& t, const std::vector<const float*>& X,
           const std::vector<double>& y, std::vector<size_t>& idx, int depth) {
    const int id = (int)t.nodes.size();
    t.nodes.emplace_back();
    double sum = 0, sum2 = 0;
    for (size_t i : idx) {
      sum += y[i];
      sum2 += y[i] * y[i];
    }
    const double mu = sum / idx.size();
    t.nodes[id].value = mu;
    t.nodes[id].var = std::max(0.0, sum2 / idx.size() - mu * mu);
    if (depth >= max_depth_ || idx.size() < 6) return id;

    // Random feature subset.
    int feats[kNumFeatures];
    std::iota(feats, feats + kNumFeatures, 0);
    for (int i = kNumFeatures - 1; i > 0; --i)
      std::swap(feats[i], feats[rng_.below(i + 1)]);

    double best_sse = std::numeric_limits<double>::infinity();
    int best_f = -1;
    float best_thr = 0.f;
    std::vector<std::pair<float, double>> v(idx.size());
    for (int fi = 0; fi < max_features_; ++fi) {
      const int f = feats[fi];
      for (size_t i = 0; i < idx.size(); ++i) v[i] = {X[idx[i]][f], y[idx[i]]};
      std::sort(v.begin(), v.end(),
                [](auto& a, auto& b) { return a.first < b.first; });
      double ls = 0, ls2 = 0, rs = 0, rs2 = 0;
      for (auto& e : v) {
        rs += e.second;
        rs2 += e.second * e.second;
      }
      for (size_t i = 0; i + 1 < v.size(); ++i) {
        ls += v[i].second;
        ls2 += v[i].second * v[i].second;
        rs -= v[i].second;
        rs2 -= v[i].second * v[i].second;
        if (v[i].first == v[i + 1].first) continue;
        const double nl = i + 1, nr = v.size() - i - 1;
        const double sse = (ls2 - ls * ls / nl) + (rs2 - rs * rs / nr);
        if (sse < best_sse) {
          best_sse = sse;
          best_f = f;
          best_thr = 0.5f * (v[i].first + v[i + 1].first);
        }
      }
    }
    if (best_f < 0) return id;
    std::vector<size_t> li, ri;
    for (size_t i : idx) (X[i][best_f] <= best_thr ? li : ri).push_back(i);
    if (li.empty() || ri.empty()) return id;
    const int l = grow(t, X, y, li, depth + 1);
    const int r = grow(t, X, y, ri, depth + 1);
    t.nodes[id].feature = best_f;
    t.nodes[id].threshold = best_thr;
    t.nodes[id].left = l;
    t.nodes[id].right = r;
    return id;
  }

  int trees_, max_features_, max_depth_;
  Rng rng_;
  std::vector<Tree> forest_;
};

bool same_choice(const xs_params& a, const xs_params& b) {
  return a.grid == b.grid && a.sort == b.sort && a.block_size == b.block_size &&
         a.lookups_per_thread == b.lookups_per_thread && a.unroll == b.unroll &&
         a.lds_stage == b.lds_stage && a.wave_per_lookup == b.wave_per_lookup &&
         a.hash_bins == b.hash_bins && a.sort_threshold == b.sort_threshold &&
         a.queue == b.queue;
}

// ---- the search ---------------------------------------------------------------

struct Search {
  const xs_tune_config& cfg;
  xs_eval_fn eval;
  void* user;
  std::vector<Cand> space;
  std::vector<double> obj;  // log(ms) objective per candidate (NaN = not run)
  std::vector<int> order;   // evaluation order
  double cutoff = std::numeric_limits<double>::infinity();
  int cut = 0;
  int best = -1;
  int best_eval = 0;

  xs_status run_one(int c) {
    double ms = 0;
    const xs_status st = eval(&space[c].p, cutoff, &ms, user);
    if (st != XS_OK) return st;
    if (!(ms > 0) || !std::isfinite(ms)) ms = cutoff;
    if (ms > cutoff) {
      ms = cutoff;  // the time-out value is the recorded objective
      ++cut;
    }
    obj[c] = std::log(ms);
    order.push_back(c);
    if (best < 0 || obj[c] < obj[best]) {
      best = c;
      best_eval = (int)order.size();
    }
    return XS_OK;
  }
};

}  // namespace
}  // namespace xs

using namespace xs;

extern "C" {

xs_status xs_tune_config_default(xs_tune_config* c) {
  clear_error();
  if (!c) return fail(XS_EINVAL, "config is NULL");
  std::memset(c, 0, sizeof(*c));
  c->precision = XS_FP64;
  c->strategy = XS_TUNE_FOREST;
  c->max_evals = 48;
  c->init_samples = 10;
  c->batch = 1;
  c->reps = 5;
  c->warmup = 1;
  c->timeout_factor = 1.5;
  c->kappa = 1.96;
  c->seed = 1234;
  c->grid_mask = 0;
  c->sort_mask = 0;
  c->confirm = 3;
  return XS_OK;
}

// The search; `baseline`, when given, is the configuration evaluated first
// (the time-out reference, and what the result can never be worse than).
// `round`, when given, is told the confirmation round before its runs (0, 1,
// ...) and -1 after the last, so an evaluator that reuses measurements can
// take fresh ones there.
static xs_status tune_search(uint32_t built_grids, const xs_tune_config* cfg,
                             xs_eval_fn eval, void* user,
                             const xs_params* baseline,
                             void (*round)(void* user, int r),
                             xs_tune_result* result) {
  clear_error();
  if (!cfg || !eval || !result)
    return fail(XS_EINVAL, "config, evaluator and result must not be NULL");
  if (cfg->precision != XS_FP64 && cfg->precision != XS_FP32)
    return fail(XS_EINVAL, "precision must be XS_FP64 or XS_FP32");
  if (cfg->strategy != XS_TUNE_EXHAUSTIVE && cfg->strategy != XS_TUNE_FOREST)
    return fail(XS_EINVAL, "unknown strategy %d", cfg->strategy);
  if (cfg->kappa < 0) return fail(XS_EINVAL, "kappa must be >= 0");
  if (cfg->active != 0 && cfg->active != 1)
    return fail(XS_EINVAL, "active must be 0 or 1");
  if (cfg->batch < 0) return fail(XS_EINVAL, "batch must be >= 0");
  if (cfg->confirm < 0 || cfg->confirm > 64)
    return fail(XS_EINVAL, "confirm must be in [0, 64]");
  if (cfg->grid_mask & ~7u) return fail(XS_EINVAL, "unknown grid mask bits");
  if (cfg->sort_mask & ~31u) return fail(XS_EINVAL, "unknown sort mask bits");
  if (cfg->n_hash_grids < 0 || cfg->n_hash_grids > XS_MAX_HASH_GRIDS)
    return fail(XS_EINVAL, "n_hash_grids must be in [0, %d]",
                XS_MAX_HASH_GRIDS);
  std::vector<int32_t> hash_bins;
  for (int i = 0; i < cfg->n_hash_grids; ++i) {
    const int32_t b = cfg->hash_bins[i];
    if (b < 1 || b > 100000 ||
        std::find(hash_bins.begin(), hash_bins.end(), b) != hash_bins.end())
      return fail(XS_EINVAL, "hash_bins must be distinct counts in [1, 100000]");
    hash_bins.push_back(b);
  }
  if (hash_bins.empty()) hash_bins.push_back(0);
  const bool active = cfg->active == 1;
  const uint32_t grids = (cfg->grid_mask ? cfg->grid_mask : 7u) & built_grids;
  const uint32_t sorts = cfg->sort_mask ? cfg->sort_mask : 31u;
  Search S{*cfg, eval, user,
           enumerate_space(cfg->precision, grids, sorts, hash_bins, active)};
  const int N = (int)S.space.size();
  if (N == 0) return fail(XS_EINVAL, "the parameter space is empty");
  S.obj.assign(N, std::numeric_limits<double>::quiet_NaN());

  // Baseline: the given configuration, else the library default for large
  // batches (hash grid if built, banded sort at the paper's threshold of
  // 20,000, block 256, one lookup per lane, two nuclides in flight, queued);
  // the first candidate if the space does not hold it.
  xs_params base{};
  if (baseline) {
    base = *baseline;
  } else {
    base.grid = (grids & 2u) ? XS_GRID_HASH
                             : ((grids & 1u) ? XS_GRID_NUCLIDE : XS_GRID_UNIONIZED);
    base.hash_bins = hash_bins[0];
    base.sort = (sorts & 16u) ? XS_SORT_BAND_MATERIAL : XS_SORT_NONE;
    base.sort_threshold = 20000;
    base.block_size = 256;
    base.lookups_per_thread = 1;
    base.unroll = 2;
    base.queue = XS_QUEUE_COMPACT;
  }
  base = canonical(base, active);
  int b0 = 0;
  for (int i = 0; i < N; ++i)
    if (same_choice(S.space[i].p, base)) b0 = i;
  if (xs_status st = S.run_one(b0)) return st;
  if (cfg->timeout_factor > 0)
    S.cutoff = cfg->timeout_factor * std::exp(S.obj[b0]);

  const int budget = cfg->strategy == XS_TUNE_EXHAUSTIVE || cfg->max_evals <= 0
                         ? N
                         : std::min(N, cfg->max_evals);
  Rng rng{cfg->seed};
  if (cfg->strategy == XS_TUNE_EXHAUSTIVE) {
    for (int i = 0; i < N && (int)S.order.size() < budget; ++i)
      if (std::isnan(S.obj[i]))
        if (xs_status st = S.run_one(i)) return st;
  } else {
    // Initial design, then surrogate-guided batches.  The initial
    // configurations form a Latin-hypercube draw over the categorical
    // dimensions (grid, sort, block, lookups per lane, nuclides in flight,
    // LDS staging): each dimension's levels are dealt out in a random order
    // so every level appears about equally often, and sample i takes the
    // unevaluated configuration that matches the most of its dealt levels
    // (ties at random).  A purely random draw of ten from ~750 often misses a
    // whole level (LDS staging is 10 % of the space), and a forest never
    // learns what a level it has not seen is worth.
    const int init = std::max(1, std::min(cfg->init_samples, budget));
    const std::vector<std::vector<int64_t>> levels = design_levels(S.space);
    std::vector<std::vector<int64_t>> deal(levels.size());
    for (size_t d = 0; d < levels.size(); ++d) {
      deal[d] = levels[d];
      for (size_t i = deal[d].size(); i > 1; --i)
        std::swap(deal[d][i - 1], deal[d][rng.below(i)]);
    }
    for (int k = 0; (int)S.order.size() < init; ++k) {
      int best = -1, best_match = -1;
      uint64_t best_tie = 0;
      for (int i = 0; i < N; ++i) {
        if (!std::isnan(S.obj[i])) continue;
        int match = 0;
        for (size_t d = 0; d < levels.size(); ++d)
          match += design_level(S.space[i].p, (int)d) ==
                   deal[d][k % deal[d].size()];
        const uint64_t tie = rng.next();
        if (match > best_match || (match == best_match && tie < best_tie)) {
          best = i;
          best_match = match;
          best_tie = tie;
        }
      }
      if (best < 0) break;
      if (xs_status st = S.run_one(best)) return st;
    }
    const int batch = std::max(1, cfg->batch);
    while ((int)S.order.size() < budget) {
      std::vector<const float*> X;
      std::vector<double> y;
      for (int c : S.order) {
        X.push_back(S.space[c].f);
        y.push_back(S.obj[c]);
      }
      Forest forest(64, kNumFeatures, 12, rng.next());
      forest.fit(X, y);
      std::vector<std::pair<double, int>> acq;
      for (int i = 0; i < N; ++i) {
        if (!std::isnan(S.obj[i])) continue;
        double mu, sd;
        forest.predict(S.space[i].f, &mu, &sd);
        acq.push_back({mu - cfg->kappa * sd, i});
      }
      if (acq.empty()) break;
      std::sort(acq.begin(), acq.end());
      const int take = std::min<int>({batch, (int)acq.size(),
                                      budget - (int)S.order.size()});
      for (int k = 0; k < take; ++k)
        if (xs_status st = S.run_one(acq[k].second)) return st;
    }
  }
  int win = S.best;
  double win_ms = std::exp(S.obj[S.best]);
  double base_ms = std::exp(S.obj[b0]);
  if (cfg->confirm >= 2 && S.order.size() >= 2) {
    // The finalists: the best `confirm` configurations by their search
    // score, then the baseline if it is not among them.  Each round times
    // every finalist once, starting one further along the list each round,
    // so slow drifts of clock or temperature fall on all of them alike; a
    // finalist's score is the median of its rounds (its search run, picked
    // for being low, is left out).  Ties keep the better-ranked finalist.
    constexpr int kRounds = 3;
    std::vector<int> fin = S.order;
    std::stable_sort(fin.begin(), fin.end(),
                     [&](int a, int b) { return S.obj[a] < S.obj[b]; });
    fin.resize(std::min<size_t>(fin.size(), (size_t)cfg->confirm));
    if (std::find(fin.begin(), fin.end(), b0) == fin.end()) fin.push_back(b0);
    const size_t F = fin.size();
    std::vector<std::vector<double>> t(F);
    for (int k = 0; k < kRounds; ++k) {
      if (round) round(user, k);
      for (size_t j = 0; j < F; ++j) {
        const size_t f = (j + (size_t)k) % F;
        double ms = 0;
        if (xs_status st = eval(&S.space[fin[f]].p, S.cutoff, &ms, user)) {
          if (round) round(user, -1);
          return st;
        }
        if (!(ms > 0) || !std::isfinite(ms) || ms > S.cutoff) ms = S.cutoff;
        t[f].push_back(ms);
      }
    }
    if (round) round(user, -1);
    std::vector<double> med(F);
    for (size_t f = 0; f < F; ++f) {
      std::sort(t[f].begin(), t[f].end());
      med[f] = t[f][kRounds / 2];
    }
    size_t w = 0;
    for (size_t f = 1; f < F; ++f)
      if (med[f] < med[w]) w = f;
    win = fin[w];
    win_ms = med[w];
    base_ms = med[std::find(fin.begin(), fin.end(), b0) - fin.begin()];
  }
  xs_tune_result r{};
  r.best = S.space[win].p;
  r.best_ms = win_ms;
  r.baseline = S.space[b0].p;
  r.baseline_ms = base_ms;
  r.evaluated = (int)S.order.size();
  r.cut = S.cut;
  r.space_size = N;
  r.best_eval =
      (int)(std::find(S.order.begin(), S.order.end(), win) - S.order.begin()) + 1;
  *result = r;
  return XS_OK;
}

xs_status xs_tune_search(uint32_t built_grids, const xs_tune_config* cfg,
                         xs_eval_fn eval, void* user, xs_tune_result* result) {
  return tune_search(built_grids, cfg, eval, user, nullptr, nullptr, result);
}

}  // extern "C"

namespace xs {
namespace {

// Times xs_lookup_batch (or xs_lookup_active) with HIP events on the
// caller's stream: `warmup` untimed runs, then up to `reps` timed runs (best
// kept); stops after the first timed run when it already exceeds the
// cut-off.  Configurations that launch the same kernels at this n share one
// measurement (within the search, and within each confirmation round).
struct DeviceEval {
  xs_tables_t h;
  int64_t n;
  const double* E;
  const int32_t* mat;
  const uint8_t* active;  // null: xs_lookup_batch
  void* out;
  void* ws;
  size_t ws_bytes;
  hipStream_t s;
  int warmup, reps;
  hipEvent_t a, b;
  std::map<std::vector<int64_t>, double> memo;
  int measured = 0;
  int round = -1;  // confirmation round, -1 during the search

  // What decides the kernels a call runs at this n.
  std::vector<int64_t> launch_key(const xs_params& p) const {
    const bool sorted = p.sort != XS_SORT_NONE && n >= p.sort_threshold;
    return {p.grid, p.grid == XS_GRID_HASH ? p.hash_bins : 0,
            sorted ? p.sort : XS_SORT_NONE, p.block_size,
            p.lookups_per_thread, p.unroll, p.lds_stage, p.wave_per_lookup,
            active && !sorted ? p.queue : 0};
  }

  xs_status call(const xs_params* p) {
    return active ? xs_lookup_active(h, n, E, mat, active, out, p, ws,
                                     ws_bytes, s)
                  : xs_lookup_batch(h, n, E, mat, out, p, ws, ws_bytes, s);
  }
};

void device_round(void* user, int r) { ((DeviceEval*)user)->round = r; }

int32_t device_eval(const xs_params* p, double cutoff_ms, double* ms,
                    void* user) {
  DeviceEval& d = *(DeviceEval*)user;
  std::vector<int64_t> key = d.launch_key(*p);
  key.push_back(d.round);  // each confirmation round measures afresh
  auto it = d.memo.find(key);
  if (it != d.memo.end()) {
    *ms = it->second;
    return XS_OK;
  }
  for (int i = 0; i < d.warmup; ++i)
    if (xs_status st = d.call(p)) return st;
  double best = std::numeric_limits<double>::infinity();
  for (int i = 0; i < std::max(1, d.reps); ++i) {
    XS_HIP(hipEventRecord(d.a, d.s));
    if (xs_status st = d.call(p)) return st;
    XS_HIP(hipEventRecord(d.b, d.s));
    XS_HIP(hipEventSynchronize(d.b));
    float t = 0;
    XS_HIP(hipEventElapsedTime(&t, d.a, d.b));
    best = std::min(best, (double)t);
    if (best > cutoff_ms) break;
  }
  if (d.round < 0) ++d.measured;
  d.memo[key] = best;
  *ms = best;
  return XS_OK;
}

// ---- the tuned-parameter file ----------------------------------------------
//
// Text, one entry per line, tab-separated:
//   device, table checksum (16 hex digits), precision, entry point (0 batch,
//   1 active), size class, the ten parameters (grid sort block_size
//   lookups_per_thread lds_stage sort_threshold queue unroll wave_per_lookup
//   hash_bins, space-separated), best time in ms.
// Lines starting with '#' and lines that do not parse are ignored.

constexpr const char* kCacheHeader =
    "# xs tuned parameters: device\tchecksum\tprecision\tactive\tsize class"
    "\tgrid sort block lookups_per_thread lds_stage sort_threshold queue "
    "unroll wave_per_lookup hash_bins\tbest ms";

struct CacheEntry {
  xs_tune_key key;
  xs_params p;
  double best_ms;
};

bool same_key(const xs_tune_key& a, const xs_tune_key& b) {
  return std::strncmp(a.device, b.device, sizeof(a.device)) == 0 &&
         a.checksum == b.checksum && a.precision == b.precision &&
         a.active == b.active && a.size_class == b.size_class;
}

std::vector<std::string> split(const std::string& s, char sep) {
  std::vector<std::string> out;
  size_t a = 0;
  for (;;) {
    const size_t b = s.find(sep, a);
    out.push_back(s.substr(a, b == std::string::npos ? std::string::npos : b - a));
    if (b == std::string::npos) break;
    a = b + 1;
  }
  return out;
}

bool parse_i64(const std::string& s, int64_t* v, int base = 10) {
  if (s.empty()) return false;
  errno = 0;
  char* end = nullptr;
  const long long x = base == 16 ? (long long)std::strtoull(s.c_str(), &end, 16)
                                 : std::strtoll(s.c_str(), &end, 10);
  if (errno != 0 || *end != '\0') return false;
  *v = (int64_t)x;
  return true;
}

bool parse_line(const std::string& line, CacheEntry* e) {
  if (line.empty() || line[0] == '#') return false;
  const std::vector<std::string> f = split(line, '\t');
  if (f.size() != 7 || f[0].empty() || f[0].size() >= sizeof(e->key.device))
    return false;
  CacheEntry r{};
  std::memcpy(r.key.device, f[0].data(), f[0].size());
  int64_t v[4];
  if (f[1].size() != 16 || !parse_i64(f[1], &v[0], 16)) return false;
  r.key.checksum = (uint64_t)v[0];
  if (!parse_i64(f[2], &v[1]) || !parse_i64(f[3], &v[2]) ||
      !parse_i64(f[4], &v[3]))
    return false;
  if ((v[1] != 0 && v[1] != 1) || (v[2] != 0 && v[2] != 1) || v[3] < 0 ||
      v[3] >= kBuckets)
    return false;
  r.key.precision = (int32_t)v[1];
  r.key.active = (int32_t)v[2];
  r.key.size_class = (int32_t)v[3];
  const std::vector<std::string> q = split(f[5], ' ');
  if (q.size() != 10) return false;
  int64_t x[10];
  for (int i = 0; i < 10; ++i)
    if (!parse_i64(q[i], &x[i])) return false;
  for (int i = 0; i < 10; ++i)
    if (i != 5 && (x[i] < INT32_MIN || x[i] > INT32_MAX)) return false;
  r.p.precision = r.key.precision;
  r.p.grid = (int32_t)x[0];
  r.p.sort = (int32_t)x[1];
  r.p.block_size = (int32_t)x[2];
  r.p.lookups_per_thread = (int32_t)x[3];
  r.p.lds_stage = (int32_t)x[4];
  r.p.sort_threshold = x[5];
  r.p.queue = (int32_t)x[6];
  r.p.unroll = (int32_t)x[7];
  r.p.wave_per_lookup = (int32_t)x[8];
  r.p.hash_bins = (int32_t)x[9];
  char* end = nullptr;
  r.best_ms = std::strtod(f[6].c_str(), &end);
  if (*end != '\0' || !(r.best_ms >= 0) || !std::isfinite(r.best_ms))
    return false;
  *e = r;
  return true;
}

std::string format_line(const CacheEntry& e) {
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "%s\t%016llx\t%d\t%d\t%d\t%d %d %d %d %d %lld %d %d %d %d\t%.6g",
                e.key.device, (unsigned long long)e.key.checksum,
                e.key.precision, e.key.active, e.key.size_class, e.p.grid,
                e.p.sort, e.p.block_size, e.p.lookups_per_thread, e.p.lds_stage,
                (long long)e.p.sort_threshold, e.p.queue, e.p.unroll,
                e.p.wave_per_lookup, e.p.hash_bins, e.best_ms);
  return buf;
}

// Reads every parsable entry; false when the file cannot be opened.
bool read_cache(const char* path, std::vector<CacheEntry>* out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string line;
  char buf[1024];
  while (std::fgets(buf, sizeof(buf), f)) {
    line += buf;
    if (line.empty() || line.back() != '\n') {
      if (!std::feof(f)) continue;  // longer than the buffer: keep reading
    }
    while (!line.empty() && (line.back() == '\n' || line.back() == '\r'))
      line.pop_back();
    CacheEntry e;
    if (parse_line(line, &e)) out->push_back(e);
    line.clear();
  }
  std::fclose(f);
  return true;
}

// Adds or replaces entries, rewriting the file through a temporary file in
// the same directory and a rename.
xs_status write_cache(const char* path, const std::vector<CacheEntry>& add) {
  std::vector<CacheEntry> all;
  read_cache(path, &all);
  for (const CacheEntry& e : add) {
    all.erase(std::remove_if(all.begin(), all.end(),
                             [&](const CacheEntry& o) {
                               return same_key(o.key, e.key);
                             }),
              all.end());
    all.push_back(e);
  }
  static std::atomic<unsigned> counter{0};
  const std::string tmp = std::string(path) + ".tmp." +
                          std::to_string((long long)getpid()) + "." +
                          std::to_string(counter.fetch_add(1));
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(XS_EINVAL, "cannot write the tuning cache %s: %s", path,
                      std::strerror(errno));
  bool ok = std::fprintf(f, "%s\n", kCacheHeader) > 0;
  for (const CacheEntry& e : all)
    ok = ok && std::fprintf(f, "%s\n", format_line(e).c_str()) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    const int err = errno;
    std::remove(tmp.c_str());
    return fail(XS_EINVAL, "cannot write the tuning cache %s: %s", path,
                std::strerror(err));
  }
  return XS_OK;
}

xs_status make_key(xs_tables_t h, int32_t precision, int32_t active,
                   int64_t n, xs_tune_key* key) {
  hipDeviceProp_t prop;
  XS_HIP(hipGetDeviceProperties(&prop, h->device));
  xs_tune_key k{};
  std::snprintf(k.device, sizeof(k.device), "%s|%s|%dCU", prop.name,
                prop.gcnArchName, prop.multiProcessorCount);
  for (char* c = k.device; *c; ++c)
    if (*c == '\t' || *c == '\n' || *c == '\r') *c = ' ';
  k.checksum = h->info.checksum;
  k.precision = precision;
  k.active = active;
  k.size_class = size_class(n);
  *key = k;
  return XS_OK;
}

void record_tuned(xs_tables_t h, int active, int64_t n, const xs_params& p) {
  std::lock_guard<std::mutex> lk(h->mu);
  h->tuned[active][p.precision][size_class(n)] = p;
  h->tuned_valid[active][p.precision][size_class(n)] = true;
}

// Checks that p is complete (no automatic field) and runs on this handle.
xs_status check_complete(xs_tables_t h, int64_t n, int active,
                         const xs_params& p, xs_params* checked) {
  if (p.grid == XS_AUTO || p.sort == XS_AUTO || p.block_size <= 0 ||
      p.lookups_per_thread <= 0 || p.lds_stage == XS_AUTO ||
      p.sort_threshold < 0 || p.queue == XS_AUTO || p.unroll <= 0 ||
      p.wave_per_lookup == XS_AUTO ||
      (p.grid == XS_GRID_HASH && p.hash_bins <= 0))
    return fail(XS_EINVAL, "tuned parameters must not contain automatic fields");
  return resolve_for(h, n, active, &p, checked);
}

}  // namespace
}  // namespace xs

extern "C" {

xs_status xs_tune(xs_tables_t h, const xs_tune_request* req,
                  xs_tune_result* results) {
  clear_error();
  if (!h) return fail(XS_EINVAL, "table handle is NULL");
  if (!req || !results) return fail(XS_EINVAL, "request and results must not be NULL");
  const xs_tune_config& cfg0 = req->config;
  if (req->reserved != 0) return fail(XS_EINVAL, "reserved field must be 0");
  if (req->n_sizes < 1 || req->n_sizes > 64 || !req->sizes)
    return fail(XS_EINVAL, "n_sizes must be in [1, 64] and sizes not NULL");
  if (cfg0.active != 0 && cfg0.active != 1)
    return fail(XS_EINVAL, "config.active must be 0 or 1");
  const bool active = cfg0.active == 1;
  int64_t n_max = 0;
  for (int i = 0; i < req->n_sizes; ++i) {
    if (req->sizes[i] < 1 || req->sizes[i] > 0x7fffffffLL)
      return fail(XS_EINVAL, "sizes[%d] out of [1, 2^31 - 1]", i);
    n_max = std::max(n_max, req->sizes[i]);
  }
  if (!req->d_E || !req->d_mat || !req->d_out)
    return fail(XS_EINVAL, "a query or output pointer is NULL");
  if (active != (req->d_active != nullptr))
    return fail(XS_EINVAL, "d_active must be given exactly when config.active "
                "is 1");
  if (cfg0.precision != XS_FP64 && cfg0.precision != XS_FP32)
    return fail(XS_EINVAL, "precision must be XS_FP64 or XS_FP32");
  if (cfg0.precision == XS_FP32 && !h->d.rec32)
    return fail(XS_ENOTBUILT, "FP32 tables were not built");
  {
    // The workspace must fit the most demanding candidate (a sort).
    xs_params probe;
    xs_params_default(&probe, cfg0.precision);
    probe.sort = XS_SORT_BAND_MATERIAL;
    probe.sort_threshold = 0;
    probe.grid = XS_GRID_NUCLIDE;
    size_t need = 0;
    if (xs_status st = xs_workspace_size(h, n_max, &probe, &need)) return st;
    if (!req->d_ws || req->ws_bytes < need)
      return fail(XS_EWORKSPACE, "tuning needs a workspace of %zu bytes", need);
  }
  // The space offers every hash grid of the handle.
  xs_tune_config cfg = cfg0;
  cfg.n_hash_grids = (int32_t)h->hash.size();
  for (size_t i = 0; i < h->hash.size(); ++i) cfg.hash_bins[i] = h->hash[i].B;
  uint32_t built = 1u;
  if (h->d.B > 0) built |= 2u;
  if (h->d.U > 0) built |= 4u;

  std::vector<xs_tune_result> out(req->n_sizes);
  std::vector<CacheEntry> fresh;
  std::vector<CacheEntry> cached;
  if (req->cache_path) read_cache(req->cache_path, &cached);
  DeviceEval d{h, 0, req->d_E, req->d_mat, req->d_active, req->d_out,
               req->d_ws, req->ws_bytes, (hipStream_t)req->stream,
               std::max(0, cfg.warmup), std::max(1, cfg.reps), nullptr,
               nullptr, {}, 0, -1};
  XS_HIP(hipEventCreate(&d.a));
  XS_HIP(hipEventCreate(&d.b));
  xs_status st = XS_OK;
  for (int i = 0; i < req->n_sizes && st == XS_OK; ++i) {
    const int64_t n = req->sizes[i];
    xs_tune_key key;
    if ((st = make_key(h, cfg.precision, cfg.active, n, &key))) break;
    xs_params def;
    untuned_defaults(h, n, cfg.precision, &def);
    xs_tune_result r{};
    bool hit = false;
    for (const CacheEntry& e : cached) {
      xs_params checked;
      if (!same_key(e.key, key)) continue;
      if (check_complete(h, n, cfg.active, e.p, &checked) != XS_OK) continue;
      r.best = checked;
      r.best_ms = e.best_ms;
      hit = true;
    }
    clear_error();
    if (hit) {
      r.baseline = def;
      r.baseline_ms = std::numeric_limits<double>::quiet_NaN();
      r.from_cache = 1;
    } else {
      // The untuned default for this batch is the baseline, so tuning never
      // returns anything slower than what an untuned call would run.
      d.n = n;
      d.memo.clear();
      d.measured = 0;
      if ((st = tune_search(built, &cfg, device_eval, &d, &def, device_round,
                            &r)))
        break;
      r.measured = d.measured;
      fresh.push_back(CacheEntry{key, r.best, r.best_ms});
    }
    r.n = n;
    record_tuned(h, cfg.active, n, r.best);
    out[i] = r;
  }
  (void)hipEventDestroy(d.a);
  (void)hipEventDestroy(d.b);
  if (st != XS_OK) return st;
  std::copy(out.begin(), out.end(), results);
  if (req->cache_path && !fresh.empty())
    if (xs_status w = write_cache(req->cache_path, fresh)) return w;
  return XS_OK;
}

xs_status xs_set_tuned(xs_tables_t h, int64_t n, int32_t active,
                       const xs_params* p) {
  clear_error();
  if (!h) return fail(XS_EINVAL, "table handle is NULL");
  if (n <= 0) return fail(XS_EINVAL, "n must be > 0");
  if (active != 0 && active != 1) return fail(XS_EINVAL, "active must be 0 or 1");
  if (!p) {
    std::lock_guard<std::mutex> lk(h->mu);
    for (int a = 0; a < 2; ++a)
      for (int prec = 0; prec < 2; ++prec)
        for (int b = 0; b < kBuckets; ++b) h->tuned_valid[a][prec][b] = false;
    return XS_OK;
  }
  xs_params checked;
  if (xs_status st = check_complete(h, n, active, *p, &checked)) return st;
  record_tuned(h, active, n, checked);
  return XS_OK;
}

xs_status xs_tune_load(xs_tables_t h, const char* path, int32_t* loaded) {
  clear_error();
  if (!h || !path) return fail(XS_EINVAL, "tables and path must not be NULL");
  std::vector<CacheEntry> all;
  read_cache(path, &all);
  xs_tune_key mine;
  if (xs_status st = make_key(h, 0, 0, 1, &mine)) return st;
  int32_t count = 0;
  for (const CacheEntry& e : all) {
    if (std::strncmp(e.key.device, mine.device, sizeof(mine.device)) != 0 ||
        e.key.checksum != mine.checksum)
      continue;
    const int64_t n = (int64_t)1 << e.key.size_class;
    xs_params checked;
    if (check_complete(h, n, e.key.active, e.p, &checked) != XS_OK) continue;
    record_tuned(h, e.key.active, n, checked);
    ++count;
  }
  clear_error();
  if (loaded) *loaded = count;
  return XS_OK;
}

xs_status xs_tune_key_of(xs_tables_t h, int32_t precision, int32_t active,
                         int64_t n, xs_tune_key* key) {
  clear_error();
  if (!h || !key) return fail(XS_EINVAL, "tables and key must not be NULL");
  if ((precision != XS_FP64 && precision != XS_FP32) ||
      (active != 0 && active != 1) || n < 1)
    return fail(XS_EINVAL, "precision, active or n out of range");
  return make_key(h, precision, active, n, key);
}

xs_status xs_tune_cache_get(const char* path, const xs_tune_key* key,
                            xs_params* p, double* best_ms) {
  clear_error();
  if (!path || !key || !p) return fail(XS_EINVAL, "a pointer is NULL");
  std::vector<CacheEntry> all;
  if (!read_cache(path, &all))
    return fail(XS_ENOTBUILT, "no tuning cache at %s", path);
  const CacheEntry* hit = nullptr;
  for (const CacheEntry& e : all)
    if (same_key(e.key, *key)) hit = &e;
  if (!hit) return fail(XS_ENOTBUILT, "no entry for this key in %s", path);
  *p = hit->p;
  if (best_ms) *best_ms = hit->best_ms;
  return XS_OK;
}

xs_status xs_tune_cache_put(const char* path, const xs_tune_key* key,
                            const xs_params* p, double best_ms) {
  clear_error();
  if (!path || !key || !p) return fail(XS_EINVAL, "a pointer is NULL");
  if (key->precision != p->precision || key->size_class < 0 ||
      key->size_class >= kBuckets || (key->active != 0 && key->active != 1))
    return fail(XS_EINVAL, "key and parameters disagree or are out of range");
  if (!(best_ms >= 0) || !std::isfinite(best_ms))
    return fail(XS_EINVAL, "best_ms must be finite and >= 0");
  const size_t len = strnlen(key->device, sizeof(key->device));
  if (len == 0 || len >= sizeof(key->device))
    return fail(XS_EINVAL, "device name empty or not terminated");
  for (size_t i = 0; i < len; ++i)
    if (key->device[i] == '\t' || key->device[i] == '\n' ||
        key->device[i] == '\r')
      return fail(XS_EINVAL, "device name holds a tab or line break");
  CacheEntry e{*key, *p, best_ms};
  return write_cache(path, {e});
}

}  // extern "C"
