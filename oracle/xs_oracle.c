/*
 * Serial CPU oracle for the batched macroscopic cross-section lookup.
 * TEST INFRASTRUCTURE ONLY: see xs_oracle.h for what it computes, the
 * readings of the paper it takes and the pins that check it.
 *
 * Section 5.1 of the paper (the hash-bin paragraph after Table 1) describes
 * the operation: each nuclide of the particle's material is searched for the
 * current energy, and the macroscopic value combines the nuclides of that
 * material.  Everything here is the plain definition, written out step by
 * step, with no blocking, reordering or fused arithmetic.
 */
#include "xs_oracle.h"

#include <math.h>

int64_t xso_bracket_count(const double* grid, int64_t n, double e) {
  int64_t count = 0;
  for (int64_t p = 0; p < n; ++p)
    if (grid[p] <= e) ++count;
  int64_t i = count - 1;
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  return i;
}

int64_t xso_bracket_bisect(const double* grid, int64_t n, double e) {
  /* first position whose point is > e; that position equals the count */
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (grid[mid] <= e)
      lo = mid + 1;
    else
      hi = mid;
  }
  int64_t i = lo - 1;
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  return i;
}

static int valid_query(const xso_tables* t, double e, int32_t m) {
  return isfinite(e) && e > 0.0 && m >= 0 && m < t->n_materials;
}

int xso_lookup(const xso_tables* t, double e, int32_t m, int search,
               double out[XSO_CHANNELS], int32_t* idx) {
  if (!valid_query(t, e, m)) {
    for (int c = 0; c < XSO_CHANNELS; ++c) out[c] = NAN;
    if (idx && m >= 0 && m < t->n_materials)
      for (int32_t j = t->mat_offsets[m]; j < t->mat_offsets[m + 1]; ++j)
        idx[j - t->mat_offsets[m]] = -1;
    return -1;
  }
  double sum[XSO_CHANNELS];
  for (int c = 0; c < XSO_CHANNELS; ++c) sum[c] = 0.0;

  const int32_t first = t->mat_offsets[m], last = t->mat_offsets[m + 1];
  for (int32_t j = first; j < last; ++j) {
    const int32_t k = t->mat_nuclides[j];
    const double rho = t->mat_density[j];
    const int64_t base = t->grid_offsets[k];
    const int64_t n = t->grid_offsets[k + 1] - base;
    const double* grid = t->energy + base;

    const int64_t i = search ? xso_bracket_count(grid, n, e)
                             : xso_bracket_bisect(grid, n, e);
    if (idx) idx[j - first] = (int32_t)i;

    double eh = e;
    if (eh < grid[0]) eh = grid[0];
    if (eh > grid[n - 1]) eh = grid[n - 1];
    const double f = (eh - grid[i]) / (grid[i + 1] - grid[i]);
    const double g = 1.0 - f;

    const double* lo = t->xs + (base + i) * XSO_CHANNELS;
    const double* hi = lo + XSO_CHANNELS;
    for (int c = 0; c < XSO_CHANNELS; ++c) {
      const double a = g * lo[c];
      const double b = f * hi[c];
      const double sigma = a + b;
      const double term = rho * sigma;
      sum[c] = sum[c] + term;
    }
  }
  for (int c = 0; c < XSO_CHANNELS; ++c) out[c] = sum[c];
  return 0;
}

int64_t xso_lookup_batch(const xso_tables* t, int64_t n, const double* e,
                         const int32_t* m, int search, double* out,
                         const int64_t* idx_offsets, int32_t* idx) {
  int64_t bad = 0;
  for (int64_t q = 0; q < n; ++q) {
    int32_t* iq = idx ? idx + idx_offsets[q] : 0;
    if (xso_lookup(t, e[q], m[q], search, out + q * XSO_CHANNELS, iq) != 0)
      ++bad;
  }
  return bad;
}

int64_t xso_lookup_batch_f32(const xso_tables* t, int64_t n, const double* e,
                             const int32_t* m, float* out) {
  int64_t bad = 0;
  for (int64_t q = 0; q < n; ++q) {
    float* o = out + q * XSO_CHANNELS;
    if (!valid_query(t, e[q], m[q])) {
      for (int c = 0; c < XSO_CHANNELS; ++c) o[c] = NAN;
      ++bad;
      continue;
    }
    float sum[XSO_CHANNELS], comp[XSO_CHANNELS];
    for (int c = 0; c < XSO_CHANNELS; ++c) {
      sum[c] = 0.0f;
      comp[c] = 0.0f;
    }
    const int32_t first = t->mat_offsets[m[q]], last = t->mat_offsets[m[q] + 1];
    for (int32_t j = first; j < last; ++j) {
      const int32_t k = t->mat_nuclides[j];
      const float rho = (float)t->mat_density[j];
      const int64_t base = t->grid_offsets[k];
      const int64_t nk = t->grid_offsets[k + 1] - base;
      const double* grid = t->energy + base;
      const int64_t i = xso_bracket_bisect(grid, nk, e[q]);
      double eh = e[q];
      if (eh < grid[0]) eh = grid[0];
      if (eh > grid[nk - 1]) eh = grid[nk - 1];
      const double f = (eh - grid[i]) / (grid[i + 1] - grid[i]);
      const float f32 = (float)f;
      const float g32 = (float)(1.0 - f);
      const double* lo = t->xs + (base + i) * XSO_CHANNELS;
      const double* hi = lo + XSO_CHANNELS;
      for (int c = 0; c < XSO_CHANNELS; ++c) {
        const float a = g32 * (float)lo[c];
        const float b = f32 * (float)hi[c];
        const float sigma = a + b;
        const float term = rho * sigma;
        const float y = term - comp[c];
        const float tt = sum[c] + y;
        comp[c] = (tt - sum[c]) - y;
        sum[c] = tt;
      }
    }
    for (int c = 0; c < XSO_CHANNELS; ++c) o[c] = sum[c];
  }
  return bad;
}
