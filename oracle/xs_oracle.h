/*
 * Serial CPU oracle for the batched macroscopic cross-section lookup.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library under paper_2402_09222_amd/) shares no code with it.
 *
 * What it computes (section 5.1, the hash-bin paragraph of the list that
 * follows Table 1): for a particle at energy E in material m, every nuclide
 * of m is searched for the grid interval that holds E, its tabulated
 * channels are interpolated linearly in E, and the results are summed
 * weighted by the nuclide densities of m.  The paper names the operation
 * but prints no formula; the readings taken where it is silent are:
 *
 *   bracket   i = clamp(#{p : E_k[p] <= E} - 1, 0, n_k - 2)
 *   clamp     Eh = min(max(E, E_k[0]), E_k[n_k - 1])
 *   fraction  f = (Eh - E_k[i]) / (E_k[i+1] - E_k[i]),  g = 1 - f   (FP64)
 *   channel   s_c = g * X_k[i][c] + f * X_k[i+1][c]   (two products, one add)
 *   sum       S_c = sum over the material list, in list order, from +0.0,
 *             of rho_j * s_c (product, then add)
 *
 * Built with -ffp-contract=off so that no multiply-add is fused.
 *
 * Parity pins (checked by the CPU tests): the count and bisection brackets
 * agree on every probe of tiny grids and with numpy.searchsorted; grid-point
 * queries return the tabulated values exactly; affine tables are
 * reproduced to a few ulp; scaling the densities by 2^s scales the result
 * exactly; exact rational evaluation bounds the rounding error; numpy.interp
 * gives the same sums within the same bound.
 */
#ifndef XS_ORACLE_H
#define XS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XSO_CHANNELS 5

typedef struct {
  int32_t n_nuclides;            /* K */
  const int64_t* grid_offsets;   /* [K+1] */
  const double* energy;          /* [P], strictly increasing per nuclide */
  const double* xs;              /* [P][5], point-major */
  int32_t n_materials;           /* M */
  const int32_t* mat_offsets;    /* [M+1] */
  const int32_t* mat_nuclides;   /* nuclide ids, list order */
  const double* mat_density;     /* densities, list order */
} xso_tables;

/* Bracket by its definition: count the grid points <= e, subtract one,
 * clamp into [0, n-2].  O(n).  n >= 2. */
int64_t xso_bracket_count(const double* grid, int64_t n, double e);

/* The same index by bisection for the first point > e.  O(log n). */
int64_t xso_bracket_bisect(const double* grid, int64_t n, double e);

/* One lookup.  search = 0 uses bisection, 1 the counting definition.
 * out[5] receives the five sums; idx (may be NULL) receives the bracket of
 * each nuclide of the material in list order.  Returns 0, or -1 when e is
 * not finite and > 0 or m is out of range: then out holds NaN and idx, if the
 * material is valid, holds -1 per nuclide. */
int xso_lookup(const xso_tables* t, double e, int32_t m, int search,
               double out[XSO_CHANNELS], int32_t* idx);

/* n lookups in input order.  out is [n][5].  idx (may be NULL) is written at
 * idx[idx_offsets[q] ...] for lookup q; idx_offsets is [n+1] (may be NULL
 * when idx is NULL). Returns the number of invalid lookups. */
int64_t xso_lookup_batch(const xso_tables* t, int64_t n, const double* e,
                         const int32_t* m, int search, double* out,
                         const int64_t* idx_offsets, int32_t* idx);

/* The FP32 form of the same lookup: the bracket and f are FP64 as above;
 * channels and densities are rounded to FP32 (nearest even), f32 = fl32(f)
 * and g32 = fl32(1 - f) are formed from the FP64 f, s_c = g32*lo + f32*hi in
 * FP32, and the sum over the material list is compensated (Kahan 1965):
 * y = rho*s - c; t = S + y; c = (t - S) - y; S = t.  out is [n][5] float.
 * Returns the number of invalid lookups (their outputs are NaN). */
int64_t xso_lookup_batch_f32(const xso_tables* t, int64_t n, const double* e,
                             const int32_t* m, float* out);

#ifdef __cplusplus
}
#endif

#endif
