// Lookup and index kernels for the XS_GRID_UNIONIZED search method.
#include "xs_lookup_impl.h"

namespace xs {

hipError_t launch_lookup_union(const DevTables& t, const xs_params& p,
                              const LookupArgs& a, hipStream_t s) {
  return launch_grid_method<XS_GRID_UNIONIZED>(t, p, a, s);
}

hipError_t launch_indices_union(const DevTables& t, int64_t n, const double* E,
                               const int32_t* mat, const int64_t* off,
                               int32_t* idx, hipStream_t s) {
  return launch_indices_grid<XS_GRID_UNIONIZED>(t, n, E, mat, off, idx, s);
}

}  // namespace xs
