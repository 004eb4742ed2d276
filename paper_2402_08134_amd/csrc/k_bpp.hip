// Exact per-row NLS by block principal pivoting: implemented in a later step;
// until then the rule is rejected at context creation.
#include "kernels.hpp"

int bpp_update(int, int, int, const void*, const int*, const int*, const double*, const void*, void*, int,
               const double*, double, Workspace&, const DevState*, hipStream_t) {
  return -1;
}
