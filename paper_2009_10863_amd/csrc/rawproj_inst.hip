// Raw-solution projection kernels for one storage format (LG_RAW_DT), so
// that the build compiles the formats in parallel.
#include "rawproj_impl.h"

#ifndef LG_RAW_DT
#error "LG_RAW_DT must be defined"
#endif

namespace lg {
template void raw_form_dt<LG_RAW_DT>(const RawBufs &, const double *, double *, hipStream_t, KEvents *);
template void raw_update_dt<LG_RAW_DT>(const RawBufs &, const Grid &, const double *, hipStream_t, KEvents *);
}  // namespace lg
