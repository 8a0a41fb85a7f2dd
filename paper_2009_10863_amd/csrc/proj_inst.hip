// Projection kernels for one storage format and one variant, chosen at
// compile time (LG_PROJ_DT, LG_PROJ_VF): the build compiles this file once
// per combination, which keeps compile times parallel.
#include "proj_impl.h"

#if !defined(LG_PROJ_DT) || !defined(LG_PROJ_VF)
#error "LG_PROJ_DT and LG_PROJ_VF must be defined"
#endif

namespace lg {
template void proj_form_dt<LG_PROJ_DT, LG_PROJ_VF>(const ProjBufs &, const double *, double *, hipStream_t,
                                                  KEvents *);
template void proj_update_dt<LG_PROJ_DT, LG_PROJ_VF>(const ProjBufs &, const Grid *, const double *,
                                                    const double *, hipStream_t, KEvents *);
}  // namespace lg
