// Projection kernels instantiated for bf16 history storage (one
// translation unit per storage format keeps compile times parallel).
#include "proj_impl.h"

namespace lg {
template void proj_form_dt<GUESS_BF16>(const ProjBufs &, const double *, double *, hipStream_t,
                                 KEvents *);
template void proj_update_dt<GUESS_BF16>(const ProjBufs &, const Grid *, const double *, const double *,
                                   hipStream_t, KEvents *);
}  // namespace lg
