// Launch entry points of the projection guess: dispatch on the storage
// format to the instantiations in proj_f64/f32/f16/bf16.hip (kernels in
// proj_impl.h).
#include "launch.h"

namespace lg {

template <int DT>
void proj_form_dt(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev);
template <int DT>
void proj_update_dt(const ProjBufs &p, const Grid *g, const double *x, const double *Ax, hipStream_t s,
                    KEvents *ev);

int launch_proj_form(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    switch (p.dtype) {
        case GUESS_F64: proj_form_dt<GUESS_F64>(p, b, x0, s, ev); break;
        case GUESS_F32: proj_form_dt<GUESS_F32>(p, b, x0, s, ev); break;
        case GUESS_F16: proj_form_dt<GUESS_F16>(p, b, x0, s, ev); break;
        case GUESS_BF16: proj_form_dt<GUESS_BF16>(p, b, x0, s, ev); break;
        default: return GUESS_EINVAL;
    }
    return GUESS_OK;
}

int launch_proj_update(const ProjBufs &p, const Grid *g, const double *x, const double *Ax,
                       hipStream_t s, KEvents *ev) {
    if (!Ax && !g) return GUESS_EINVAL;
    switch (p.dtype) {
        case GUESS_F64: proj_update_dt<GUESS_F64>(p, g, x, Ax, s, ev); break;
        case GUESS_F32: proj_update_dt<GUESS_F32>(p, g, x, Ax, s, ev); break;
        case GUESS_F16: proj_update_dt<GUESS_F16>(p, g, x, Ax, s, ev); break;
        case GUESS_BF16: proj_update_dt<GUESS_BF16>(p, g, x, Ax, s, ev); break;
        default: return GUESS_EINVAL;
    }
    return GUESS_OK;
}

}  // namespace lg
