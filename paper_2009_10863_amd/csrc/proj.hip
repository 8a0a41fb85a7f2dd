// Launch entry points of the projection guess: dispatch on the storage
// format and the variant to the instantiations of proj_inst.hip (kernels in
// proj_impl.h).
#include "launch.h"

namespace lg {

template <int DT, int VF>
void proj_form_dt(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev);
template <int DT, int VF>
void proj_update_dt(const ProjBufs &p, const Grid *g, const double *x, const double *Ax, hipStream_t s,
                    KEvents *ev);

namespace {
template <int DT>
int form_vf(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    switch (p.vf) {
        case 0: proj_form_dt<DT, 0>(p, b, x0, s, ev); return GUESS_OK;
        case 1: proj_form_dt<DT, 1>(p, b, x0, s, ev); return GUESS_OK;
        case 2: proj_form_dt<DT, 2>(p, b, x0, s, ev); return GUESS_OK;
        case 3: proj_form_dt<DT, 3>(p, b, x0, s, ev); return GUESS_OK;
    }
    return GUESS_EINVAL;
}
template <int DT>
int update_vf(const ProjBufs &p, const Grid *g, const double *x, const double *Ax, hipStream_t s,
              KEvents *ev) {
    switch (p.vf) {
        case 0: proj_update_dt<DT, 0>(p, g, x, Ax, s, ev); return GUESS_OK;
        case 1: proj_update_dt<DT, 1>(p, g, x, Ax, s, ev); return GUESS_OK;
        case 2: proj_update_dt<DT, 2>(p, g, x, Ax, s, ev); return GUESS_OK;
        case 3: proj_update_dt<DT, 3>(p, g, x, Ax, s, ev); return GUESS_OK;
    }
    return GUESS_EINVAL;
}
}  // namespace

int launch_proj_form(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    switch (p.dtype) {
        case GUESS_F64: return form_vf<GUESS_F64>(p, b, x0, s, ev);
        case GUESS_F32: return form_vf<GUESS_F32>(p, b, x0, s, ev);
        case GUESS_F16: return form_vf<GUESS_F16>(p, b, x0, s, ev);
        case GUESS_BF16: return form_vf<GUESS_BF16>(p, b, x0, s, ev);
    }
    return GUESS_EINVAL;
}

int launch_proj_update(const ProjBufs &p, const Grid *g, const double *x, const double *Ax,
                       hipStream_t s, KEvents *ev) {
    if (!Ax && !g) return GUESS_EINVAL;
    switch (p.dtype) {
        case GUESS_F64: return update_vf<GUESS_F64>(p, g, x, Ax, s, ev);
        case GUESS_F32: return update_vf<GUESS_F32>(p, g, x, Ax, s, ev);
        case GUESS_F16: return update_vf<GUESS_F16>(p, g, x, Ax, s, ev);
        case GUESS_BF16: return update_vf<GUESS_BF16>(p, g, x, Ax, s, ev);
    }
    return GUESS_EINVAL;
}

}  // namespace lg
