// Launch entry points of the raw-solution projection: dispatch on the
// storage format to the instantiations of rawproj_inst.hip (kernels in
// rawproj_impl.h).
#include "launch.h"

namespace lg {

template <int DT>
void raw_form_dt(const RawBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev);
template <int DT>
void raw_update_dt(const RawBufs &p, const Grid &g, const double *x, hipStream_t s, KEvents *ev);

int launch_raw_form(const RawBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    switch (p.dtype) {
        case GUESS_F64: raw_form_dt<GUESS_F64>(p, b, x0, s, ev); return GUESS_OK;
        case GUESS_F32: raw_form_dt<GUESS_F32>(p, b, x0, s, ev); return GUESS_OK;
        case GUESS_F16: raw_form_dt<GUESS_F16>(p, b, x0, s, ev); return GUESS_OK;
        case GUESS_BF16: raw_form_dt<GUESS_BF16>(p, b, x0, s, ev); return GUESS_OK;
    }
    return GUESS_EINVAL;
}

int launch_raw_update(const RawBufs &p, const Grid &g, const double *x, hipStream_t s, KEvents *ev) {
    switch (p.dtype) {
        case GUESS_F64: raw_update_dt<GUESS_F64>(p, g, x, s, ev); return GUESS_OK;
        case GUESS_F32: raw_update_dt<GUESS_F32>(p, g, x, s, ev); return GUESS_OK;
        case GUESS_F16: raw_update_dt<GUESS_F16>(p, g, x, s, ev); return GUESS_OK;
        case GUESS_BF16: raw_update_dt<GUESS_BF16>(p, g, x, s, ev); return GUESS_OK;
    }
    return GUESS_EINVAL;
}

}  // namespace lg
