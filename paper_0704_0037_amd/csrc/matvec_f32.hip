// Interaction-matrix product, single precision: kernel instantiations and launch.
#include "matvec_launch.hpp"

namespace dda {

template <>
dda_status matvec_device<float>(Ctx &c, const float2 *x, float2 *y, int nrhs, const float2 *scale, float2 *dots,
                              hipStream_t s, const int *done, hipEvent_t *ev) {
    return matvec_device_impl<float>(c, x, y, nrhs, scale, dots, s, done, ev);
}

// double-precision vectors through single-precision transforms and tensor
dda_status matvec_device_mixed(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                               hipStream_t s, const int *done, hipEvent_t *ev) {
    if (!c.ghat32) {
        set_error("single-precision products need a context set up with opts.fp32");
        return DDA_ENOTSUP;
    }
    dda_status st = ensure_work<float>(c, nrhs);
    if (st != DDA_OK) return st;
    return matvec_device_impl<float, double>(c, x, y, nrhs, scale, dots, s, done, ev);
}

}  // namespace dda
