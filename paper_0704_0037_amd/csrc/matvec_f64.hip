// Interaction-matrix product, double precision: kernel instantiations and launch.
#include "matvec_launch.hpp"

namespace dda {

template <>
dda_status matvec_device<double>(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                              hipStream_t s, const int *done, hipEvent_t *ev) {
    return matvec_device_impl<double>(c, x, y, nrhs, scale, dots, s, done, ev);
}

}  // namespace dda
