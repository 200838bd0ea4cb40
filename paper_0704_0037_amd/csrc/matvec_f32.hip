// Interaction-matrix product, single precision: kernel instantiations and launch.
#include "matvec_launch.hpp"

namespace dda {

template <>
dda_status matvec_device<float>(Ctx &c, const float2 *x, float2 *y, int nrhs, const float2 *scale, float2 *dots,
                              hipStream_t s, const int *done, hipEvent_t *ev) {
    return matvec_device_impl<float>(c, x, y, nrhs, scale, dots, s, done, ev);
}

}  // namespace dda
