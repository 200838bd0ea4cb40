// Interaction-matrix product, double precision: kernel instantiations and launch.
#include "matvec_launch.hpp"

namespace dda {

dda_status matvec_materials(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                            hipStream_t s, const int *done, hipEvent_t *ev);

template <>
dda_status matvec_device<double>(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, double2 *dots,
                              hipStream_t s, const int *done, hipEvent_t *ev) {
    if (wrapped(c)) return matvec_materials(c, x, y, nrhs, scale, dots, s, done, ev);
    return matvec_device_impl<double>(c, x, y, nrhs, scale, dots, s, done, ev);
}

// the unit-polarizability product of an inhomogeneous particle (the materials enter around it)
dda_status matvec_device_unit(Ctx &c, const double2 *x, double2 *y, int nrhs, const double2 *scale, hipStream_t s,
                              const int *done, hipEvent_t *ev) {
    return matvec_device_impl<double>(c, x, y, nrhs, scale, nullptr, s, done, ev);
}

}  // namespace dda
