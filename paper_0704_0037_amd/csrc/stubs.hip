// Entry points not yet implemented in this build: they report DDA_ENOTSUP.
#include "ctx.hpp"

extern "C" {
dda_status dda_solve(dda_ctx *, const dda_beam *, int32_t, double, const dda_solve_opts *, void *, dda_solve_info *) {
    dda::set_error("dda_solve: not built");
    return DDA_ENOTSUP;
}
dda_status dda_cross_sections(dda_ctx *, const dda_beam *, const void *, double *) {
    dda::set_error("dda_cross_sections: not built");
    return DDA_ENOTSUP;
}
dda_status dda_farfield(dda_ctx *, const dda_beam *, const void *, int32_t, const double *, double *) {
    dda::set_error("dda_farfield: not built");
    return DDA_ENOTSUP;
}
dda_status dda_mueller(dda_ctx *, const dda_beam *, const void *, const void *, double, const double *, int32_t,
                       double *) {
    dda::set_error("dda_mueller: not built");
    return DDA_ENOTSUP;
}
}
