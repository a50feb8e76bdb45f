// Vector-Jacobian product of the right-hand side (placeholder until the
// gather-form kernels land).
#include "common.hpp"

namespace sph {
size_t adjoint_ws_bytes(int64_t n) { Carve c(nullptr); c.take<double>(n); return c.used; }
size_t leapfrog_ws_bytes(int64_t n) { Carve c(nullptr); c.take<double>(n); return c.used; }
size_t leapfrog_adjoint_ws_bytes(int64_t n) { Carve c(nullptr); c.take<double>(n); return c.used; }
}  // namespace sph

using namespace sph;

extern "C" int sph_rhs_adjoint(const sph_grid *, const sph_state *, const sph_params *,
                               const sph_deriv_cot *, const sph_state_grad *, double *, void *,
                               size_t, void *) {
    return fail(SPH_ERR_NOT_IMPLEMENTED, "sph_rhs_adjoint is not implemented yet");
}

extern "C" int sph_leapfrog(const sph_grid *, const sph_state *, const sph_params *, double, int,
                            const sph_fields *, double *, void *, size_t, void *) {
    return fail(SPH_ERR_NOT_IMPLEMENTED, "sph_leapfrog is not implemented yet");
}

extern "C" int sph_leapfrog_adjoint(const sph_grid *, const sph_state *, const sph_params *, double,
                                    int, const double *, const sph_cfields *, const sph_fields *,
                                    double *, void *, size_t, void *) {
    return fail(SPH_ERR_NOT_IMPLEMENTED, "sph_leapfrog_adjoint is not implemented yet");
}

extern "C" size_t sph_checkpoint_bytes(int64_t n, int steps) {
    return (size_t)(steps + 1) * 23u * (size_t)(n > 0 ? n : 0) * sizeof(double);
}
