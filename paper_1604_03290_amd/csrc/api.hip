// Library-wide entry points: version, error strings, workspace sizes, device
// status readback.
#include <cstdarg>
#include <cstdio>

#include "common.hpp"

namespace sph {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

size_t build_ws_bytes(int64_t n, int64_t ncells);
size_t neighbours_ws_bytes(int64_t n);
size_t rhs_ws_bytes(int64_t n);
size_t adjoint_ws_bytes(int64_t n);
size_t leapfrog_ws_bytes(int64_t n);
size_t leapfrog_adjoint_ws_bytes(int64_t n);
size_t pairs_ws_bytes(int64_t n);
size_t gravity_ws_bytes(int64_t n, int64_t node_cap);

}  // namespace sph

using namespace sph;

extern "C" const char *sph_version(void) { return "libsph 0.1 gfx950"; }

extern "C" const char *sph_last_error(void) { return g_err; }

extern "C" size_t sph_workspace_bytes(int op, int64_t n, int64_t ncells) {
    if (n <= 0) n = 1;
    if (op == SPH_OP_GRAVITY) return gravity_ws_bytes(n, ncells);
    if (ncells <= 0) ncells = 1;
    switch (op) {
        case SPH_OP_BUILD: return build_ws_bytes(n, ncells);
        case SPH_OP_NEIGHBOURS: return neighbours_ws_bytes(n);
        case SPH_OP_RHS: return rhs_ws_bytes(n);
        case SPH_OP_ADJOINT: return adjoint_ws_bytes(n);
        case SPH_OP_LEAPFROG: return leapfrog_ws_bytes(n);
        case SPH_OP_LEAPFROG_ADJOINT: return leapfrog_adjoint_ws_bytes(n);
        case SPH_OP_PAIRS: return pairs_ws_bytes(n);
        default: return 0;
    }
}

extern "C" int sph_workspace_status(const void *ws, void *stream) {
    clear_error();
    if (!ws) return fail(SPH_ERR_INVALID_ARG, "workspace is NULL");
    int32_t flag = 0;
    hipStream_t s = (hipStream_t)stream;
    SPH_HIP_TRY(hipMemcpyAsync(&flag, ws, sizeof flag, hipMemcpyDeviceToHost, s));
    SPH_HIP_TRY(hipStreamSynchronize(s));
    if (flag) return fail(flag, "device flag %d", flag);
    return SPH_OK;
}
