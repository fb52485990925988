// Host-side part of the C ABI: error reporting, version and the argument
// validation shared by the entry points.
#include <cmath>
#include <string>

#include "common.hpp"

namespace tidas {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int32_t validate_array(const tidas_array* a) {
    if (!a) return fail(TIDAS_EINVAL, "null array descriptor");
    if (a->n_elem < 1) return fail(TIDAS_EINVAL, "array: n_elem must be >= 1");
    if (!finite_pos(a->pitch)) return fail(TIDAS_EINVAL, "array: pitch must be finite and > 0");
    if (!finite_pos(a->c)) return fail(TIDAS_EINVAL, "array: c must be finite and > 0");
    return TIDAS_OK;
}

int32_t validate_tx(const tidas_tx* t, bool need_pulse) {
    if (!t) return fail(TIDAS_EINVAL, "null transmit descriptor");
    if (t->n_angles < 1) return fail(TIDAS_EINVAL, "tx: n_angles must be >= 1");
    if (!t->angles) return fail(TIDAS_EINVAL, "tx: null angles");
    for (int a = 0; a < t->n_angles; ++a)
        if (!std::isfinite(t->angles[a]) || std::fabs(t->angles[a]) >= 1.5707963267948966)
            return fail(TIDAS_EINVAL, "tx: angles must be finite and inside (-pi/2, pi/2)");
    if (!finite_pos(t->fs)) return fail(TIDAS_EINVAL, "tx: fs must be finite and > 0");
    if (!std::isfinite(t->t0)) return fail(TIDAS_EINVAL, "tx: t0 must be finite");
    if (need_pulse) {
        if (!finite_pos(t->fc)) return fail(TIDAS_EINVAL, "tx: fc must be finite and > 0");
        if (!finite_pos(t->cycles)) return fail(TIDAS_EINVAL, "tx: cycles must be finite and > 0");
    }
    return TIDAS_OK;
}

int32_t validate_rx(const tidas_rx* r) {
    if (!r) return fail(TIDAS_EINVAL, "null receive descriptor");
    if (!finite_pos(r->fnumber)) return fail(TIDAS_EINVAL, "rx: fnumber must be finite and > 0");
    return TIDAS_OK;
}

int32_t validate_grid(const tidas_grid* g) {
    if (!g) return fail(TIDAS_EINVAL, "null grid descriptor");
    if (g->nz < 1 || g->nx < 1) return fail(TIDAS_EINVAL, "grid: nz and nx must be >= 1");
    if (!finite_pos(g->dz) || !finite_pos(g->dx)) return fail(TIDAS_EINVAL, "grid: dz and dx must be finite and > 0");
    if (!std::isfinite(g->z0) || !std::isfinite(g->x0)) return fail(TIDAS_EINVAL, "grid: z0 and x0 must be finite");
    return TIDAS_OK;
}

// flag words of the source files with debug checks
uint32_t tidas_debug_read_das(bool reset);
uint32_t tidas_debug_read_conv(bool reset);
uint32_t tidas_debug_read_study(bool reset);

}  // namespace tidas

extern "C" const char* tidas_version(void) { return "tidas-mi355x 0.1 (gfx950)"; }

extern "C" int32_t tidas_debug_flags(uint32_t* flags, int32_t reset) {
    if (!flags) return tidas::fail(TIDAS_EINVAL, "tidas_debug_flags: null flags pointer");
#ifdef TIDAS_DEBUG
    if (hipDeviceSynchronize() != hipSuccess) return tidas::fail(TIDAS_EHIP, "tidas_debug_flags: synchronize");
    const bool r = reset != 0;
    const uint32_t v = tidas::tidas_debug_read_das(r) | tidas::tidas_debug_read_conv(r) |
                       tidas::tidas_debug_read_study(r);
    if (v == ~0u) return tidas::fail(TIDAS_EHIP, "tidas_debug_flags: flag word copy failed");
    *flags = v;
    return TIDAS_OK;
#else
    (void)reset;
    *flags = 0;
    return tidas::fail(TIDAS_EUNSUPPORTED, "tidas_debug_flags: not a debug build (TIDAS_DEBUG)");
#endif
}

extern "C" const char* tidas_last_error(void) { return tidas::g_last_error.c_str(); }
