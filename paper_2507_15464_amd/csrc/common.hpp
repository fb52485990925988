// Shared host/device helpers of the tiDAS library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/tidas.h"

namespace tidas {

// ---------------------------------------------------------------- status ----
void set_error(const std::string& msg);

inline int32_t fail(int32_t code, const std::string& msg) {
    set_error(msg);
    return code;
}

inline int32_t check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TIDAS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return TIDAS_OK;
}

inline int32_t check_hip(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(TIDAS_ENOMEM, std::string(what) + ": out of device memory");
    if (e != hipSuccess) return fail(TIDAS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return TIDAS_OK;
}

// ---------------------------------------------------------- debug checks ----
// Built with -DTIDAS_DEBUG (libtidas_debug.so), kernels check values and
// indices against what their derivation promises; a failed check sets its
// bit in its source file's flag word (nothing traps, and every access stays
// as in the release build).  tidas_debug_flags returns the OR of the words.
// (the bits, TIDAS_DBG_*, are declared in tidas.h)
#ifdef TIDAS_DEBUG
#define TIDAS_DEBUG_FLAGS_DEFINE(name)                                                               \
    static __device__ unsigned int tidas_dbg_word;                                                   \
    uint32_t tidas_debug_read_##name(bool reset) {                                                   \
        unsigned int v = 0;                                                                          \
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(tidas_dbg_word), sizeof(v)) != hipSuccess) v = ~0u;   \
        if (reset) {                                                                                 \
            const unsigned int z = 0;                                                                \
            if (hipMemcpyToSymbol(HIP_SYMBOL(tidas_dbg_word), &z, sizeof(z)) != hipSuccess) v = ~0u; \
        }                                                                                            \
        return v;                                                                                    \
    }
#define TIDAS_DCHECK(cond, bit)                                    \
    do {                                                           \
        if (!(cond)) atomicOr(&tidas_dbg_word, (unsigned)(bit)); \
    } while (0)
#else
#define TIDAS_DEBUG_FLAGS_DEFINE(name) \
    uint32_t tidas_debug_read_##name(bool) { return 0; }
#define TIDAS_DCHECK(cond, bit) \
    do {                        \
    } while (0)
#endif

// ------------------------------------------------------------ workspace ----
// Entry points that need device scratch take (workspace, workspace_bytes): a
// caller buffer of at least the size their query returns, 256-byte aligned,
// or NULL with 0 bytes, in which case the call allocates the scratch
// stream-ordered on its own stream and frees it the same way.
struct Workspace {
    char* ptr = nullptr;
    bool owned = false;
};

// Argument check (before anything is enqueued).
inline int32_t workspace_check(const char* who, const void* ws, size_t bytes, size_t need) {
    if (!ws) {
        if (bytes != 0) return fail(TIDAS_EINVAL, std::string(who) + ": workspace_bytes must be 0 with a null workspace");
        return TIDAS_OK;
    }
    if (bytes < need) return fail(TIDAS_EINVAL, std::string(who) + ": workspace smaller than its size query");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
        return fail(TIDAS_EINVAL, std::string(who) + ": workspace not 256-byte aligned");
    return TIDAS_OK;
}

// The caller's buffer, or `need` bytes allocated stream-ordered.
inline int32_t workspace_acquire(const char* who, void* ws, size_t need, hipStream_t s, Workspace& w) {
    if (ws) {
        w.ptr = (char*)ws;
        w.owned = false;
        return TIDAS_OK;
    }
    w.owned = true;
    if (need == 0) return TIDAS_OK;
    return check_hip(hipMallocAsync((void**)&w.ptr, need, s), who);
}

inline int32_t workspace_release(const char* who, Workspace& w, hipStream_t s) {
    if (!w.owned || !w.ptr) return TIDAS_OK;
    const int32_t st = check_hip(hipFreeAsync(w.ptr, s), who);
    w.ptr = nullptr;
    return st;
}

// Validation of the descriptors shared by several entry points.  Returns
// TIDAS_OK or TIDAS_EINVAL with a message.
int32_t validate_array(const tidas_array* a);
int32_t validate_tx(const tidas_tx* t, bool need_pulse);
int32_t validate_rx(const tidas_rx* r);
int32_t validate_grid(const tidas_grid* g);

inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Ragged-batch arguments shared by the DAS and line-model batch entry points.
int32_t validate_batch(const char* name, const tidas_frame* frames, int32_t n_frames, void* workspace,
                       size_t workspace_bytes, bool need_rf, bool need_conv);

// -------------------------------------------------------------- device ----
// Hann apodization 0.5 (1 + cos(pi t)) = cos^2(pi t / 2) for |t| <= 1, from
// the Taylor series of cos(pi t / 2) in u = t^2 through u^6 (truncation
// error below 7e-9 on [0, 1]), evaluated by Horner's rule.
__device__ __forceinline__ float hann_weight(float t) {
    const float u = t * t;
    constexpr double h = 1.5707963267948966;  // pi / 2
    constexpr double h2 = h * h;
    constexpr double c1 = -h2 / 2.0;
    constexpr double c2 = h2 * h2 / 24.0;
    constexpr double c3 = -h2 * h2 * h2 / 720.0;
    constexpr double c4 = h2 * h2 * h2 * h2 / 40320.0;
    constexpr double c5 = -h2 * h2 * h2 * h2 * h2 / 3628800.0;
    constexpr double c6 = h2 * h2 * h2 * h2 * h2 * h2 / 479001600.0;
    float q = (float)c6;
    q = fmaf(q, u, (float)c5);
    q = fmaf(q, u, (float)c4);
    q = fmaf(q, u, (float)c3);
    q = fmaf(q, u, (float)c2);
    q = fmaf(q, u, (float)c1);
    q = fmaf(q, u, 1.0f);
    return q * q;
}

// Raw buffer resource over `bytes` bytes starting at `base`: loads outside
// [0, bytes) return 0, which is exactly the zero-outside-the-record rule of
// the channel read (negative offsets wrap to huge unsigned values and miss).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float buffer_load_f32(__amdgpu_buffer_rsrc_t r, int32_t byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

}  // namespace tidas
