// Host-side driver of the C ABI's argument validation and size queries, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code of the
// library (tests/test_host_sanitizers.py).  Every call here is rejected, or
// answered, before any device work: no GPU is needed.  Prints one line per
// failed check and exits non-zero if any failed.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/tidas.h"

static int failures = 0;

static void expect(const char* what, long long got, long long want) {
    if (got != want) {
        std::printf("FAIL %s: got %lld, want %lld\n", what, got, want);
        ++failures;
    }
}

int main() {
    void* A = reinterpret_cast<void*>(0x1000);  // never dereferenced: validation fails first
    void* B = reinterpret_cast<void*>(0x2000);
    void* C = reinterpret_cast<void*>(0x3000);
    float* F = reinterpret_cast<float*>(0x4000);
    tidas_array arr{64, 0.3e-3, 1540.0};
    double ang0 = 0.0, ang_bad = 2.0;
    tidas_tx tx{1, &ang0, 40e6, 0.0, 5e6, 2.0};
    tidas_rx rx{1.5};
    tidas_grid grid{64, 32, 1e-3, 1e-4, -1e-3, 1e-4};
    const int E = TIDAS_EINVAL, U = TIDAS_EUNSUPPORTED;

    // das_beamform / tidas_beamform
    expect("das null rf", das_beamform(&arr, &tx, &rx, &grid, nullptr, 2048, 1, F, nullptr, 0, nullptr), E);
    tidas_array bad_arr{0, 0.3e-3, 1540.0};
    expect("das bad array", das_beamform(&bad_arr, &tx, &rx, &grid, F, 2048, 1, (float*)B, nullptr, 0, nullptr), E);
    tidas_tx bad_tx{1, &ang_bad, 40e6, 0.0, 5e6, 2.0};
    expect("das bad angle", das_beamform(&arr, &bad_tx, &rx, &grid, F, 2048, 1, (float*)B, nullptr, 0, nullptr), E);
    tidas_grid bad_grid{0, 32, 1e-3, 1e-4, -1e-3, 1e-4};
    expect("das bad grid", das_beamform(&arr, &tx, &rx, &bad_grid, F, 2048, 1, (float*)B, nullptr, 0, nullptr), E);
    expect("das aliasing", das_beamform(&arr, &tx, &rx, &grid, F, 2048, 1, F, nullptr, 0, nullptr), E);
    expect("beamform null", tidas_beamform(&arr, &tx, &rx, &grid, nullptr, 2048, 1, nullptr, nullptr, F, nullptr, 0, nullptr), E);

    // line model and its forms
    expect("apply even K", tidas_apply(F, 64, (float*)A, 1, 16, 16, (float*)B, nullptr), E);
    expect("apply null", tidas_apply(nullptr, 65, (float*)A, 1, 16, 16, (float*)B, nullptr), E);
    expect("apply alias", tidas_apply(F, 65, (float*)A, 1, 16, 16, (float*)A, nullptr), E);
    expect("adjoint B=0", tidas_adjoint(F, 65, (float*)A, 0, 16, 16, (float*)B, nullptr), E);
    expect("noalloc even K", tidas_apply_noalloc(F, 2, (float*)A, 1, 16, 16, (float*)B, nullptr), E);
    expect("apply_ex nan", tidas_apply_ex(F, 5, (float*)A, 1, 16, 16, __builtin_nanf(""), 0.0f, nullptr, (float*)B,
                                          nullptr), E);
    expect("line kernel even", tidas_line_kernel(64, 1, 64, 64), E);
    expect("prepared bytes 0", (long long)tidas_prepared_bytes(0, 64), 0);
    expect("prepare short", tidas_prepare(F, 65, 64, A, 16, nullptr), E);
    expect("lateral even", tidas_apply_lateral(F, 4, (float*)A, 1, 8, 8, (float*)B, nullptr), E);
    expect("kgrad even", tidas_kernel_grad(4, (float*)A, (float*)B, 1, 8, 8, F, nullptr, 0, nullptr), E);
    expect("kgrad path", tidas_kernel_grad_kernel(16, A, B), TIDAS_KGRAD_SPLIT_BF16);
    expect("kgrad path unaligned", tidas_kernel_grad_kernel(16, reinterpret_cast<void*>(0x1004), B), TIDAS_KGRAD_FP32);
    expect("deconv alias", tidas_deconvolve(F, 65, (float*)A, 1, 8, 8, 1e-3f, 1e-2f, 3, (float*)A, (float*)B,
                                            nullptr, 0, nullptr), E);
    expect("deconv eta", tidas_deconvolve(F, 65, (float*)A, 1, 8, 8, 1e-3f, 0.0f, 3, (float*)B, (float*)C, nullptr, 0,
                                          nullptr), E);
    double nrm = 0.0;
    expect("norm iters", tidas_operator_norm_sq(F, 65, 8, 0, (float*)A, &nrm, nullptr, 0, nullptr), E);
    expect("build null", tidas_build_kernels(&arr, &tx, &rx, &grid, 2048, 65, 0, nullptr, nullptr, nullptr,
                                             nullptr, 0, nullptr), E);
    expect("simulate negative", tidas_simulate_rf(&arr, &tx, (const double*)A, -1, 2048, F, nullptr, 0, nullptr), E);

    // the debug-flag query of a release build
    uint32_t dbg_flags = 7;
    expect("debug flags release", tidas_debug_flags(&dbg_flags, 1), U);
    expect("debug flags zeroed", (long long)dbg_flags, 0);
    expect("debug flags null", tidas_debug_flags(nullptr, 0), E);

    // caller workspaces: queries and checks
    expect("build ws exact", (long long)tidas_build_kernels_workspace_bytes(64, 65, 0), 0);
    const size_t bws = tidas_build_kernels_workspace_bytes(64, 65, 1);
    expect("build ws short", tidas_build_kernels(&arr, &tx, &rx, &grid, 2048, 65, 1, nullptr, F, nullptr, A, bws - 1,
                                                 nullptr), E);
    expect("simulate ws", (long long)tidas_simulate_rf_workspace_bytes(1, 64, 100), 8 * (64 * 100 + 1));
    expect("simulate ws misaligned", tidas_simulate_rf(&arr, &tx, (const double*)A, 3, 100, F,
                                                       reinterpret_cast<void*>(0x100010), 8 * 6401, nullptr), E);
    expect("kgrad ws no pointer", tidas_kernel_grad(5, (float*)A, (float*)B, 1, 8, 8, F, nullptr, 64, nullptr), E);
    expect("deconv ws even K", (long long)tidas_deconvolve_workspace_bytes(64, 1, 8, 8), 0);
    expect("norm ws Z=0", (long long)tidas_operator_norm_sq_workspace_bytes(65, 0), 0);

    // ragged batches: host tables
    expect("batch bytes", (long long)tidas_batch_workspace_bytes(3), 512);
    std::vector<tidas_frame> frames(3);
    for (int f = 0; f < 3; ++f)
        frames[f] = tidas_frame{tidas_grid{100 + 50 * f, 40 + 7 * f, 0.0, 1.0, 0.0, 1.0}, nullptr, F,
                                (const float*)A, (float*)B + f};
    const size_t need = tidas_apply_batch_workspace_bytes(frames.data(), 3, 65);
    if (need <= tidas_batch_workspace_bytes(3)) {
        std::printf("FAIL batch workspace %zu\n", need);
        ++failures;
    }
    expect("batch bytes even K", (long long)tidas_apply_batch_workspace_bytes(frames.data(), 3, 64), 0);
    expect("batch variant", tidas_apply_batch(frames.data(), 3, 65, A, need, 99, nullptr), E);
    expect("batch short", tidas_apply_batch(frames.data(), 3, 65, A, 16, 0, nullptr), E);
    expect("batch prepare short", tidas_apply_batch_prepare(frames.data(), 3, 65, A, 16, nullptr), E);
    frames[1].out = (float*)A;  // aliases its input
    expect("batch prepare alias", tidas_apply_batch_prepare(frames.data(), 3, 65, reinterpret_cast<void*>(0x10000),
                                                            need, nullptr), E);
    expect("das batch short", das_beamform_batch(&arr, &tx, &rx, 2048, frames.data(), 3, A, 8, 0, nullptr), E);

    // single-point study and its helpers
    tidas_array big{192, 0.3e-3, 1540.0};
    expect("kossoff", tidas_kossoff_tx_count(&big, 5e6, 25e-3, 0.6), 24);
    expect("kossoff bad", tidas_kossoff_tx_count(&big, 5e6, -1.0, 0.6), E);
    const size_t sw = tidas_point_study_workspace_bytes(33, 10, 1400, 1000);
    expect("study bytes 0", (long long)tidas_point_study_workspace_bytes(33, 0, 1400, 1000), 0);
    tidas_array a33{33, 0.3e-3, 1540.0};
    expect("study n_tx parity", tidas_point_study(&a33, &tx, &rx, 8, 1400, 10, 6e-3, 2e-3, 4, 1000, 100, (double*)A,
                                                  (double*)B, (double*)C, nullptr, nullptr, F, sw, nullptr), E);
    expect("study short ws", tidas_point_study(&a33, &tx, &rx, 9, 1400, 10, 6e-3, 2e-3, 4, 1000, 100, (double*)A,
                                               (double*)B, (double*)C, nullptr, nullptr, F, sw - 1, nullptr), E);
    tidas_array a600{600, 0.3e-3, 1540.0};
    expect("study too many elements", tidas_point_study(&a600, &tx, &rx, 10, 1400, 10, 6e-3, 2e-3, 4, 1000, 100,
                                                        (double*)A, (double*)B, (double*)C, nullptr, nullptr, F, sw,
                                                        nullptr), U);

    // surrogate network
    int32_t widths[5] = {4, 256, 256, 256, 129};
    expect("mlp params", tidas_mlp_param_count(widths), 4 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 129 + 129);
    int32_t bad_w[5] = {4, 0, 256, 256, 129};
    expect("mlp bad widths", tidas_mlp_param_count(bad_w), -1);
    expect("mlp forward null", tidas_mlp_forward(widths, nullptr, F, F, 8, nullptr, F, A, 1 << 20, nullptr), E);
    expect("adam step 0", tidas_mlp_adam(widths, F, F, F, F, (uint16_t*)A, 1e-3f, 0.9f, 0.999f, 1e-8f, 0, nullptr), E);

    if (std::strlen(tidas_last_error()) == 0) {
        std::printf("FAIL last error empty\n");
        ++failures;
    }
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
