// Lateral pass of the separable 2-D extension of the line model (gfx950).
//
// After the depth pass (the line model, Sec. 2.4 eqn:line_conv), each depth
// row is convolved along the lateral axis with that row's kernel (the
// lateral profile of the row's PSF, tidas_build_kernels lateral mode):
//
//   out[b][i][j] = sum_{m=-h..h} Kx[i][m+h] * in[b][i][j-m],   in = 0 outside [0, X).
//
// One wave per 256-column segment of one row of one frame (4 independent
// waves per workgroup, each with its own LDS region): the segment with
// its halo (zero outside the row) is staged in LDS and each lane produces 4
// consecutive outputs.  For the usual tap counts (17, 33, 65) the tap loop is
// unrolled at compile time, the row's taps are scalar loads and every window
// sample is read from LDS once; other counts stage the taps in LDS too and
// take them in groups of 4 over a sliding register window.  The pass is
// bound by HBM (8 bytes per pixel).

#include "common.hpp"

namespace tidas {
namespace {

constexpr int LAT_SEG = 256;  // columns per wave
constexpr int LAT_PER_LANE = 4;
constexpr int LAT_STAGE = 8;  // staging loads per lane issued together (segments of up to 512 samples)
constexpr int LAT_WAVES = 1;  // waves per workgroup (4 independent waves per group measured 1.2-1.4x slower)

// LDS floats of one wave's segment (and taps), a multiple of 4
__host__ __device__ constexpr int lat_wave_floats(int K, bool taps_in_lds) {
    return (LAT_SEG + K - 1 + (taps_in_lds ? K : 0) + 3) / 4 * 4;
}

// KT > 0: a compile-time tap count (taps in scalar registers, the tap loop
// unrolled, every window sample read from LDS once); KT = 0: any K (taps
// staged in LDS, groups of 4 taps over a sliding register window).
template <int KT>
__global__ __launch_bounds__(64 * LAT_WAVES) void lateral_pass_kernel(const float* __restrict__ kx, int32_t K_rt,
                                                                      const float* __restrict__ in, int32_t Z,
                                                                      int32_t X, int32_t n_seg, int32_t n_waves,
                                                                      float* __restrict__ out) {
    // (every byte offset below stays in int32: X + 2 K < 2^29 is checked on the host)
    const int K = KT > 0 ? KT : K_rt;
    // per wave: LAT_SEG + K - 1 samples, then (KT = 0) K taps, padded to 16 bytes
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int w_raw = blockIdx.x * LAT_WAVES + wv;  // wave-uniform: scalar tap loads, one descriptor per wave
    const bool live = w_raw < n_waves;  // a spare wave of the last workgroup repeats the last segment, unstored
    const int w = live ? w_raw : n_waves - 1;
    float* seg = lds + wv * lat_wave_floats(K, KT == 0);  // columns j0 - h .. j0 + LAT_SEG - 1 + h
    const int sg = w % n_seg;
    const int row = w / n_seg;  // b * Z + i
    const int i = row % Z;
    const int h = (K - 1) / 2;
    const int j0 = sg * LAT_SEG;
    const int lane = threadIdx.x & 63;
    const int L = LAT_SEG + K - 1;
    float* taps = seg + L;
    // the segment: unconditional loads, all in flight before the first LDS
    // write; a column outside [0, X) gets the offset 2^31, past the row's
    // record, and reads 0.  Each offset is its own opaque register value: the
    // compiler would otherwise fold the 64-column steps into immediate offsets
    // on one shared register, and a negative register offset (the halo left of
    // the row) plus an immediate gave wrong values.
    const auto rs = make_rsrc(in + (size_t)row * X, (uint32_t)X * 4u);
    auto col_off = [&](int j) {
        uint32_t off = (j >= 0 && j < X) ? (uint32_t)j * 4u : 0x80000000u;
        asm volatile("" : "+v"(off));
        return (int32_t)off;
    };
    float stg[LAT_STAGE];
#pragma unroll
    for (int u = 0; u < LAT_STAGE; ++u) stg[u] = buffer_load_f32(rs, col_off(j0 - h + lane + 64 * u));
#pragma unroll
    for (int u = 0; u < LAT_STAGE; ++u)
        if (lane + 64 * u < L) seg[lane + 64 * u] = stg[u];
    for (int q = lane + 64 * LAT_STAGE; q < L; q += 64) seg[q] = buffer_load_f32(rs, col_off(j0 - h + q));
    if constexpr (KT == 0)
        for (int t = lane; t < K; t += 64) taps[t] = kx[(size_t)i * K + t];
    __syncthreads();
    // lane's outputs j0 + 4 lane + q, q < 4: sum_t taps[t] seg[4 lane + 2h + q - t]
    float acc[LAT_PER_LANE];
#pragma unroll
    for (int q = 0; q < LAT_PER_LANE; ++q) acc[q] = 0.0f;
    if constexpr (KT > 0) {
        constexpr int H = (KT - 1) / 2;
        const float* trow = kx + (size_t)i * KT;  // wave-uniform: scalar loads
        float win[KT + LAT_PER_LANE - 1];          // win[k] = seg[4 lane + k]
#pragma unroll
        for (int k = 0; k < KT + LAT_PER_LANE - 1; ++k) win[k] = seg[LAT_PER_LANE * lane + k];
#pragma unroll
        for (int t = 0; t < KT; ++t) {
            const float tap = trow[t];
#pragma unroll
            for (int q = 0; q < LAT_PER_LANE; ++q) acc[q] = fmaf(tap, win[2 * H + q - t], acc[q]);
        }
    } else {
        const int base = LAT_PER_LANE * lane + 2 * h;
        int t = 0;
        if (K >= 5) {
            // taps in groups of 4 over a 7-sample window v[k] = seg[base - t - 3 + k]
            // (every index in [4 lane, 255 + 2h] for h >= 2); the next group's
            // window keeps 3 of these samples and reads 4
            float v[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) v[k] = seg[base - 3 + k];
            for (; t + 3 < K; t += 4) {
                float tp[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) tp[u] = taps[t + u];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = 0; q < LAT_PER_LANE; ++q) acc[q] = fmaf(tp[u], v[q - u + 3], acc[q]);
                if (t + 7 < K) {
                    v[6] = v[2];
                    v[5] = v[1];
                    v[4] = v[0];
#pragma unroll
                    for (int k = 0; k < 4; ++k) v[k] = seg[base - t - 7 + k];
                }
            }
        }
        for (; t < K; ++t) {  // the last K mod 4 taps (all of them when K < 5)
            const float k = taps[t];
#pragma unroll
            for (int q = 0; q < LAT_PER_LANE; ++q) acc[q] = fmaf(k, seg[base + q - t], acc[q]);
        }
    }
    // stores through the row's range check: columns past X (and every column
    // of a spare wave, whose record is empty) are dropped, so no store is
    // conditional; separate opaque offsets keep the four stores from being
    // merged into one wide store whose range check would treat them together
    const auto ro = make_rsrc(out + (size_t)row * X, live ? (uint32_t)X * 4u : 0u);
#pragma unroll
    for (int q = 0; q < LAT_PER_LANE; ++q) {
        int off = (j0 + LAT_PER_LANE * lane + q) * 4;
        asm volatile("" : "+v"(off));
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[q]), ro, off, 0, 0);
    }
}

}  // namespace
}  // namespace tidas

using namespace tidas;

extern "C" int32_t tidas_apply_lateral(const float* kernels_x, int32_t K, const float* in, int32_t B, int32_t Z,
                                       int32_t X, float* out, void* stream) {
    if (!kernels_x || !in || !out) return fail(TIDAS_EINVAL, "tidas_apply_lateral: null pointer");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_apply_lateral: K must be odd and >= 1");
    if (B < 1 || Z < 1 || X < 1) return fail(TIDAS_EINVAL, "tidas_apply_lateral: B, Z, X must be >= 1");
    if ((const void*)in == (const void*)out || (const void*)kernels_x == (const void*)out)
        return fail(TIDAS_EINVAL, "tidas_apply_lateral: output aliases an input");
    if (K > 1535) return fail(TIDAS_EUNSUPPORTED, "tidas_apply_lateral: K too large for the LDS segments");
    if ((int64_t)X + 2 * (int64_t)K + LAT_SEG >= (1 << 29))
        return fail(TIDAS_EUNSUPPORTED, "tidas_apply_lateral: rows too long for 32-bit offsets");
    const int32_t n_seg = (X + LAT_SEG - 1) / LAT_SEG;
    const int64_t n_waves = (int64_t)B * Z * n_seg;
    if (n_waves > INT32_MAX) return fail(TIDAS_EUNSUPPORTED, "tidas_apply_lateral: too many rows");
    const dim3 grid((uint32_t)((n_waves + LAT_WAVES - 1) / LAT_WAVES)), block(64 * LAT_WAVES);
    hipStream_t s = (hipStream_t)stream;
    const int32_t nw = (int32_t)n_waves;
    const bool fixed = K == 17 || K == 33 || K == 65;
    const size_t lds = (size_t)LAT_WAVES * lat_wave_floats(K, !fixed) * sizeof(float);
    switch (K) {
        case 17: hipLaunchKernelGGL(lateral_pass_kernel<17>, grid, block, lds, s, kernels_x, K, in, Z, X, n_seg, nw, out); break;
        case 33: hipLaunchKernelGGL(lateral_pass_kernel<33>, grid, block, lds, s, kernels_x, K, in, Z, X, n_seg, nw, out); break;
        case 65: hipLaunchKernelGGL(lateral_pass_kernel<65>, grid, block, lds, s, kernels_x, K, in, Z, X, n_seg, nw, out); break;
        default: hipLaunchKernelGGL(lateral_pass_kernel<0>, grid, block, lds, s, kernels_x, K, in, Z, X, n_seg, nw, out); break;
    }
    return check_launch("tidas_apply_lateral");
}
