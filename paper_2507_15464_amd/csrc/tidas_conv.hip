// The tiDAS line model (Sec. 2.4, eqn:line_conv) as a per-output-row depth
// convolution of a reflectivity map, and its transpose.
//
//   forward:  Y[b][i][j]  = sum_t K[i][t] * R[b][i - t + h][j]          t = 0..K-1
//   adjoint:  Rb[b][s][j] = sum_t K[s + t - h][t] * Yb[b][s + t - h][j]
//
// gfx950 mapping.  A workgroup owns a tile of 64 lateral columns (one per
// lane) x TZ = WAVES * RZ depth rows (RZ consecutive rows per wave).  The
// input rows the tile needs, [i0 - h, i0 + TZ + h), are staged once in LDS
// with coalesced 256-byte row loads (zero outside the image), so each input
// value is fetched from HBM/L2 about (TZ + K - 1) / TZ times.  Each lane keeps
// RZ accumulators.  The kernel taps are identical for the 64 lanes of a wave
// (they depend on the row only), so they are read with scalar loads into
// SGPRs and used directly as the scalar operand of v_fma_f32: no LDS or VGPR
// traffic for taps at all.
//
// Forward: for a block of RZ consecutive taps [t0, t0 + RZ) the RZ x RZ
// products need 2 RZ - 1 consecutive input rows; a sliding window of those
// rows lives in VGPRs and moves by RZ rows per block, so each LDS read feeds
// RZ FMAs.  Each output row's RZ taps of the block are contiguous in the bank
// (one wide scalar load).
// Adjoint: source row i contributes to the wave's output rows s = wi0 + r with
// tap K[i][i - wi0 + h - r]: RZ contiguous taps of row i, so the loop runs over
// source rows, one LDS read and one wide scalar load per RZ FMAs.
//
// Blocks are remapped so that each XCD receives a contiguous range of
// tiles (consecutive depth tiles of one column strip), which keeps the shared
// halo rows in that XCD's L2.
#include "common.hpp"

namespace tidas {

// Bijective remap of the linear block id: hardware dispatches block L to XCD
// L % 8; logical tiles [x * q + min(x, r), ...) go to XCD x.
__device__ __forceinline__ int xcd_remap(int L, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = L & 7, slot = L >> 3;
    return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

struct ConvGeom {
    int32_t K, h, B, Z, X;
    int32_t n_rt, n_ct, n_blocks;
};

template <int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void tidas_fwd_kernel(const ConvGeom g, const float* __restrict__ Kb,
                                                               const float* __restrict__ R,
                                                               float* __restrict__ Y) {
    constexpr int TZ = RZ * WAVES;
    extern __shared__ float tile[];  // [RZ pad + TZ + K - 1][64]
    const int lg = xcd_remap(blockIdx.x, g.n_blocks);
    const int rt = lg % g.n_rt;
    const int ct = (lg / g.n_rt) % g.n_ct;
    const int b = lg / (g.n_rt * g.n_ct);
    const int i0 = rt * TZ, j0 = ct * 64;
    const int K = g.K, h = g.h, Z = g.Z, X = g.X;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = j0 + lane;
    const bool col_ok = j < X;
    const float* Rb = R + (size_t)b * Z * X;

    // stage input rows i0 - h .. i0 + TZ + h - 1 after RZ zero rows of padding
    const int rows = TZ + K - 1;
    for (int r = wave; r < RZ; r += WAVES) tile[r * 64 + lane] = 0.0f;
    for (int r = wave; r < rows; r += WAVES) {
        const int s = i0 - h + r;
        float v = 0.0f;
        if (col_ok && s >= 0 && s < Z) v = Rb[(size_t)s * X + j];
        tile[(RZ + r) * 64 + lane] = v;
    }
    __syncthreads();

    const int wi0 = i0 + wave * RZ;
    // tap row pointers (rows past the image are clamped; their outputs are not stored)
    const float* krow[RZ];
#pragma unroll
    for (int r = 0; r < RZ; ++r) krow[r] = Kb + (size_t)min(wi0 + r, Z - 1) * K;

    float acc[RZ];
    float win[2 * RZ];
#pragma unroll
    for (int r = 0; r < RZ; ++r) acc[r] = 0.0f;
    // window of tap block starting at t0: input rows wi0 + h - t0 - (RZ-1) + k,
    // k = 0 .. 2RZ-2, i.e. tile rows RZ + wave*RZ + 2h - t0 - (RZ-1) + k
    int base = RZ + wave * RZ + 2 * h - (RZ - 1);
#pragma unroll
    for (int k = 0; k < 2 * RZ - 1; ++k) win[k] = tile[(base + k) * 64 + lane];

    const int nfull = K / RZ;
    for (int blk = 0; blk < nfull; ++blk) {
        const int t0 = blk * RZ;
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
#pragma unroll
            for (int jj = 0; jj < RZ; ++jj) acc[r] = fmaf(krow[r][t0 + jj], win[RZ - 1 + r - jj], acc[r]);
        }
        // slide the window up by RZ rows
        base -= RZ;
#pragma unroll
        for (int k = 2 * RZ - 2; k >= RZ; --k) win[k] = win[k - RZ];
#pragma unroll
        for (int k = 0; k < RZ; ++k) win[k] = tile[(base + k) * 64 + lane];
    }
    const int t0 = nfull * RZ;
    const int rem = K - t0;  // 0 .. RZ-1 remaining taps (uniform)
    if (rem > 0) {
#pragma unroll
        for (int jj = 0; jj < RZ; ++jj) {
            if (jj < rem) {
#pragma unroll
                for (int r = 0; r < RZ; ++r) acc[r] = fmaf(krow[r][t0 + jj], win[RZ - 1 + r - jj], acc[r]);
            }
        }
    }
    if (col_ok) {
        float* Yb = Y + (size_t)b * Z * X;
#pragma unroll
        for (int r = 0; r < RZ; ++r)
            if (wi0 + r < Z) Yb[(size_t)(wi0 + r) * X + j] = acc[r];
    }
}

template <int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void tidas_adj_kernel(const ConvGeom g, const float* __restrict__ Kb,
                                                               const float* __restrict__ Ybar,
                                                               float* __restrict__ Rbar) {
    constexpr int TZ = RZ * WAVES;
    extern __shared__ float tile[];  // [TZ + K - 1][64]
    const int lg = xcd_remap(blockIdx.x, g.n_blocks);
    const int rt = lg % g.n_rt;
    const int ct = (lg / g.n_rt) % g.n_ct;
    const int b = lg / (g.n_rt * g.n_ct);
    const int i0 = rt * TZ, j0 = ct * 64;
    const int K = g.K, h = g.h, Z = g.Z, X = g.X;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = j0 + lane;
    const bool col_ok = j < X;
    const float* Yb = Ybar + (size_t)b * Z * X;

    const int rows = TZ + K - 1;
    for (int r = wave; r < rows; r += WAVES) {
        const int s = i0 - h + r;
        float v = 0.0f;
        if (col_ok && s >= 0 && s < Z) v = Yb[(size_t)s * X + j];
        tile[r * 64 + lane] = v;
    }
    __syncthreads();

    const int wi0 = i0 + wave * RZ;
    float acc[RZ];
#pragma unroll
    for (int r = 0; r < RZ; ++r) acc[r] = 0.0f;

    // source rows i = wi0 - h + u, u = 0 .. K + RZ - 2; tap of output r: tb - r, tb = u
    const int u_lo = max(0, h - wi0);                 // skip rows above the image
    const int u_hi = min(K + RZ - 2, Z - 1 - wi0 + h); // and below it
    // interior rows have every tap tb - r, r < RZ, inside [0, K)
    const int u_in_lo = max(u_lo, RZ - 1);
    const int u_in_hi = min(u_hi, K - 1);
    for (int u = u_lo; u <= u_hi; ++u) {
        const int i = wi0 - h + u;
        const float y = tile[(i - (i0 - h)) * 64 + lane];
        const float* kr = Kb + (size_t)i * K + u;  // kr[-r] = K[i][u - r]
        if (u >= u_in_lo && u <= u_in_hi) {
#pragma unroll
            for (int r = 0; r < RZ; ++r) acc[r] = fmaf(kr[-r], y, acc[r]);
        } else {
#pragma unroll
            for (int r = 0; r < RZ; ++r) {
                const int t = u - r;
                if (t >= 0 && t < K) acc[r] = fmaf(kr[-r], y, acc[r]);
            }
        }
    }
    if (col_ok) {
        float* Rb = Rbar + (size_t)b * Z * X;
#pragma unroll
        for (int r = 0; r < RZ; ++r)
            if (wi0 + r < Z) Rb[(size_t)(wi0 + r) * X + j] = acc[r];
    }
}

constexpr int CONV_RZ = 16;
constexpr int CONV_WAVES = 4;
constexpr size_t LDS_LIMIT = 160 * 1024;

static int32_t conv_common(const char* name, const float* kernels, int32_t K, const float* in, int32_t B,
                           int32_t Z, int32_t X, float* out, ConvGeom& g) {
    if (!kernels || !in || !out) return fail(TIDAS_EINVAL, std::string(name) + ": null pointer");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, std::string(name) + ": K must be odd and >= 1");
    if (B < 1 || Z < 1 || X < 1) return fail(TIDAS_EINVAL, std::string(name) + ": B, Z, X must be >= 1");
    if ((const void*)in == (const void*)out || (const void*)kernels == (const void*)out)
        return fail(TIDAS_EINVAL, std::string(name) + ": output aliases an input");
    const size_t lds = (size_t)(CONV_RZ + CONV_RZ * CONV_WAVES + K - 1) * 64 * sizeof(float);
    if (lds > LDS_LIMIT) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": K too large for the LDS tile");
    g.K = K;
    g.h = (K - 1) / 2;
    g.B = B;
    g.Z = Z;
    g.X = X;
    g.n_rt = (Z + CONV_RZ * CONV_WAVES - 1) / (CONV_RZ * CONV_WAVES);
    g.n_ct = (X + 63) / 64;
    const int64_t nb = (int64_t)g.n_rt * g.n_ct * B;
    if (nb > INT32_MAX) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": too many tiles");
    g.n_blocks = (int32_t)nb;
    return TIDAS_OK;
}

}  // namespace tidas

using namespace tidas;

extern "C" int32_t tidas_apply(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z,
                               int32_t X, float* image, void* stream) {
    ConvGeom g;
    int32_t st = conv_common("tidas_apply", kernels, K, refl, B, Z, X, image, g);
    if (st) return st;
    const size_t lds = (size_t)(CONV_RZ + CONV_RZ * CONV_WAVES + K - 1) * 64 * sizeof(float);
    hipLaunchKernelGGL((tidas_fwd_kernel<CONV_RZ, CONV_WAVES>), dim3(g.n_blocks), dim3(CONV_WAVES * 64), lds,
                       (hipStream_t)stream, g, kernels, refl, image);
    return check_launch("tidas_apply");
}

extern "C" int32_t tidas_adjoint(const float* kernels, int32_t K, const float* image_bar, int32_t B, int32_t Z,
                                 int32_t X, float* refl_bar, void* stream) {
    ConvGeom g;
    int32_t st = conv_common("tidas_adjoint", kernels, K, image_bar, B, Z, X, refl_bar, g);
    if (st) return st;
    const size_t lds = (size_t)(CONV_RZ * CONV_WAVES + K - 1) * 64 * sizeof(float);
    hipLaunchKernelGGL((tidas_adj_kernel<CONV_RZ, CONV_WAVES>), dim3(g.n_blocks), dim3(CONV_WAVES * 64), lds,
                       (hipStream_t)stream, g, kernels, image_bar, refl_bar);
    return check_launch("tidas_adjoint");
}
