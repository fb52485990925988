// Gradient of the line model in its per-row kernels (gfx950).
//
// The line model (Sec. 2.4, eqn:line_conv) is linear in its kernels, so for
// Ybar = dL/dY the kernel gradient is a correlation of Ybar with the
// reflectivity map along depth, summed over frames and lateral columns:
//
//   Kbar[i][m+h] = sum_b sum_j Ybar[b][i][j] * R[b][i-m][j],   R = 0 outside [0, Z).
//
// Read as matrices over the inner index n = (b, j), Kbar[i][m+h] is entry
// (i, i - m) of Ybar R^T (Z x Z): the band |i - s| <= h of one dense product.
// That is a contraction with a long inner dimension (B X), so it runs on the
// matrix cores: in split-bfloat16 form (below) when rows can be read 16 bytes
// at a time, else on the FP32 matrix cores (v_mfma_f32_32x32x2_f32, float32
// products and sums).  Both share the tiling:
//
//   * a workgroup of 4 waves owns 128 output rows; wave w owns rows
//     i0 + 32 w .. + 31 and the NT 32-row source tiles starting at
//     i0 + 32 w - h (+ 32 NT per band pass when the band needs more tiles
//     than one pass holds), one 32 x 32 accumulator per tile;
//   * the inner index walks column chunks of one frame (32 columns in
//     float32, 16 in split form): Ybar's 128 rows and the band's 32 (3 + NT)
//     source rows of the chunk are staged in LDS (float32 rows padded to 36
//     floats: the 16-byte column reads of 8 consecutive rows hit distinct
//     banks), the next chunk's values wait in registers;
//   * in each product the two lane halves take different columns of the
//     chunk (one each in float32, eight each in split form), so one
//     instruction sums 2 or 16 inner terms;
//   * the inner index is cut into a fixed number of contiguous ranges, one
//     per workgroup column of the grid; each range's sums land in its own
//     slice of a temporary buffer and a second kernel adds the slices in a
//     fixed order, in double precision: the result is reproducible bit for
//     bit on one device type.
//
// Edges need no branches: source rows outside the frame read 0 through the
// buffer range check, columns at or past X are given an offset past the
// record, rows past Z give zero accumulators that are not stored.

#include <algorithm>

#include "common.hpp"

namespace tidas {
namespace {

typedef float kg_floatx4 __attribute__((ext_vector_type(4)));
typedef float kg_floatx16 __attribute__((ext_vector_type(16)));

constexpr int KG_TZ = 128;      // output rows per workgroup
constexpr int KG_CW = 32;       // columns per staged chunk
constexpr int KG_LS = 36;       // LDS row stride (floats)
constexpr int KG_MAX_NT = 6;    // source tiles per wave and band pass
constexpr int KG_THREADS = 256;

struct KgGeom {
    int32_t K, h, B, Z, X;
    int32_t n_rt, n_pass, n_split;
    int32_t n_cc;      // 32-column chunks per frame
    int64_t n_chunk;   // B * n_cc
};

__device__ __forceinline__ float kg_load(__amdgpu_buffer_rsrc_t r, int32_t byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

__device__ __forceinline__ const float* kg_uniform(const float* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const float*>(((uint64_t)hi << 32) | lo);
}

// grid: n_rt * n_pass * n_split workgroups; part: [n_split][Z][K].  Serves
// frames whose rows cannot be read 16 bytes at a time (X % 4 != 0 or
// unaligned); the split-bfloat16 kernel below serves the others.
template <int NT>
__global__ __launch_bounds__(KG_THREADS, 2) void kgrad_kernel(const KgGeom g, const float* __restrict__ Yb,
                                                              const float* __restrict__ R, float* __restrict__ part) {
    constexpr int BR = 32 * (3 + NT);       // band rows staged per chunk
    constexpr int RPI = 8;                  // rows one staging instruction covers
    constexpr int RY = KG_TZ / RPI;         // Ybar staging loads per thread
    constexpr int RR = BR / RPI;            // band staging loads per thread
    __shared__ __attribute__((aligned(16))) float sY[KG_TZ * KG_LS];
    __shared__ __attribute__((aligned(16))) float sR[BR * KG_LS];

    const int rt = blockIdx.x % g.n_rt;
    const int pass = (blockIdx.x / g.n_rt) % g.n_pass;
    const int sp = blockIdx.x / (g.n_rt * g.n_pass);
    const int i0 = rt * KG_TZ;
    const int s_lo = i0 - g.h + pass * 32 * NT;  // first staged source row
    const int X = g.X, Z = g.Z;
    const uint32_t frame_bytes = (uint32_t)((size_t)Z * X * sizeof(float));
    const size_t fstride = (size_t)Z * X;

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int half = lane >> 5, r32 = lane & 31;
    // staging: thread t moves column st_col of rows st_row + RPI k
    const int st_col = t & 31;
    const int st_row = t >> 5;

    const int64_t c_begin = g.n_chunk * sp / g.n_split;
    const int64_t c_end = g.n_chunk * (sp + 1) / g.n_split;
    // chunk c = frame b, columns 32 cc ..; walked incrementally
    int b_next = (int)(c_begin / g.n_cc), cc_next = (int)(c_begin % g.n_cc);

    float vy[RY], vr[RR];
    auto load = [&](__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
    };
    auto fetch = [&]() {
        const int b = b_next, j = cc_next * KG_CW + st_col;
        if (++cc_next == g.n_cc) {
            cc_next = 0;
            ++b_next;
        }
        const auto ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(kg_uniform(Yb + (size_t)b * fstride)),
                                                          (short)0, (int)frame_bytes, 0x00020000);
        const auto rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(kg_uniform(R + (size_t)b * fstride)),
                                                          (short)0, (int)frame_bytes, 0x00020000);
        // columns at or past X: the top offset bit puts the load past the
        // record (an opaque mask, so the loads stay unconditional)
        uint32_t cm = j < X ? 0u : 0x80000000u;
        asm volatile("" : "+v"(cm));
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int row = i0 + st_row + RPI * k;
            vy[k] = load(ry, (uint32_t)((row * X + j) * 4) | cm);
        }
#pragma unroll
        for (int k = 0; k < RR; ++k) {
            const int row = s_lo + st_row + RPI * k;
            vr[k] = load(rr, (uint32_t)((row * X + j) * 4) | cm);
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int k = 0; k < RY; ++k) sY[(st_row + RPI * k) * KG_LS + st_col] = vy[k];
#pragma unroll
        for (int k = 0; k < RR; ++k) sR[(st_row + RPI * k) * KG_LS + st_col] = vr[k];
    };

    kg_floatx16 acc[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;

    // this lane's rows in LDS: Ybar row 32 w + r32, band rows 32 (w + q) + r32;
    // lane half `half` reads columns 16 half .. 16 half + 15
    const float* ya = sY + (32 * wave + r32) * KG_LS + 16 * half;
    const float* rb = sR + (32 * wave + r32) * KG_LS + 16 * half;

    if (c_begin < c_end) fetch();
    for (int64_t c = c_begin; c < c_end; ++c) {
        __syncthreads();  // the previous chunk's reads are done
        stage();
        __syncthreads();
        if (c + 1 < c_end) fetch();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const kg_floatx4 a = *reinterpret_cast<const kg_floatx4*>(ya + 4 * u);
            kg_floatx4 bq[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) bq[q] = *reinterpret_cast<const kg_floatx4*>(rb + 32 * q * KG_LS + 4 * u);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int q = 0; q < NT; ++q)
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], bq[q][e], acc[q], 0, 0, 0);
        }
    }

    // accumulator q, register v: output row i = i0 + 32 w + 8 (v / 4) + 4 half
    // + v % 4, source row s = s_lo + 32 (w + q) + r32, tap m = i - s
    float* out = part + (size_t)sp * Z * g.K;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int s = s_lo + 32 * (wave + q) + r32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = i0 + 32 * wave + 8 * (v >> 2) + 4 * half + (v & 3);
            const int m = i - s;
            if (i < Z && m >= -g.h && m <= g.h) out[(size_t)i * g.K + (m + g.h)] = acc[q][v];
        }
    }
}

// Split-bfloat16 form (X % 4 == 0, 16-byte aligned frames): every staged value v
// is cut exactly, by truncation, into three bfloat16 parts v0 + v1 + v2 (v0
// the top 16 bits, v1 the top 16 bits of v - v0, v2 the rest, at most 8
// significant bits), stored as three LDS planes, and a·b is taken as a0b0 +
// a0b1 + a1b0 + a0b2 + a1b1 + a2b0 on v_mfma_f32_32x32x16_bf16 (each product
// exact, the dropped terms below 2^-20 |ab|, sums in float32): 6 x 32
// matrix cycles per 16 inner terms and tile instead of 8 x 64 in float32.
// Chunks of 16 columns, plane rows of 32 bytes: the 16-byte reads of 8
// consecutive rows start 8 banks apart and so hit distinct banks without
// padding, and 37 KB of LDS at NT = 5 leaves room for three workgroups per
// compute unit (as many as the registers allow).
typedef __bf16 kg_bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t kg_u32x2 __attribute__((ext_vector_type(2)));
constexpr int KB_CW = 16;  // columns per chunk
constexpr int KB_LS = 16;  // plane row stride (bfloat16): 32 bytes, no padding

__device__ __forceinline__ void kg_split3(float v, uint32_t& w0, uint32_t& w1, uint32_t& w2) {
    const uint32_t u = __float_as_uint(v);
    const float r1 = v - __uint_as_float(u & 0xffff0000u);
    const uint32_t u1 = __float_as_uint(r1);
    const float r2 = r1 - __uint_as_float(u1 & 0xffff0000u);
    w0 = u;
    w1 = u1;
    w2 = __float_as_uint(r2);
}

template <int NT>
__global__ __launch_bounds__(KG_THREADS, 2) void kgrad_bf16_kernel(const KgGeom g, const float* __restrict__ Yb,
                                                                   const float* __restrict__ R,
                                                                   float* __restrict__ part) {
    constexpr int BR = 32 * (3 + NT);          // band rows staged per chunk
    constexpr int PY = KG_TZ * KB_LS;          // one Ybar plane (bfloat16)
    constexpr int PR = BR * KB_LS;             // one band plane
    constexpr int RY = KG_TZ / 64;             // Ybar staging loads per thread (64 rows each)
    constexpr int RR = (BR + 63) / 64;         // band staging loads per thread
    __shared__ __attribute__((aligned(16))) uint16_t sY[3 * PY];
    __shared__ __attribute__((aligned(16))) uint16_t sR[3 * PR];

    const int rt = blockIdx.x % g.n_rt;
    const int pass = (blockIdx.x / g.n_rt) % g.n_pass;
    const int sp = blockIdx.x / (g.n_rt * g.n_pass);
    const int i0 = rt * KG_TZ;
    const int s_lo = i0 - g.h + pass * 32 * NT;
    const int X = g.X, Z = g.Z;
    const uint32_t frame_bytes = (uint32_t)((size_t)Z * X * sizeof(float));
    const size_t fstride = (size_t)Z * X;

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int half = lane >> 5, r32 = lane & 31;
    // staging: thread t moves columns 4 (t % 4) .. + 3 of rows t / 4 + 64 k
    const int st_col = 4 * (t & 3), st_row = t >> 2;

    const int64_t c_begin = g.n_chunk * sp / g.n_split;
    const int64_t c_end = g.n_chunk * (sp + 1) / g.n_split;
    int b_next = (int)(c_begin / g.n_cc), cc_next = (int)(c_begin % g.n_cc);

    kg_floatx4 vy[RY], vr[RR];
    auto fetch = [&]() {
        const int b = b_next, j = cc_next * KB_CW + st_col;
        if (++cc_next == g.n_cc) {
            cc_next = 0;
            ++b_next;
        }
        const auto ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(kg_uniform(Yb + (size_t)b * fstride)),
                                                          (short)0, (int)frame_bytes, 0x00020000);
        const auto rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(kg_uniform(R + (size_t)b * fstride)),
                                                          (short)0, (int)frame_bytes, 0x00020000);
        uint32_t cm = j < X ? 0u : 0x80000000u;  // columns past X: past the record
        asm volatile("" : "+v"(cm));
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int row = i0 + st_row + 64 * k;
            vy[k] = __builtin_bit_cast(kg_floatx4,
                                       __builtin_amdgcn_raw_buffer_load_b128(ry, (uint32_t)((row * X + j) * 4) | cm, 0, 0));
        }
#pragma unroll
        for (int k = 0; k < RR; ++k) {
            const int row = s_lo + st_row + 64 * k;
            vr[k] = __builtin_bit_cast(kg_floatx4,
                                       __builtin_amdgcn_raw_buffer_load_b128(rr, (uint32_t)((row * X + j) * 4) | cm, 0, 0));
        }
    };
    // the three planes of 4 values, 4 bfloat16 each (two 32-bit words per plane)
    auto put = [&](uint16_t* base, int plane_stride, int row, const kg_floatx4& v) {
        uint32_t w[3][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) kg_split3(v[e], w[0][e], w[1][e], w[2][e]);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            kg_u32x2 q;
            q[0] = __builtin_amdgcn_perm(w[p][1], w[p][0], 0x07060302u);
            q[1] = __builtin_amdgcn_perm(w[p][3], w[p][2], 0x07060302u);
            *reinterpret_cast<kg_u32x2*>(base + p * plane_stride + row * KB_LS + st_col) = q;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int k = 0; k < RY; ++k) put(sY, PY, st_row + 64 * k, vy[k]);
#pragma unroll
        for (int k = 0; k < RR; ++k)
            if (st_row + 64 * k < BR) put(sR, PR, st_row + 64 * k, vr[k]);
    };

    kg_floatx16 acc[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;

    // lane half `half` holds inner columns 8 half .. 8 half + 7 of the chunk
    const uint16_t* ya = sY + (32 * wave + r32) * KB_LS + 8 * half;
    const uint16_t* rb = sR + (32 * wave + r32) * KB_LS + 8 * half;
    constexpr int TA[6] = {0, 0, 1, 0, 1, 2};
    constexpr int TB[6] = {0, 1, 0, 2, 1, 0};

    if (c_begin < c_end) fetch();
    for (int64_t c = c_begin; c < c_end; ++c) {
        __syncthreads();  // the previous chunk's reads are done
        stage();
        __syncthreads();
        if (c + 1 < c_end) fetch();
        kg_bf16x8 a[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) a[p] = *reinterpret_cast<const kg_bf16x8*>(ya + p * PY);
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            kg_bf16x8 bq[3];
#pragma unroll
            for (int p = 0; p < 3; ++p) bq[p] = *reinterpret_cast<const kg_bf16x8*>(rb + p * PR + 32 * q * KB_LS);
#pragma unroll
            for (int u = 0; u < 6; ++u)
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[TA[u]], bq[TB[u]], acc[q], 0, 0, 0);
        }
    }

    float* out = part + (size_t)sp * Z * g.K;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int s = s_lo + 32 * (wave + q) + r32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = i0 + 32 * wave + 8 * (v >> 2) + 4 * half + (v & 3);
            const int m = i - s;
            if (i < Z && m >= -g.h && m <= g.h) out[(size_t)i * g.K + (m + g.h)] = acc[q][v];
        }
    }
}

// out[e] = sum over slices s = 0 .. n_split - 1 of part[s][e], in that order, in double
__global__ __launch_bounds__(256) void kgrad_reduce_kernel(const float* __restrict__ part, int32_t n_split,
                                                           int64_t n, float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float* p = part + e;
    double s = 0.0;
    int k = 0;
    for (; k + 8 <= n_split; k += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(k + u) * n];  // loads in flight together
#pragma unroll
        for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; k < n_split; ++k) s += (double)p[(size_t)k * n];
    out[e] = (float)s;
}

int kg_cu_count() {
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
    }
    return n_cu;
}

// vec (X % 4 == 0, 16-byte aligned frames): the split-bfloat16 kernel over
// 16-column chunks; otherwise the float32 kernel over 32-column chunks
template <int NT>
void launch_kgrad(bool vec, const KgGeom& g, const float* Yb, const float* R, float* part, hipStream_t stream) {
    const dim3 grid((uint32_t)((int64_t)g.n_rt * g.n_pass * g.n_split));
    if (vec) hipLaunchKernelGGL((kgrad_bf16_kernel<NT>), grid, dim3(KG_THREADS), 0, stream, g, Yb, R, part);
    else hipLaunchKernelGGL((kgrad_kernel<NT>), grid, dim3(KG_THREADS), 0, stream, g, Yb, R, part);
}

}  // namespace

// Tiling of one call: band tiles per pass, passes, inner ranges.  The ranges
// give about two workgroups per compute unit (each holds under 64 KB of LDS;
// three per compute unit, which the split kernel's registers and LDS allow,
// measured slower: 64.8 against 49.4 us on 64 frames of 1024 x 256, K = 129).
static KgGeom kgrad_geometry(int32_t K, int32_t B, int32_t Z, int32_t X, int chunk_cols, int* nt_out) {
    KgGeom g;
    g.K = K;
    g.h = (K - 1) / 2;
    g.B = B;
    g.Z = Z;
    g.X = X;
    g.n_rt = (Z + KG_TZ - 1) / KG_TZ;
    const int nt_all = (K + 31 + 31) / 32;  // tiles covering the 31 + K source rows of 32 output rows
    g.n_pass = (nt_all + KG_MAX_NT - 1) / KG_MAX_NT;
    const int nt = (nt_all + g.n_pass - 1) / g.n_pass;
    g.n_cc = (X + chunk_cols - 1) / chunk_cols;
    g.n_chunk = (int64_t)B * g.n_cc;
    const int64_t per_split = (int64_t)g.n_rt * g.n_pass;
    const int64_t want = (2 * (int64_t)kg_cu_count() + per_split - 1) / per_split;
    g.n_split = (int32_t)std::max<int64_t>(1, std::min<int64_t>(want, g.n_chunk));
    *nt_out = nt;
    return g;
}

}  // namespace tidas

using namespace tidas;

static bool kgrad_split_path(int32_t X, const void* refl, const void* image_bar) {
    return (X % 4) == 0 && ((uintptr_t)refl % 16) == 0 && ((uintptr_t)image_bar % 16) == 0;
}

extern "C" int32_t tidas_kernel_grad_kernel(int32_t X, const void* refl, const void* image_bar) {
    if (X < 1) return fail(TIDAS_EINVAL, "tidas_kernel_grad_kernel: X must be >= 1");
    return kgrad_split_path(X, refl, image_bar) ? TIDAS_KGRAD_SPLIT_BF16 : TIDAS_KGRAD_FP32;
}

// partial-sum slices of one call: [ranges][Z][K] floats
static size_t kgrad_part_bytes(int32_t K, int32_t B, int32_t Z, int32_t X, bool vec) {
    int nt = 1;
    const KgGeom g = kgrad_geometry(K, B, Z, X, vec ? KB_CW : KG_CW, &nt);
    return (size_t)g.n_split * Z * K * sizeof(float);
}

extern "C" size_t tidas_kernel_grad_workspace_bytes(int32_t K, int32_t B, int32_t Z, int32_t X) {
    if (K < 1 || (K % 2) == 0 || B < 1 || Z < 1 || X < 1) return 0;
    return std::max(kgrad_part_bytes(K, B, Z, X, true), kgrad_part_bytes(K, B, Z, X, false));
}

extern "C" int32_t tidas_kernel_grad(int32_t K, const float* refl, const float* image_bar, int32_t B, int32_t Z,
                                     int32_t X, float* kernels_bar, void* workspace, size_t workspace_bytes,
                                     void* stream) {
    if (!refl || !image_bar || !kernels_bar) return fail(TIDAS_EINVAL, "tidas_kernel_grad: null pointer");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_kernel_grad: K must be odd and >= 1");
    if (B < 1 || Z < 1 || X < 1) return fail(TIDAS_EINVAL, "tidas_kernel_grad: B, Z, X must be >= 1");
    if ((const void*)kernels_bar == (const void*)refl || (const void*)kernels_bar == (const void*)image_bar)
        return fail(TIDAS_EINVAL, "tidas_kernel_grad: output aliases an input");
    // every staged row offset (rows from -h - 32 to Z + h + 224) fits int32
    if (((int64_t)Z + 2 * (int64_t)K + 512) * X * 4 >= INT32_MAX)
        return fail(TIDAS_EUNSUPPORTED, "tidas_kernel_grad: frame too large for 32-bit offsets");
    int nt = 1;
    const bool vec = kgrad_split_path(X, refl, image_bar);
    const KgGeom g = kgrad_geometry(K, B, Z, X, vec ? KB_CW : KG_CW, &nt);
    if ((int64_t)g.n_rt * g.n_pass * g.n_split > INT32_MAX)
        return fail(TIDAS_EUNSUPPORTED, "tidas_kernel_grad: grid too large");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)Z * K;
    const size_t need = (size_t)g.n_split * n * sizeof(float);
    int32_t st = workspace_check("tidas_kernel_grad", workspace, workspace_bytes,
                                 tidas_kernel_grad_workspace_bytes(K, B, Z, X));
    if (st) return st;
    Workspace ws;
    if ((st = workspace_acquire("tidas_kernel_grad: partial sums", workspace, need, s, ws))) return st;
    float* part = (float*)ws.ptr;
    switch (nt) {
        case 1: launch_kgrad<1>(vec, g, image_bar, refl, part, s); break;
        case 2: launch_kgrad<2>(vec, g, image_bar, refl, part, s); break;
        case 3: launch_kgrad<3>(vec, g, image_bar, refl, part, s); break;
        case 4: launch_kgrad<4>(vec, g, image_bar, refl, part, s); break;
        case 5: launch_kgrad<5>(vec, g, image_bar, refl, part, s); break;
        default: launch_kgrad<6>(vec, g, image_bar, refl, part, s); break;
    }
    st = check_launch("tidas_kernel_grad");
    if (!st) {
        hipLaunchKernelGGL(kgrad_reduce_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, part, g.n_split,
                           n, kernels_bar);
        st = check_launch("tidas_kernel_grad(reduce)");
    }
    const int32_t st2 = workspace_release("tidas_kernel_grad: partial sums", ws, s);
    return st ? st : st2;
}
