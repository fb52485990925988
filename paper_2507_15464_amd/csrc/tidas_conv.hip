// The tiDAS line model (Sec. 2.4, eqn:line_conv) as a per-output-row depth
// convolution of a reflectivity map, and its transpose.
//
//   forward:  Y[b][i][j]  = sum_t K[i][t] * R[b][i - t + h][j]          t = 0..K-1
//   adjoint:  Rb[b][s][j] = sum_t K[s + t - h][t] * Yb[b][s + t - h][j]
//
// Kernels, in the order the dispatcher tries them (conv_launch):
//   tidas_b4_kernel    split-bfloat16 matrix cores, 128 x 256 tiles (K <= 161,
//                      batches with a tile per compute unit)
//   tidas_bx6_kernel   split-bfloat16 matrix cores, 64 x 256 tiles (K <= 321;
//                      also the tile of the ragged batch kernel)
//   tidas_mfma_kernel  float32 matrix cores (larger K)
//   tidas_fwd_kernel / tidas_adj_kernel  vector ALU (the first version,
//                      described next; the fallback when no tile fits LDS)
//
// Vector-ALU mapping.  A workgroup owns a tile of 64 lateral columns (one per
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
#include <algorithm>
#include <climits>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "common.hpp"

namespace tidas {

TIDAS_DEBUG_FLAGS_DEFINE(conv)

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
    int32_t vec4;  // input rows may be read as float4 (X % 4 == 0 and 16-byte aligned base)
    // epilogue: out = alpha * (operator applied to the input) + beta * base
    // (base may be null; it may alias out, element for element)
    float alpha, beta;
    const float* base;
};

__device__ __forceinline__ float epilogue(const ConvGeom& g, float acc, size_t idx) {
    float v = g.alpha * acc;
    if (g.base) v = fmaf(g.beta, g.base[idx], v);
    return v;
}

template <int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void tidas_fwd_kernel(const ConvGeom g, const float* __restrict__ Kb,
                                                               const float* __restrict__ R,
                                                               float* Y) {
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
#pragma unroll
        for (int r = 0; r < RZ; ++r)
            if (wi0 + r < Z) {
                const size_t idx = (size_t)b * Z * X + (size_t)(wi0 + r) * X + j;
                Y[idx] = epilogue(g, acc[r], idx);
            }
    }
}

template <int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void tidas_adj_kernel(const ConvGeom g, const float* __restrict__ Kb,
                                                               const float* __restrict__ Ybar,
                                                               float* Rbar) {
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
#pragma unroll
        for (int r = 0; r < RZ; ++r)
            if (wi0 + r < Z) {
                const size_t idx = (size_t)b * Z * X + (size_t)(wi0 + r) * X + j;
                Rbar[idx] = epilogue(g, acc[r], idx);
            }
    }
}

// ------------------------------------------------------------------------
// Matrix-core path.  Over a tile of 32 output rows x 256 columns the line model
// is a dense product Y_tile = M_tile R_tile with the banded matrix
// M_tile[r][c] = K[i0 + r][r - c + 2h] (zero off the band) and R_tile the input
// rows [i0 - h, i0 + 32 + h).  It runs on v_mfma_f32_16x16x4_f32 (exact float32
// products, float32 accumulation).  Operand layouts of that instruction:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): register q of lane l holds D[4 (l / 16) + q][l % 16]
// 8 waves per tile; wave w owns output rows 16 (w / 4) .. +16 and a 64-column
// quarter of the tile, as four 16 x 16 accumulators ("chains").  Chain c of
// lane column j covers image column 4 j + c, so one 16-byte load per lane
// (four consecutive columns of one input row) feeds all four chains, and the
// four results of an output row are again four consecutive columns (one
// 16-byte store).  Each wave walks only the band: input rows
// r0 .. r0 + 15 + K - 1, four per step, (K + 15) / 4 steps.
// The kernel rows of the tile sit in LDS (direct-to-LDS buffer loads) with 20
// zeros of padding before tap 0 and a row stride = 1 (mod 32) words, so the two
// k-groups of a half-wave fall on even and odd banks: no conflicts.  The
// reflectivity operand is streamed from L2 through a register ring, PD steps
// ahead.  The adjoint is the same product with the transposed band
// M^T[s][i] = K[i][i - s + h], staged as KT[s][t] = K[s + h - t][K - 1 - t].
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int MF_TZ = 32;        // output rows per tile (two 16-row M-blocks)
constexpr int MF_TN = 256;       // columns per tile (four 64-column quarters)
constexpr int MF_THREADS = 512;  // 8 waves
constexpr int MF_LPAD = 20;      // zero taps before tap 0 in the LDS kernel rows

__host__ __device__ constexpr int mf_nsteps(int K) { return (K + 15 + 3) / 4; }
__host__ __device__ constexpr int mf_kstride(int K) {
    // >= K + 15 + MF_LPAD (largest tap index read) + 1 and = 1 (mod 32)
    return ((K + 15 + MF_LPAD + 1 + 31 - 1) / 32) * 32 + 1;
}
// rounded up to whole 64-entry chunks: the last direct-to-LDS wave load writes a full chunk
__host__ __device__ constexpr size_t mf_lds_bytes(int K) {
    return (size_t)((MF_TZ * mf_kstride(K) + 63) / 64) * 64 * sizeof(float);
}

// One 32 x 256 output tile of one frame.  Kb: the frame's [Z][K] bank; Ib, Ob,
// base_b: the frame's [Z][X] input, output and (optional) epilogue base.  kt:
// the workgroup's LDS kernel tile.  VEC: X % 4 == 0 and 16-byte aligned rows
// (one 16-byte load / store per lane and step); otherwise four dword loads.
// All threads of the workgroup call it (it contains barriers).
template <bool ADJ, int PD, bool VEC>
__device__ __forceinline__ void mfma_tile(const float* __restrict__ Kb, const float* __restrict__ Ib, float* Ob,
                                          const float* base_b, float alpha, float beta, int K, int Z, int X, int i0,
                                          int j0, float* kt) {
    const int h = (K - 1) >> 1;
    const int KS = mf_kstride(K);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr uint32_t OOB = 0x80000000u;

    // kernel tile, flat [MF_TZ][KS]: one dword wave load = 64 consecutive entries;
    // entries outside the taps (or past the image) read 0 through the range check
    {
        const auto rs_k = make_rsrc(Kb, (uint32_t)((size_t)Z * K * sizeof(float)));
        const int nchunks = (MF_TZ * KS + 63) / 64;
        for (int ch = wave; ch < nchunks; ch += MF_THREADS / 64) {
            const int e0 = ch * 64;
            const int e = e0 + lane;
            const int r = e / KS;
            const int t = e - r * KS - MF_LPAD;
            const int row = i0 + r;
            uint32_t off = OOB;
            if (r < MF_TZ && t >= 0 && t < K && row < Z) {
                if (!ADJ) {
                    off = (uint32_t)(((size_t)row * K + t) * 4);
                } else {
                    const int src = row + h - t;
                    if (src >= 0 && src < Z) off = (uint32_t)(((size_t)src * K + (K - 1 - t)) * 4);
                }
            }
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_k, (__attribute__((address_space(3))) void*)(kt + e0), 4, off,
                                                     0, 0, 0);
        }
    }

    const int r0 = (wave >> 2) * 16;  // M-block rows within the tile
    const int n0 = (wave & 3) * 64;   // column quarter
    const int li = lane & 15, lk = lane >> 4;
    const int nsteps = mf_nsteps(K);
    // B: step s reads input row i0 - h + r0 + 4 s + lk, columns col .. col + 3.
    // int32 byte offsets from the frame base: rows above the image are negative
    // (huge unsigned), rows below are past the end: both read 0.
    const auto rs_in = make_rsrc(Ib, (uint32_t)((size_t)Z * X * sizeof(float)));
    const int col = j0 + n0 + 4 * li;
    const int step_bytes = 4 * X * 4;
    const int off0 = ((i0 - h + r0 + lk) * X + col) * 4;
    auto load_b = [&](int off) -> floatx4 {
        if (VEC) return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs_in, off, 0, 0));
        floatx4 v;
        v[0] = buffer_load_f32(rs_in, off);
        v[1] = buffer_load_f32(rs_in, off + 4);
        v[2] = buffer_load_f32(rs_in, off + 8);
        v[3] = buffer_load_f32(rs_in, off + 12);
        return v;
    };
    floatx4 q[PD];
#pragma unroll
    for (int u = 0; u < PD; ++u) q[u] = load_b(off0 + u * step_bytes);
    __builtin_amdgcn_s_waitcnt(0);  // drain the LDS-direct loads
    __syncthreads();

    // A: step s, lane (li, lk): M[r0 + li][r0 + 4 s + lk] -> tap t = li - lk - 4 s + 2h
    const float* a_ptr = kt + (r0 + li) * KS + (li - lk + 2 * h + MF_LPAD);
    floatx4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int last = nsteps - 1;
    float a_cur = a_ptr[0];
    int s0 = 0;
    for (; s0 + PD <= nsteps; s0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            const int st = s0 + u;
            const float a_nxt = a_ptr[-4 * min(st + 1, last)];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_cur, q[u][c], acc[c], 0, 0, 0);
            q[u] = load_b(off0 + (st + PD) * step_bytes);
            a_cur = a_nxt;
        }
    }
#pragma unroll
    for (int u = 0; u < PD; ++u) {
        const int st = s0 + u;
        if (st < nsteps) {
            const float a = a_ptr[-4 * st];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, q[u][c], acc[c], 0, 0, 0);
        }
    }

#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        const int row = i0 + r0 + 4 * lk + qq;
        if (row >= Z) continue;
        const size_t idx = (size_t)row * X + col;
        if (VEC) {
            if (col < X) {
                float4 v = make_float4(alpha * acc[0][qq], alpha * acc[1][qq], alpha * acc[2][qq], alpha * acc[3][qq]);
                if (base_b) {
                    const float4 bv = *reinterpret_cast<const float4*>(base_b + idx);
                    v.x = fmaf(beta, bv.x, v.x);
                    v.y = fmaf(beta, bv.y, v.y);
                    v.z = fmaf(beta, bv.z, v.z);
                    v.w = fmaf(beta, bv.w, v.w);
                }
                *reinterpret_cast<float4*>(Ob + idx) = v;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (col + c < X) {
                    float v = alpha * acc[c][qq];
                    if (base_b) v = fmaf(beta, base_b[idx + c], v);
                    Ob[idx + c] = v;
                }
            }
        }
    }
}

template <bool ADJ, int PD, bool VEC>
__global__ __launch_bounds__(MF_THREADS) void tidas_mfma_kernel(const ConvGeom g, const float* __restrict__ Kb,
                                                                const float* __restrict__ In, float* Out) {
    extern __shared__ float smem[];
    const int lg = xcd_remap(blockIdx.x, g.n_blocks);
    const int rt_i = lg % g.n_rt;
    const int ct = (lg / g.n_rt) % g.n_ct;
    const int b = lg / (g.n_rt * g.n_ct);
    const size_t fo = (size_t)b * g.Z * g.X;
    mfma_tile<ADJ, PD, VEC>(Kb, In + fo, Out + fo, g.base ? g.base + fo : nullptr, g.alpha, g.beta, g.K, g.Z, g.X,
                            rt_i * MF_TZ, ct * MF_TN, smem);
}

// Ragged batch of the line model: one persistent launch over the 32 x 256
// tiles of all frames (each frame with its own grid, bank, input and output),
// the tile list cut into 8 contiguous chunks, chunk x served by the
// workgroups on XCD x.  Fixed strides: every workgroup's loop ends.
struct ConvFrameDev {  // at most 128 bytes (the workspace holds 128 bytes per frame)
    const float* kernels;
    const float* in;
    float* out;
    int32_t Z, X;
    int32_t vec;  // X % 4 == 0 and 16-byte aligned input and output
    int32_t pad;
    int64_t tile_start;
    int64_t img_off;  // four-block batch: byte offset of the frame's band images in the workspace
};

static_assert(sizeof(ConvFrameDev) <= 128, "batch table entry too large");

template <int PD>
__global__ __launch_bounds__(MF_THREADS) void tidas_batch_kernel(const ConvFrameDev* __restrict__ fr, int32_t n_frames,
                                                                 int64_t total, int32_t K) {
    extern __shared__ float smem[];
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per_xcd = ((int)gridDim.x - x + 7) >> 3;
    const int64_t lo = total * x / 8, hi = total * (x + 1) / 8;
    for (int64_t t = lo + slot; t < hi; t += per_xcd) {
        int a = 0, b = n_frames - 1;  // largest f with tile_start <= t
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (fr[mid].tile_start <= t) a = mid;
            else b = mid - 1;
        }
        const ConvFrameDev f = fr[a];
        const int64_t local = t - f.tile_start;
        const int row_tiles = (f.Z + MF_TZ - 1) / MF_TZ;
        const int i0 = (int)(local % row_tiles) * MF_TZ;
        const int j0 = (int)(local / row_tiles) * MF_TN;
        __syncthreads();  // the previous tile's readers of the LDS kernel tile are done
        if (f.vec)
            mfma_tile<false, PD, true>(f.kernels, f.in, f.out, nullptr, 1.0f, 0.0f, K, f.Z, f.X, i0, j0, smem);
        else
            mfma_tile<false, PD, false>(f.kernels, f.in, f.out, nullptr, 1.0f, 0.0f, K, f.Z, f.X, i0, j0, smem);
    }
}

// ------------------------------------------------------------------------
// Split-bfloat16 matrix-core path (preferred whenever its LDS tile fits).
// The same banded product on v_mfma_f32_32x32x16_bf16.  Every float32 operand
// v is cut exactly, by truncation, into three bfloat16 parts v = v0 + v1 + v2:
// v0 = the top 16 bits of v, v1 = the top 16 bits of r1 = v - v0 (exact: r1
// has at most 16 significant bits), v2 = r1 - v1 (at most 8 significant bits,
// so exactly a bfloat16).  A product a b is taken as the six terms
//   a0 b0 + a0 b1 + a1 b0 + a0 b2 + a1 b1 + a2 b0,
// each exact in float32, accumulated in float32; the dropped a1 b2 + a2 b1 +
// a2 b2 is below 2^-20 |a b| (|a1| < 2^-7 |a|, |a2| < 2^-14 |a|), so the sum
// carries float32-level error (the split-bfloat16 scheme of Henry, Tang and
// Heinecke, ARITH 2019).  Six products at the dense bf16 matrix rate are
// 2.6x the float32 matrix rate: the line model becomes bound by memory
// instead of the matrix cores.  Non-finite inputs give NaN.
//
// Tile: 64 output rows x 256 columns, 4 waves.  Wave w owns columns 64 w ..
// +63 as two chains (chain c of lane column j is image column 2 j + c, so an
// 8-byte load of two consecutive columns feeds both) and all 64 rows as two
// 32-row M-blocks: 4 accumulators of 32 x 32.  Operand layouts of the
// instruction: A lane l holds A[l % 32][8 (l / 32) .. +7], B lane l holds
// B[8 (l / 32) .. +7][l % 32], register i of D lane l holds
// D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].  The k dimension walks the
// tile's source window [i0 - h, i0 - h + 16 NS) in steps of 16 rows: per
// step lane (j, g) loads window rows 16 s + 8 g .. +7 at its two columns
// (eight coalesced 8-byte loads), splits them in registers, and M-block b
// runs the six products for the steps its band [32 b, 32 b + 31 + 2h] meets.
// The loads run BX_PD - 1 steps ahead through a register ring.  The tile's
// band matrix, M[r][c] = K[i0 + r][r - c + 2h] (adjoint: K[i0 - h + c][c - r];
// zero off the band and outside the bank), is split once into three bfloat16
// planes in LDS with a row stride of 8 (mod 16) bf16, so the 16-byte A reads
// of eight consecutive rows hit distinct banks, and it serves nf consecutive
// frames (same rows and columns); the ring runs on across frame boundaries.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int BX_TZ = 64;        // output rows per tile (two 32-row M-blocks)
constexpr int BX_TN = 256;       // columns per tile
constexpr int BX_THREADS = 256;  // 4 waves
constexpr int BX_PD = 4;         // register ring: the current step and three in flight

// k-steps per tile, rounded up to whole groups of BX_PD (the extra steps meet a
// zero band and cost matrix work only)
__host__ __device__ constexpr int bx_nsteps(int K) { return ((BX_TZ + K - 1 + 15) / 16 + 3) / 4 * 4; }
__host__ __device__ constexpr int bx_lstride(int K) { return 16 * bx_nsteps(K) + 8; }
__host__ __device__ constexpr size_t bx_lds_bytes(int K) { return (size_t)3 * BX_TZ * bx_lstride(K) * 2; }

// A wave-uniform pointer moved into scalar registers (a buffer descriptor
// built from a pointer the compiler cannot prove uniform costs a loop per load).
template <typename T>
__device__ __forceinline__ const T* uniform_ptr(const T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

// bfloat16 parts of the exact split, each as the top half of a 32-bit word
// (every operand of the line model, map and bank, passes here: a debug build
// flags non-finite ones)
__device__ __forceinline__ void split3(float v, uint32_t& w0, uint32_t& w1, uint32_t& w2) {
    TIDAS_DCHECK(__builtin_isfinite(v), TIDAS_DBG_NONFINITE_IN);
    const uint32_t u = __float_as_uint(v);
    const float r1 = v - __uint_as_float(u & 0xffff0000u);
    const uint32_t u1 = __float_as_uint(r1);
    const float r2 = r1 - __uint_as_float(u1 & 0xffff0000u);
    w0 = u;
    w1 = u1;
    w2 = __float_as_uint(r2);
}

// eight words -> eight bfloat16 (top halves), element e in half (e & 1) of word e / 2
__device__ __forceinline__ bf16x8 pack8(const uint32_t (&w)[8]) {
    u32x4 p;
#pragma unroll
    for (int d = 0; d < 4; ++d) p[d] = __builtin_amdgcn_perm(w[2 * d + 1], w[2 * d], 0x07060302u);  // one v_perm_b32
    return __builtin_bit_cast(bf16x8, p);
}

// The tile's band matrix in split form ("band image"): three planes of
// [64][LS] bfloat16, entry (r, c) = M[r][c] of the 64-row tile at i0, zero off
// the band, outside the bank and in the padding columns c >= 16 NS.
__host__ __device__ constexpr size_t bx_band_bytes(int K) { return bx_lds_bytes(K); }

template <bool ADJ>
__device__ __forceinline__ float bx_band_value(const float* __restrict__ Kb, int K, int Z, int i0, int r, int c) {
    const int h = (K - 1) >> 1;
    const int t = ADJ ? c - r : r - c + 2 * h;
    const int row = ADJ ? i0 - h + c : i0 + r;
    const bool ok = c < 16 * bx_nsteps(K) && t >= 0 && t < K && row >= 0 && row < Z;
    return ok ? Kb[(size_t)row * K + t] : 0.0f;
}

template <bool ADJ>
__device__ __forceinline__ void bx_band_put(uint16_t* img, int plane, int o, float v) {
    uint32_t w0, w1, w2;
    split3(v, w0, w1, w2);
    img[o] = (uint16_t)(w0 >> 16);
    img[plane + o] = (uint16_t)(w1 >> 16);
    img[2 * plane + o] = (uint16_t)(w2 >> 16);
}

// Band images of every 64-row tile of a bank, mode mode0 + blockIdx.z (0
// forward, 1 adjoint), tile rt at prepared + (blockIdx.z n_rt + rt) bx_band_bytes(K).
__global__ __launch_bounds__(256) void bx_prepare_kernel(const float* __restrict__ Kb, int32_t K, int32_t Z,
                                                         int32_t n_rt, uint16_t* __restrict__ prepared, int32_t mode0) {
    const int LS = bx_lstride(K);
    const int rt = blockIdx.y, adj = mode0 + (int)blockIdx.z;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= BX_TZ * LS) return;
    const int r = e / LS, c = e - (e / LS) * LS;
    uint16_t* img = prepared + (size_t)(blockIdx.z * n_rt + rt) * (bx_band_bytes(K) / 2);
    const float v = adj ? bx_band_value<true>(Kb, K, Z, rt * BX_TZ, r, c) : bx_band_value<false>(Kb, K, Z, rt * BX_TZ, r, c);
    bx_band_put<false>(img, BX_TZ * LS, e, v);
}

// Band image into LDS.  From a prepared image: a straight copy by
// direct-to-LDS 16-byte loads (every wave load moves 1 KB; the image is a
// whole number of them since LS = 0 (mod 8)).  From the bank: a rolled loop
// over the entries (the ragged batch path, whose frames each bring a bank).
// Neither (both null): the band already in LDS is kept (the next column tile
// of the same row tile).
template <bool ADJ>
__device__ __forceinline__ void bx_band_to_lds(const uint16_t* __restrict__ img, const float* __restrict__ Kb, int K,
                                               int Z, int i0, uint16_t* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (img) {
        const int n_loads = (int)(bx_band_bytes(K) / 1024);
        const auto rs = make_rsrc(img, (uint32_t)bx_band_bytes(K));
        for (int q = wave; q < n_loads; q += BX_THREADS / 64)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(lds + q * 512), 16,
                                                     q * 1024 + lane * 16, 0, 0, 0);
        __builtin_amdgcn_s_waitcnt(0);  // the copy is in LDS (also drains the input prefetch)
    } else if (Kb) {
        const int LS = bx_lstride(K);
        const int n = BX_TZ * LS;
        // entry e = r LS + c, (r, c) stepped without a division per entry
        // (dc < LS: at most one carry past the row end per step)
        const int dr = BX_THREADS / LS, dc = BX_THREADS - dr * LS;
        int r = threadIdx.x / LS, c = threadIdx.x - r * LS;
#pragma unroll 4
        for (int e = threadIdx.x; e < n; e += BX_THREADS) {
            bx_band_put<ADJ>(lds, n, e, bx_band_value<ADJ>(Kb, K, Z, i0, r, c));
            r += dr;
            c += dc;
            if (c >= LS) {
                c -= LS;
                ++r;
            }
        }
    }
}

// nf consecutive frames (stride Z X floats) of one 64 x 256 tile.  All threads
// of the workgroup call it (it contains barriers).  VEC: X % 4 == 0 and
// 16-byte aligned rows (one 8-byte load / store per lane and row); otherwise
// dword accesses.
template <bool ADJ, bool VEC>
__device__ __forceinline__ void bx_tile(const uint16_t* __restrict__ img, const float* __restrict__ Kb,
                                        const float* __restrict__ In, float* Out, const float* Base, int nf,
                                        float alpha, float beta, int K, int Z, int X, int i0, int j0, uint16_t* lds) {
    const int h = (K - 1) >> 1;
    const int NS = bx_nsteps(K);
    const int LS = bx_lstride(K);
    const int plane = BX_TZ * LS;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = lane & 31, g = lane >> 5;
    const int col = j0 + 64 * wave + 2 * j;
    const size_t fstride = (size_t)Z * X;
    const uint32_t frame_bytes = (uint32_t)(fstride * sizeof(float));
    const int row_bytes = X * 4;
    // byte offset of window row 8 g at this lane's columns; rows above the image
    // are negative (huge unsigned), rows below are past the end: both read 0
    const int off0 = ((i0 - h + 8 * g) * X + col) * 4;

    // buffer descriptor of frame f (frame 0 stands in past the last frame: its
    // loads are then pushed out of range)
    auto frame_rsrc = [&](int f) {
        const int fu = __builtin_amdgcn_readfirstlane(f < nf ? f : 0);  // wave-uniform: keep it scalar
        return make_rsrc(uniform_ptr(In + (size_t)fu * fstride), frame_bytes);
    };
    // rows of local step s through descriptor rs; !valid (past the last frame)
    // reads nothing: the offsets are pushed out of range, so the loads return 0
    // without traffic
    auto load8 = [&](__amdgpu_buffer_rsrc_t rs, int s, bool valid, floatx2(&x)[8]) {
        const int so = __builtin_amdgcn_readfirstlane(valid ? s * 16 * row_bytes : INT32_MIN - off0);
        const int o = off0 + so;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (VEC) {
                x[e] = __builtin_bit_cast(floatx2, __builtin_amdgcn_raw_buffer_load_b64(rs, o + e * row_bytes, 0, 0));
            } else {
                x[e][0] = buffer_load_f32(rs, o + e * row_bytes);
                x[e][1] = buffer_load_f32(rs, o + e * row_bytes + 4);
            }
        }
    };

    floatx2 ring[BX_PD][8];
    // Walk order: window steps ascending for output rows in even 128-row bands
    // (i0 / 128 even), descending in odd ones.  Every line-model kernel sums a
    // row's 16-row chunks in this order (the products outside a row's band are
    // exact zeros), so all of them give the same bits; and a tile whose walk
    // is mirrored against its neighbour's reads their shared rows at the same
    // time, so the second read hits L2.
    const bool rev = ((i0 / 128) & 1) != 0;
    auto local_step = [&](int q) { return rev ? NS - 1 - q : q; };
    // first steps' input loads in flight while the band image is brought in
    {
        const auto rs0 = frame_rsrc(0);
#pragma unroll
        for (int u = 0; u < BX_PD - 1; ++u) load8(rs0, local_step(u), true, ring[u]);
    }
    bx_band_to_lds<ADJ>(img, Kb, K, Z, i0, lds);
    __syncthreads();

    floatx16 acc[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[b][c][i] = 0.0f;

    const uint16_t* a_base = lds + j * LS + 8 * g;
    constexpr int TA[6] = {0, 0, 1, 0, 1, 2};
    constexpr int TB[6] = {0, 1, 0, 2, 1, 0};

    // Results of frame f.  Every store and base load is issued (rows past Z and
    // columns past X get an out-of-range offset, which the buffer unit drops or
    // reads as 0): conditional memory operations would make the wait counts
    // after the epilogue drain the whole prefetch ring.
    const int vbase = ((i0 + 4 * g) * X + col) * 4;
    constexpr int OOB = INT32_MIN;
    auto store_frame = [&](int f) {
        const auto rs_o = make_rsrc(uniform_ptr(Out + (size_t)f * fstride), frame_bytes);
        const bool has_base = Base != nullptr;
        const auto rs_b = make_rsrc(uniform_ptr((has_base ? Base : Out) + (size_t)f * fstride), frame_bytes);
        // lane offset of row rr of the tile, chain c (OOB when outside the image);
        // VEC accesses both chains at the chain-0 offset (X % 4 == 0 and col is
        // even, so col < X implies col + 1 < X)
        auto voff = [&](int rr, int c) {
            const bool ok = i0 + 4 * g + rr < Z && col + c < X;
            return ok ? vbase + rr * row_bytes + 4 * c : OOB;
        };
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            floatx2 v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = floatx2{alpha * acc[b][0][i], alpha * acc[b][1][i]};
            if (has_base) {  // all base loads of the M-block first, then the updates
                floatx2 bv[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int rr = 32 * b + 8 * (i >> 2) + (i & 3);
                    if (VEC) {
                        bv[i] = __builtin_bit_cast(floatx2, __builtin_amdgcn_raw_buffer_load_b64(rs_b, voff(rr, 0), 0, 0));
                    } else {
                        bv[i][0] = buffer_load_f32(rs_b, voff(rr, 0));
                        bv[i][1] = buffer_load_f32(rs_b, voff(rr, 1));
                    }
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    v[i][0] = fmaf(beta, bv[i][0], v[i][0]);
                    v[i][1] = fmaf(beta, bv[i][1], v[i][1]);
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int rr = 32 * b + 8 * (i >> 2) + (i & 3);
                if (VEC) {
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v[i]), rs_o, voff(rr, 0), 0, 0);
                } else {
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[i][0]), rs_o, voff(rr, 0), 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[i][1]), rs_o, voff(rr, 1), 0, 0);
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[b][c][i] = 0.0f;
        }
    };

    // position q of frame f on ring slot U = q % BX_PD; first refill slot
    // (U + BX_PD - 1) % BX_PD (consumed by the previous step) BX_PD - 1 positions ahead
    // split operand of one ring slot (both chains)
    auto split_slot = [&](const floatx2(&x)[8], bf16x8(&Bp)[2][3]) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            uint32_t w0[8], w1[8], w2[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) split3(x[e][c], w0[e], w1[e], w2[e]);
            Bp[c][0] = pack8(w0);
            Bp[c][1] = pack8(w1);
            Bp[c][2] = pack8(w2);
        }
    };
    // software pipeline: the matrix products of a step use the split operand
    // made during the previous step, while this step splits the next slot's
    // rows, so the products never wait on the conversion
    bf16x8 BpA[2][3], BpB[2][3];
    split_slot(ring[0], BpA);

    // Position q + U of the current frame; its prefetch targets position
    // q + U + BX_PD - 1, which lies in the next frame (at q + U + BX_PD - 1 - NS)
    // when WRAP (the frame's last group of four) and U > 0.  The wrap is known
    // at compile time, so a step is one basic block.
    auto step = [&](auto U_, auto WRAP_, int q, __amdgpu_buffer_rsrc_t rs_cur, __amdgpu_buffer_rsrc_t rs_nxt,
                    bool nxt_valid) {
        constexpr int U = decltype(U_)::value;
        constexpr bool WRAP = decltype(WRAP_)::value && U > 0;
        bf16x8(&Bcur)[2][3] = (U % 2 == 0) ? BpA : BpB;
        bf16x8(&Bnxt)[2][3] = (U % 2 == 0) ? BpB : BpA;
        if (WRAP)
            load8(rs_nxt, local_step(q + U + BX_PD - 1 - NS), nxt_valid, ring[(U + BX_PD - 1) % BX_PD]);
        else
            load8(rs_cur, local_step(q + U + BX_PD - 1), true, ring[(U + BX_PD - 1) % BX_PD]);
        const int s = local_step(q + U);
        // keep the prefetch at the top of the step: the scheduler would sink the
        // loads below the matrix instructions to shorten their live ranges
        __builtin_amdgcn_sched_barrier(0);
        // both M-blocks on every step: outside a block's band its A is zero, and
        // straight-line code keeps the accumulators in place (no joins)
        bf16x8 A[2][3];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int p = 0; p < 3; ++p)
                A[b][p] = *reinterpret_cast<const bf16x8*>(a_base + p * plane + 32 * b * LS + 16 * s);
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[b][TA[t]], Bcur[c][TB[t]], acc[b][c], 0, 0, 0);
        split_slot(ring[(U + 1) % BX_PD], Bnxt);
        // issue order: each matrix product followed by four vector instructions
        // of the next slot's split.  Instructions issue in order per wave, so a
        // burst of 24 products would hold the split back until the matrix unit
        // had accepted them all; interleaved, the split runs under the products.
#pragma unroll
        for (int i = 0; i < 24; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // four VALU
        }
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    static_assert(BX_PD == 4, "the unrolled ring below has four slots");
    // NS is a multiple of four: each frame is whole groups of four straight-line
    // steps (fixed ring slots), and the epilogue sits outside the group loop, so
    // the wait counts before each step leave the younger steps' loads in flight
    using NoWrap = std::false_type;
    using Wrap = std::true_type;
    for (int f = 0; f < nf; ++f) {
        const auto rs_cur = frame_rsrc(f), rs_nxt = frame_rsrc(f + 1);
        const bool nxt_valid = f + 1 < nf;
        int q = 0;
        for (; q < NS - BX_PD; q += BX_PD) {
            step(I0{}, NoWrap{}, q, rs_cur, rs_nxt, nxt_valid);
            step(I1{}, NoWrap{}, q, rs_cur, rs_nxt, nxt_valid);
            step(I2{}, NoWrap{}, q, rs_cur, rs_nxt, nxt_valid);
            step(I3{}, NoWrap{}, q, rs_cur, rs_nxt, nxt_valid);
        }
        step(I0{}, Wrap{}, q, rs_cur, rs_nxt, nxt_valid);
        step(I1{}, Wrap{}, q, rs_cur, rs_nxt, nxt_valid);
        step(I2{}, Wrap{}, q, rs_cur, rs_nxt, nxt_valid);
        step(I3{}, Wrap{}, q, rs_cur, rs_nxt, nxt_valid);
        store_frame(f);
    }
}

// ------------------------------------------------------------------------
// Four-M-block variant for K <= 161 and batches that fill the GPU.
// A workgroup (8 waves) owns 128 output rows x 256 columns; wave w owns
// columns 32 w .. +31 (one chain: lane column j is image column j) and all
// 128 rows as four 32-row M-blocks, so every split input element feeds up to
// four M-blocks x six products (twice the two-block tile's reuse: half the
// split work per product), and the source window per output row is (128 +
// K - 1) / 128 instead of (64 + K - 1) / 64.  M-block b needs window steps
// [2 b, 2 b + NSB) only; LDS holds each block's own band window (three planes
// of 32 x (16 NSB + 8) bfloat16), and the walk over the NSB + 6 steps of a
// frame is unrolled at compile time (NSB is a template parameter), so every
// step issues exactly the products of the blocks its rows reach, with no
// branches.  The 16-row chunks and their order are those of the two-block
// tile: the results are bit-identical.
constexpr int B4_TZ = 128;
constexpr int B4_TN = 256;
constexpr int B4_THREADS = 512;  // 8 waves

__host__ __device__ constexpr int b4_lstride(int nsb) { return 16 * nsb + 8; }
// one block's three planes, padded to a multiple of 8 KB: each of the eight
// waves copies the same number of 1 KB pieces of every block
__host__ __device__ constexpr int b4_block_bytes(int nsb) { return (3 * 32 * b4_lstride(nsb) * 2 + 8191) / 8192 * 8192; }
__host__ __device__ constexpr size_t b4_image_bytes(int nsb) { return (size_t)4 * b4_block_bytes(nsb); }
// smallest supported NSB covering K (0: K too large for the four-block tile)
__host__ __device__ constexpr int b4_nsb(int K) {
    const int need = (32 + K - 1 + 15) / 16;
    return need <= 4 ? 4 : need <= 6 ? 6 : need <= 8 ? 8 : need <= 10 ? 10 : need <= 12 ? 12 : 0;
}

// Band image of the 128-row tile at i0 in the four-block layout
// [block (stride b4_block_bytes)][plane][32][16 NSB + 8]: entry (b, r, c) = M[32 b + r][32 b + c] of
// the tile (apply: K[i0 + 32b + r][r - c + 2h]; adjoint: K[i0 - h + 32b + c][c - r]).
// Entry e (over [block][row][column]) of the band image of 128-row tile rt,
// written to the tile's image img (three planes per block).
__device__ __forceinline__ void b4_prepare_entry(const float* __restrict__ Kb, int32_t K, int32_t Z, int32_t nsb,
                                                 int rt, int adj, int e, uint16_t* __restrict__ img) {
    const int LS = b4_lstride(nsb);
    const int per_block = 32 * LS;
    if (e >= 4 * per_block) return;
    const int b = e / per_block, rc = e - b * per_block;
    const int r = rc / LS, c = rc - r * LS;
    const int h = (K - 1) >> 1;
    const int i0 = rt * B4_TZ;
    const int t = adj ? c - r : r - c + 2 * h;
    const int row = adj ? i0 - h + 32 * b + c : i0 + 32 * b + r;
    const bool ok = c < 16 * nsb && t >= 0 && t < K && row >= 0 && row < Z;
    const float v = ok ? Kb[(size_t)row * K + t] : 0.0f;
    uint16_t* blk = img + (size_t)b * (b4_block_bytes(nsb) / 2);
    uint32_t w0, w1, w2;
    split3(v, w0, w1, w2);
    blk[rc] = (uint16_t)(w0 >> 16);
    blk[per_block + rc] = (uint16_t)(w1 >> 16);
    blk[2 * per_block + rc] = (uint16_t)(w2 >> 16);
}

__global__ __launch_bounds__(256) void b4_prepare_kernel(const float* __restrict__ Kb, int32_t K, int32_t Z,
                                                         int32_t n_rt, int32_t nsb, uint16_t* __restrict__ prepared,
                                                         int32_t mode0) {
    const int rt = blockIdx.y, adj = mode0 + (int)blockIdx.z;
    uint16_t* img = prepared + (size_t)(blockIdx.z * n_rt + rt) * (b4_image_bytes(nsb) / 2);
    b4_prepare_entry(Kb, K, Z, nsb, rt, adj, blockIdx.x * 256 + threadIdx.x, img);
}

// Forward band images of every 128-row tile of every frame of a ragged batch
// (grid.y = global tile index; frame f's images at byte offset img_off).
__global__ __launch_bounds__(256) void b4_batch_prepare_kernel(const ConvFrameDev* __restrict__ tab, int32_t n_tab,
                                                               int32_t K, int32_t nsb, uint16_t* __restrict__ images) {
    const int t = blockIdx.y;
    int a = 0, b = n_tab - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (tab[mid].tile_start <= t) a = mid;
        else b = mid - 1;
    }
    const ConvFrameDev fr = tab[a];
    const int rt = t - (int)fr.tile_start;
    uint16_t* img = images + fr.img_off / 2 + (size_t)rt * (b4_image_bytes(nsb) / 2);
    b4_prepare_entry(fr.kernels, K, fr.Z, nsb, rt, 0, blockIdx.x * 256 + threadIdx.x, img);
}

template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<0>), ..., f(integral_constant<N - 1>) in order, unrolled
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// Results are stored non-temporally (the cache-policy bit nt): the output is
// not read again by the launch, and keeping it out of L2 leaves the L2 to the
// input rows that neighbouring row tiles read twice.  Measured: 32.1-33.5 ->
// 30.7-30.9 us on the benchmark's 64 frames of 1024 x 256, 137-164 -> 125-130
// us on 64 frames of 2048 x 512 (whose frames outgrow an XCD's L2).
constexpr int B4_STORE_NT = 2;

struct B4Geom {
    int32_t K, B, Z, X, nf;
    int32_t n_rt, n_ct, n_blocks;
    float alpha, beta;
    const float* base;
};

// BATCH: a ragged batch (tidas_apply_batch).  Workgroup lg takes 128-row
// tile rt of the frame whose tile range holds lg (table `tab`, tile_start in
// 128-row tiles), with that frame's prepared band image at byte offset
// img_off from `images`; the frame's 256-column tiles take the place of the
// frames of a plain launch (the ring runs on from one to the next), each
// addressed from a base 256 columns further on, so rows past the image still
// fall outside the range and read 0; columns past X are computed but not stored.
// PLAIN: alpha = 1 and no base, the results stored as accumulated (the
// epilogue's base values then hold no registers).
template <bool ADJ, int NSB, bool BATCH, bool PLAIN>
__global__ __launch_bounds__(B4_THREADS) void tidas_b4_kernel(const B4Geom g, const uint16_t* __restrict__ images,
                                                              const float* __restrict__ In, float* Out,
                                                              const ConvFrameDev* __restrict__ tab, int32_t n_tab) {
    constexpr int NW = NSB + 6;   // window steps of the tile
    constexpr int LS = b4_lstride(NSB);
    constexpr int PB = 32 * LS;   // one plane of one block, in bf16
    // ring slots: window step s of every frame lives in slot s % PD, and the
    // loads that run ahead into the next frame land in slot (NW + s) % PD, so
    // PD must divide NW
    constexpr int PD = NW % 4 == 0 ? 4 : NW % 5 == 0 ? 5 : NW % 6 == 0 ? 6 : 7;
    static_assert(NW % PD == 0, "ring slots must divide the window steps");
    extern __shared__ uint16_t b4_smem[];
    const int lg = xcd_remap(blockIdx.x, g.n_blocks);
    int rt, ct, nf, Z, X;
    const float* In0;
    float* Out0;
    const float* Base0;
    const uint16_t* img_tiles;  // band image of tile 0 of this workgroup's frame
    size_t fstride;             // floats from one frame (batch: column tile) to the next
    if constexpr (BATCH) {
        int a = 0, b = n_tab - 1;  // largest frame with tile_start <= lg
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (tab[mid].tile_start <= lg) a = mid;
            else b = mid - 1;
        }
        const ConvFrameDev fr = tab[__builtin_amdgcn_readfirstlane(a)];
        Z = __builtin_amdgcn_readfirstlane(fr.Z);
        X = __builtin_amdgcn_readfirstlane(fr.X);
        rt = lg - __builtin_amdgcn_readfirstlane((int)fr.tile_start);
        ct = 0;
        nf = (X + B4_TN - 1) / B4_TN;
        In0 = uniform_ptr(fr.in);
        Out0 = const_cast<float*>(uniform_ptr(fr.out));
        Base0 = nullptr;
        img_tiles = uniform_ptr(images + fr.img_off / 2);
        fstride = B4_TN;
    } else {
        rt = lg % g.n_rt;
        ct = (lg / g.n_rt) % g.n_ct;
        const int fg = lg / (g.n_rt * g.n_ct);
        const int f0 = fg * g.nf;
        nf = min(g.nf, g.B - f0);
        Z = g.Z;
        X = g.X;
        fstride = (size_t)Z * X;
        In0 = In + (size_t)f0 * fstride;
        Out0 = Out + (size_t)f0 * fstride;
        Base0 = g.base ? g.base + (size_t)f0 * fstride : nullptr;
        img_tiles = images;
    }
    const int K = g.K;
    const int h = (K - 1) >> 1;
    const int i0 = rt * B4_TZ;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = lane & 31, gk = lane >> 5;
    const int col = ct * B4_TN + 32 * wave + j;
    // bytes addressable from frame (column tile) f's base: up to the image's end
    auto frame_bytes = [&](int f) {
        return (uint32_t)(((size_t)Z * X - (BATCH ? (size_t)f * B4_TN : 0)) * sizeof(float));
    };
    const int row_bytes = X * 4;
    // byte offset of window row 8 gk of step 0 at this lane's column; rows
    // above or below the image fall outside the frame and read 0
    const int off0 = ((i0 - h + 8 * gk) * X + col) * 4;

    auto frame_rsrc = [&](int f) {
        const int fu = __builtin_amdgcn_readfirstlane(f < nf ? f : 0);
        return make_rsrc(uniform_ptr(In0 + (size_t)fu * fstride), frame_bytes(fu));
    };
    // rows of window step s of frame (batch: column tile) f; in a batch, lanes
    // whose column lies past X in that column tile read nothing (their offset
    // leaves the range), so the ragged edge costs no traffic
    auto load8 = [&](__amdgpu_buffer_rsrc_t rs, int s, bool valid, float(&x)[8], int f) {
        const int so = __builtin_amdgcn_readfirstlane(valid ? s * 16 * row_bytes : INT32_MIN - off0);
        int o = off0 + so;
        if constexpr (BATCH) o = f * B4_TN + col < X ? o : INT32_MIN;
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = buffer_load_f32(rs, o + e * row_bytes);
    };

    // The walk over the window.  Even row tiles take the window steps in
    // ascending order, odd row tiles in descending order (the order of the
    // two-block tile for the same rows, so both give the same bits): the 128 rows that
    // neighbouring tiles share are then read by both in the same half of the
    // frame (the second half of the upper tile's walk is the first half of the
    // lower tile's reversed walk, and so on down), so the second read of a row
    // is served by the L2 instead of HBM.  Iteration I takes window step
    // S = I (ascending) or NW - 1 - I (descending).  In either order the k-th
    // block to start (block k ascending, 3 - k descending) is active from
    // iteration 2 k to NSB - 1 + 2 k.
    auto run_tile = [&](auto REV_) {
        constexpr bool REV = decltype(REV_)::value;
        auto step_of = [](int it) { return REV ? NW - 1 - it : it; };
        auto block_of = [](int k) { return REV ? 3 - k : k; };

        // Band image: a straight copy by direct-to-LDS 16-byte loads, 1 KB per
        // wave load, block by block in the order the walk needs them; each wave
        // copies L pieces of every block.  The k-th block is first used at
        // iteration 2 k, so in the first frame each wave waits (vmcnt) for its
        // own pieces of that block just before that iteration and the workgroup
        // meets at a barrier; the copy of the later blocks overlaps the first
        // iterations.  The first iterations' input loads are issued before the copy.
        constexpr int BSE = b4_block_bytes(NSB) / 2;  // block stride in bf16
        constexpr int L = b4_block_bytes(NSB) / 8192;
        float ring[PD][8];
        {
            const auto rs0 = frame_rsrc(0);
            const uint16_t* img = img_tiles + (size_t)rt * (b4_image_bytes(NSB) / 2);
            const auto rs = make_rsrc(img, (uint32_t)b4_image_bytes(NSB));
            auto copy_block = [&](int k) {
#pragma unroll
                for (int u = 0; u < L; ++u) {
                    const int piece = block_of(k) * 8 * L + 8 * u + wave;
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void*)(b4_smem + piece * 512), 16,
                        piece * 1024 + lane * 16, 0, 0, 0);
                }
            };
            // what the first iteration needs goes first: its input rows and
            // the first block, then the other prefetched rows and blocks
            load8(rs0, step_of(0), true, ring[0], 0);
            copy_block(0);
#pragma unroll
            for (int u = 1; u < PD - 1; ++u) load8(rs0, step_of(u), true, ring[u], 0);
#pragma unroll
            for (int k = 1; k < 4; ++k) copy_block(k);
        }
        // at iteration 2 k of the first frame: this wave's pieces of the k-th
        // block have landed once at most n vector-memory operations issued after
        // them are outstanding (the pieces of the later blocks, the input loads
        // of iterations 1 .. PD - 2 for the first block, those issued by
        // iterations 0 .. 2 k - 1; later stores and loads only make the wait longer)
        auto band_ready = [&](auto K_) {
            constexpr int k = decltype(K_)::value;
            constexpr int n = (3 - k) * L + (k == 0 ? 8 * (PD - 2) : 8 * 2 * k);
            static_assert(n <= 63, "vmcnt range");
            __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00);
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");  // no band read is moved above the barrier
        };

        floatx16 acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[b][i] = 0.0f;

        auto split8 = [&](const float(&x)[8], bf16x8(&Bp)[3]) {
            uint32_t w0[8], w1[8], w2[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) split3(x[e], w0[e], w1[e], w2[e]);
            Bp[0] = pack8(w0);
            Bp[1] = pack8(w1);
            Bp[2] = pack8(w2);
        };
        bf16x8 BpA[3], BpB[3];
        split8(ring[0], BpA);

        const uint16_t* a_base = b4_smem + j * LS + 8 * gk;
        constexpr int TA[6] = {0, 0, 1, 0, 1, 2};
        constexpr int TB[6] = {0, 1, 0, 2, 1, 0};
        // Results.  The k-th block's last iteration is NSB - 1 + 2 k; its 16
        // results per lane are stored at the next iteration (k = 0..2 within
        // the frame, k = 3 at iteration 0 of the next frame or after the last),
        // so the stores spread over the frame instead of waiting at its end.
        // D row 8 (i / 4) + 4 gk + i % 4 of block b is tile row 32 b + that.
        // Every store is issued: rows below the image lie past the frame's last
        // byte and columns past X start at INT32_MIN, so the range check drops both.
        const int vbase = ((i0 + 4 * gk) * X + col) * 4;
        const int vstart = col < X ? vbase : INT32_MIN;
        constexpr bool plain = PLAIN;
        const bool has_base = !PLAIN && Base0 != nullptr;
        // base values of the block to be stored two iterations on (two buffers:
        // consecutive blocks are stored two iterations apart)
        float bv[2][16];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int i = 0; i < 16; ++i) bv[u][i] = 0.0f;
        // offset of block b's first result row; rebuilt from opaque values at
        // each use, else the compiler hoists all 64 offsets out of the frame loop
        auto block_offsets = [&](int b, int f, int(&voff)[16]) {
            int o = BATCH ? (f * B4_TN + col < X ? vbase : INT32_MIN) : vstart, rb = row_bytes;
            asm volatile("" : "+v"(o), "+s"(rb));
            o += 32 * b * rb;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                voff[i] = o;
                o += (i & 3) == 3 ? 5 * rb : rb;
            }
        };
        auto frame_out = [&](int f, const float* P) {
            // frames before the first or past the last: no record, every access dropped
            const int fu = __builtin_amdgcn_readfirstlane(f >= 0 && f < nf ? f : 0);
            return make_rsrc(uniform_ptr(P + (size_t)fu * fstride), f >= 0 && f < nf ? frame_bytes(fu) : 0u);
        };
        auto load_base = [&](int b, int f, float(&dst)[16]) {
            if (has_base) {
                const auto rs_b = frame_out(f, Base0);
                int voff[16];
                block_offsets(b, f, voff);
#pragma unroll
                for (int i = 0; i < 16; ++i) dst[i] = buffer_load_f32(rs_b, voff[i]);
            }
        };
        auto store_block = [&](int b, int f, floatx16& a, const float(&bsrc)[16]) {
            const auto rs_o = frame_out(f, Out0);
            int voff[16];
            block_offsets(b, f, voff);
            if (plain) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(a[i]), rs_o, voff[i], 0, B4_STORE_NT);
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const float v = fmaf(g.beta, bsrc[i], g.alpha * a[i]);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs_o, voff[i], 0, B4_STORE_NT);
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) a[i] = 0.0f;
        };

        for (int f = 0; f < nf; ++f) {
            const auto rs_cur = frame_rsrc(f), rs_nxt = frame_rsrc(f + 1);
            const bool nxt_valid = f + 1 < nf;
            static_for<NW>([&](auto I_) {
                constexpr int I = decltype(I_)::value;
                constexpr int S = REV ? NW - 1 - I : I;
                bf16x8(&Bcur)[3] = (I % 2 == 0) ? BpA : BpB;
                bf16x8(&Bnxt)[3] = (I % 2 == 0) ? BpB : BpA;
                if constexpr (I % 2 == 0 && I <= 6)
                    if (f == 0) band_ready(std::integral_constant<int, I / 2>{});
                // prefetch the iteration PD - 1 ahead (of this frame or the next)
                if constexpr (I + PD - 1 < NW)
                    load8(rs_cur, step_of(I + PD - 1), true, ring[(I + PD - 1) % PD], f);
                else
                    load8(rs_nxt, step_of(I + PD - 1 - NW), nxt_valid, ring[(I + PD - 1) % PD], f + 1);
                // the last block of the previous frame (none before the first)
                if constexpr (I == 0) store_block(block_of(3), f - 1, acc[block_of(3)], bv[1]);
                // the k-th block of this frame, its last iteration just done
                if constexpr (I >= NSB && I <= NSB + 4 && (I - NSB) % 2 == 0) {
                    constexpr int k = (I - NSB) / 2;
                    store_block(block_of(k), f, acc[block_of(k)], bv[k % 2]);
                }
                // base values for the store two iterations on
                if constexpr (I + 2 >= NSB && I + 2 <= NSB + 6 && (I + 2 - NSB) % 2 == 0) {
                    constexpr int k = (I + 2 - NSB) / 2;
                    load_base(block_of(k), f, bv[k % 2]);
                }
                __builtin_amdgcn_sched_barrier(0);
                // blocks whose band reaches window step S: b with 2 b <= S < 2 b + NSB
                constexpr int b_lo = (S >= NSB) ? (S - NSB) / 2 + 1 : 0;
                constexpr int b_hi = (S / 2 < 3) ? S / 2 : 3;
                // band operands of the step, plane-major: the first products
                // (plane 0 of every block) wait for the first reads only
                bf16x8 A[4][3];
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    static_for<4>([&](auto B_) {
                        constexpr int b = decltype(B_)::value;
                        if constexpr (b >= b_lo && b <= b_hi)
                            A[b][p] = *reinterpret_cast<const bf16x8*>(a_base + b * BSE + p * PB + 16 * (S - 2 * b));
                    });
#pragma unroll
                for (int t = 0; t < 6; ++t)
                    static_for<4>([&](auto B_) {
                        constexpr int b = decltype(B_)::value;
                        if constexpr (b >= b_lo && b <= b_hi)
                            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[b][TA[t]], Bcur[TB[t]], acc[b], 0, 0, 0);
                    });
                split8(ring[(I + 1) % PD], Bnxt);
                constexpr int n_mfma = 6 * (b_hi - b_lo + 1);
                constexpr int per = (48 + n_mfma - 1) / n_mfma;
                __builtin_amdgcn_sched_group_barrier(0x100, 3 * (b_hi - b_lo + 1), 0);  // the band reads first
                static_for<n_mfma>([&](auto) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, per, 0);  // vector instructions of the next split
                });
            });
        }
        store_block(block_of(3), nf - 1, acc[block_of(3)], bv[1]);
    };
    if (rt & 1) run_tile(std::true_type{});
    else run_tile(std::false_type{});
}

struct BxGeom {
    int32_t K, B, Z, X, nf;
    int32_t n_rt, n_ct, n_blocks;
    float alpha, beta;
    const float* base;
};

template <bool ADJ, bool VEC>
__global__ __launch_bounds__(BX_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void tidas_bx6_kernel(
    const BxGeom g, const uint16_t* __restrict__ images, const float* __restrict__ In, float* Out) {
    extern __shared__ uint16_t bx_smem[];
    const int lg = xcd_remap(blockIdx.x, g.n_blocks);
    const int rt = lg % g.n_rt;
    const int ct = (lg / g.n_rt) % g.n_ct;
    const int fg = lg / (g.n_rt * g.n_ct);
    const int f0 = fg * g.nf;
    const int nf = min(g.nf, g.B - f0);
    const size_t fo = (size_t)f0 * g.Z * g.X;
    const uint16_t* img = images + (size_t)rt * (bx_band_bytes(g.K) / 2);
    bx_tile<ADJ, VEC>(img, nullptr, In + fo, Out + fo, g.base ? g.base + fo : nullptr, nf, g.alpha, g.beta, g.K, g.Z,
                      g.X, rt * BX_TZ, ct * BX_TN, bx_smem);
}

// Ragged batch on the split-bfloat16 tile: as tidas_batch_kernel, over the
// 64-row tiles of all frames.  A visit takes one row tile of one frame: its
// band is filled from the frame's bank once and serves every 256-column tile
// of that row.  The tile is inlined into the visit loop; K goes through an
// opaque copy made per visit, else the loop-invariant parts of the band fill
// are hoisted out of the loop and hold registers through the whole tile.
// (Kept out of line instead, the call saved and restored ~100 callee-saved
// registers through scratch on every visit and built every buffer
// descriptor from pointer arguments in vector registers.)
__global__ __launch_bounds__(BX_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void tidas_bx6_batch_kernel(
    const ConvFrameDev* __restrict__ fr, int32_t n_frames, int64_t total, int32_t K) {
    extern __shared__ uint16_t bx_smem[];
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per_xcd = ((int)gridDim.x - x + 7) >> 3;
    const int64_t lo = total * x / 8, hi = total * (x + 1) / 8;
    for (int64_t t = lo + slot; t < hi; t += per_xcd) {
        int a = 0, b = n_frames - 1;  // largest f with tile_start <= t
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (fr[mid].tile_start <= t) a = mid;
            else b = mid - 1;
        }
        // the table entry is wave-uniform: move it to scalar registers, or every
        // buffer descriptor built from it becomes a per-lane loop
        const ConvFrameDev f = fr[__builtin_amdgcn_readfirstlane(a)];
        const int Zf = __builtin_amdgcn_readfirstlane(f.Z), Xf = __builtin_amdgcn_readfirstlane(f.X);
        const bool vec = __builtin_amdgcn_readfirstlane(f.vec) != 0;
        const int i0 = __builtin_amdgcn_readfirstlane((int)(t - f.tile_start) * BX_TZ);
        const float* kb = uniform_ptr(f.kernels);
        const float* in = uniform_ptr(f.in);
        float* out = const_cast<float*>(uniform_ptr(f.out));
        int Kv = K;
        asm volatile("" : "+s"(Kv));
        __syncthreads();  // the previous visit's readers of the LDS band are done
        for (int j0 = 0; j0 < Xf; j0 += BX_TN) {
            const float* fill = j0 == 0 ? kb : nullptr;  // one fill per row tile
            if (vec) bx_tile<false, true>(nullptr, fill, in, out, nullptr, 1, 1.0f, 0.0f, Kv, Zf, Xf, i0, j0, bx_smem);
            else bx_tile<false, false>(nullptr, fill, in, out, nullptr, 1, 1.0f, 0.0f, Kv, Zf, Xf, i0, j0, bx_smem);
        }
    }
}

// The split-bfloat16 tile fits: its LDS band, and every int32 byte offset of
// the source window (at most K + 160 rows beyond the image) below 2^31.
static bool bx_fits(int K, int Z, int X) {
    return bx_lds_bytes(K) <= 160 * 1024 && ((int64_t)Z + 2 * K + 256) * X * 4 < INT32_MAX;
}

static int device_cu_count() {
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
    }
    return n_cu;
}

// Band images of the bank's tiles for modes mode0 .. mode0 + n_modes - 1 (0
// forward, 1 adjoint): out holds [n_modes][tile][band image].
static void launch_prepare(const float* kernels, int32_t K, int32_t Z, int mode0, int n_modes, uint16_t* out,
                           hipStream_t stream) {
    const int n_rt = (Z + BX_TZ - 1) / BX_TZ;
    const int per_tile = BX_TZ * bx_lstride(K);
    const dim3 grid((unsigned)((per_tile + 255) / 256), (unsigned)n_rt, (unsigned)n_modes);
    hipLaunchKernelGGL(bx_prepare_kernel, grid, dim3(256), 0, stream, kernels, K, Z, n_rt, out, mode0);
}

static size_t prepared_bytes(int32_t K, int32_t Z, int n_modes) {
    return (size_t)n_modes * ((Z + BX_TZ - 1) / BX_TZ) * bx_band_bytes(K);
}

// images: the band images of the operator's mode (forward or adjoint), tile
// rt at images + rt bx_band_bytes(K) / 2
static void launch_bx6(bool adj, bool vec, const uint16_t* images, int32_t K, const float* in, int32_t B, int32_t Z,
                       int32_t X, float alpha, float beta, const float* base, float* out, hipStream_t stream) {
    BxGeom g;
    g.K = K;
    g.B = B;
    g.Z = Z;
    g.X = X;
    g.n_rt = (Z + BX_TZ - 1) / BX_TZ;
    g.n_ct = (X + BX_TN - 1) / BX_TN;
    // frames per workgroup: about two workgroups per compute unit in one
    // round; each reuses its band for its frames
    const int64_t tiles = (int64_t)g.n_rt * g.n_ct;
    const int64_t per_round = 2 * (int64_t)device_cu_count();
    g.nf = (int32_t)std::max<int64_t>(1, std::min<int64_t>(B, tiles * B / per_round));
    g.n_blocks = (int32_t)(tiles * ((B + g.nf - 1) / g.nf));
    g.alpha = alpha;
    g.beta = beta;
    g.base = base;
    const size_t lds = bx_lds_bytes(K);
    const dim3 grid(g.n_blocks), block(BX_THREADS);
    if (adj) {
        if (vec) hipLaunchKernelGGL((tidas_bx6_kernel<true, true>), grid, block, lds, stream, g, images, in, out);
        else hipLaunchKernelGGL((tidas_bx6_kernel<true, false>), grid, block, lds, stream, g, images, in, out);
    } else {
        if (vec) hipLaunchKernelGGL((tidas_bx6_kernel<false, true>), grid, block, lds, stream, g, images, in, out);
        else hipLaunchKernelGGL((tidas_bx6_kernel<false, false>), grid, block, lds, stream, g, images, in, out);
    }
}

// ---- four-M-block tiles
static bool b4_image_ok(int K) {
    const int nsb = b4_nsb(K);
    return nsb > 0 && b4_image_bytes(nsb) <= 160 * 1024;
}
static bool b4_fits(int K, int Z, int X) {
    return b4_image_ok(K) && ((int64_t)Z + 2 * K + 512) * X * 4 < INT32_MAX;
}
// worth it when the batch alone fills every compute unit
static bool b4_path(int32_t K, int32_t B, int32_t Z, int32_t X) {
    const int64_t tiles = (int64_t)((Z + B4_TZ - 1) / B4_TZ) * ((X + B4_TN - 1) / B4_TN) * B;
    return b4_fits(K, Z, X) && tiles >= device_cu_count() && tiles <= INT32_MAX;
}
static size_t b4_bytes(int32_t K, int32_t Z, int n_modes) {
    return (size_t)n_modes * ((Z + B4_TZ - 1) / B4_TZ) * b4_image_bytes(b4_nsb(K));
}
static void launch_b4_prepare(const float* kernels, int32_t K, int32_t Z, int mode0, int n_modes, uint16_t* out,
                              hipStream_t stream) {
    const int nsb = b4_nsb(K);
    const int n_rt = (Z + B4_TZ - 1) / B4_TZ;
    const int per_tile = 4 * 32 * b4_lstride(nsb);
    const dim3 grid((unsigned)((per_tile + 255) / 256), (unsigned)n_rt, (unsigned)n_modes);
    hipLaunchKernelGGL(b4_prepare_kernel, grid, dim3(256), 0, stream, kernels, K, Z, n_rt, nsb, out, mode0);
}
template <bool ADJ, bool PLAIN>
static void launch_b4_mode(const B4Geom& g, int nsb, const uint16_t* images, const float* in, float* out,
                           hipStream_t stream) {
    const dim3 grid(g.n_blocks), block(B4_THREADS);
    const size_t lds = b4_image_bytes(nsb);
    switch (nsb) {
        case 4: hipLaunchKernelGGL((tidas_b4_kernel<ADJ, 4, false, PLAIN>), grid, block, lds, stream, g, images, in, out, nullptr, 0); break;
        case 6: hipLaunchKernelGGL((tidas_b4_kernel<ADJ, 6, false, PLAIN>), grid, block, lds, stream, g, images, in, out, nullptr, 0); break;
        case 8: hipLaunchKernelGGL((tidas_b4_kernel<ADJ, 8, false, PLAIN>), grid, block, lds, stream, g, images, in, out, nullptr, 0); break;
        case 10: hipLaunchKernelGGL((tidas_b4_kernel<ADJ, 10, false, PLAIN>), grid, block, lds, stream, g, images, in, out, nullptr, 0); break;
        default: hipLaunchKernelGGL((tidas_b4_kernel<ADJ, 12, false, PLAIN>), grid, block, lds, stream, g, images, in, out, nullptr, 0); break;
    }
}
// images: the four-block band images of the operator's mode, tile rt at
// images + rt b4_image_bytes(nsb) / 2
static void launch_b4(bool adj, const uint16_t* images, int32_t K, const float* in, int32_t B, int32_t Z, int32_t X,
                      float alpha, float beta, const float* base, float* out, hipStream_t stream) {
    B4Geom g;
    g.K = K;
    g.B = B;
    g.Z = Z;
    g.X = X;
    g.n_rt = (Z + B4_TZ - 1) / B4_TZ;
    g.n_ct = (X + B4_TN - 1) / B4_TN;
    // frames per workgroup: one workgroup per compute unit in one round
    const int64_t tiles = (int64_t)g.n_rt * g.n_ct;
    g.nf = (int32_t)std::max<int64_t>(1, std::min<int64_t>(B, tiles * B / device_cu_count()));
    g.n_blocks = (int32_t)(tiles * ((B + g.nf - 1) / g.nf));
    g.alpha = alpha;
    g.beta = beta;
    g.base = base;
    // alpha = 1 and no base: the plain store (no base registers held)
    const bool plain = alpha == 1.0f && base == nullptr;
    if (adj) {
        if (plain) launch_b4_mode<true, true>(g, b4_nsb(K), images, in, out, stream);
        else launch_b4_mode<true, false>(g, b4_nsb(K), images, in, out, stream);
    } else {
        if (plain) launch_b4_mode<false, true>(g, b4_nsb(K), images, in, out, stream);
        else launch_b4_mode<false, false>(g, b4_nsb(K), images, in, out, stream);
    }
}

static bool mfma_fits(int K, int Z, int X) {
    // LDS tile fits; every int32 byte offset,
    // including rows prefetched past the band (< K + 4 PD + 64 rows beyond
    // the image), stays below 2^31
    return mf_lds_bytes(K) <= 160 * 1024 && ((int64_t)Z + 2 * K + 256) * X * 4 < INT32_MAX;
}

static void launch_mfma(bool adj, bool vec, const float* kernels, int32_t K, const float* in, int32_t B, int32_t Z,
                        int32_t X, float alpha, float beta, const float* base, float* out, hipStream_t stream) {
    ConvGeom g;
    g.K = K;
    g.h = (K - 1) / 2;
    g.B = B;
    g.Z = Z;
    g.X = X;
    g.n_rt = (Z + MF_TZ - 1) / MF_TZ;
    g.n_ct = (X + MF_TN - 1) / MF_TN;
    g.n_blocks = g.n_rt * g.n_ct * B;
    g.vec4 = vec;
    g.alpha = alpha;
    g.beta = beta;
    g.base = base;
    const size_t lds = mf_lds_bytes(K);
    const dim3 grid(g.n_blocks), block(MF_THREADS);
    if (adj) {
        if (vec) hipLaunchKernelGGL((tidas_mfma_kernel<true, 8, true>), grid, block, lds, stream, g, kernels, in, out);
        else hipLaunchKernelGGL((tidas_mfma_kernel<true, 8, false>), grid, block, lds, stream, g, kernels, in, out);
    } else {
        if (vec) hipLaunchKernelGGL((tidas_mfma_kernel<false, 8, true>), grid, block, lds, stream, g, kernels, in, out);
        else hipLaunchKernelGGL((tidas_mfma_kernel<false, 8, false>), grid, block, lds, stream, g, kernels, in, out);
    }
}

constexpr int CONV_RZ = 16;
constexpr int CONV_WAVES = 4;
constexpr size_t LDS_LIMIT = 160 * 1024;

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

static int32_t conv_validate(const char* name, const void* kernels, int32_t K, const float* in, int32_t B, int32_t Z,
                             int32_t X, float alpha, float beta, const float* base, const float* out) {
    if (!kernels || !in || !out) return fail(TIDAS_EINVAL, std::string(name) + ": null pointer");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, std::string(name) + ": K must be odd and >= 1");
    if (B < 1 || Z < 1 || X < 1) return fail(TIDAS_EINVAL, std::string(name) + ": B, Z, X must be >= 1");
    if ((const void*)in == (const void*)out || kernels == (const void*)out)
        return fail(TIDAS_EINVAL, std::string(name) + ": output aliases an input");
    if (base && ((const void*)base == (const void*)in || (const void*)base == kernels))
        return fail(TIDAS_EINVAL, std::string(name) + ": base aliases an input");
    if (!std::isfinite(alpha) || !std::isfinite(beta))
        return fail(TIDAS_EINVAL, std::string(name) + ": alpha and beta must be finite");
    return TIDAS_OK;
}

static bool bx_path(int32_t K, int32_t B, int32_t Z, int32_t X) {
    return bx_fits(K, Z, X) && (int64_t)((Z + BX_TZ - 1) / BX_TZ) * ((X + BX_TN - 1) / BX_TN) * B <= INT32_MAX;
}

static bool vec_ok(int32_t X, const float* in, const float* out, const float* base) {
    return (X % 4) == 0 && aligned16(in) && aligned16(out) && (!base || aligned16(base));
}

// Validate, pick the matrix-core or the VALU kernel, launch.  Enqueues nothing
// when it returns TIDAS_EINVAL / TIDAS_EUNSUPPORTED.  The split-bfloat16 path
// prepares the band images it needs in a stream-ordered temporary buffer, or,
// when `band` is given, in that device buffer of `band_bytes` bytes (too
// small: TIDAS_EUNSUPPORTED before anything is enqueued).
static int32_t conv_launch(bool adj, const char* name, const float* kernels, int32_t K, const float* in, int32_t B,
                           int32_t Z, int32_t X, float alpha, float beta, const float* base, float* out,
                           hipStream_t stream, void* band = nullptr, size_t band_bytes = 0) {
    int32_t st = conv_validate(name, kernels, K, in, B, Z, X, alpha, beta, base, out);
    if (st) return st;
    const bool vec = vec_ok(X, in, out, base);
    const bool four = b4_path(K, B, Z, X);
    if (four || bx_path(K, B, Z, X)) {
        // the band images of this one mode, in the layout of the chosen tile
        const size_t need = four ? b4_bytes(K, Z, 1) : prepared_bytes(K, Z, 1);
        void* buf = band;
        if (band) {
            if (need > band_bytes)
                return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": the band images (" + std::to_string(need) +
                                                    " bytes) exceed the " + std::to_string(band_bytes) +
                                                    "-byte scratch buffer");
        } else if ((st = check_hip(hipMallocAsync(&buf, need, stream), "band buffer"))) {
            return st;
        }
        if (four) launch_b4_prepare(kernels, K, Z, adj ? 1 : 0, 1, (uint16_t*)buf, stream);
        else launch_prepare(kernels, K, Z, adj ? 1 : 0, 1, (uint16_t*)buf, stream);
        st = check_launch(name);
        if (!st) {
            if (four) launch_b4(adj, (const uint16_t*)buf, K, in, B, Z, X, alpha, beta, base, out, stream);
            else launch_bx6(adj, vec, (const uint16_t*)buf, K, in, B, Z, X, alpha, beta, base, out, stream);
            st = check_launch(name);
        }
        if (band) return st;
        const int32_t st2 = check_hip(hipFreeAsync(buf, stream), "band buffer");
        return st ? st : st2;
    }
    const bool use_mfma = mfma_fits(K, Z, X) && (int64_t)((Z + MF_TZ - 1) / MF_TZ) * ((X + MF_TN - 1) / MF_TN) * B <= INT32_MAX;
    if (use_mfma) {
        launch_mfma(adj, vec, kernels, K, in, B, Z, X, alpha, beta, base, out, stream);
        return check_launch(name);
    }
    const size_t lds = (size_t)((adj ? 0 : CONV_RZ) + CONV_RZ * CONV_WAVES + K - 1) * 64 * sizeof(float);
    if (lds > LDS_LIMIT) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": K too large for the LDS tile");
    ConvGeom g;
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
    g.vec4 = 0;
    g.alpha = alpha;
    g.beta = beta;
    g.base = base;
    if (adj)
        hipLaunchKernelGGL((tidas_adj_kernel<CONV_RZ, CONV_WAVES>), dim3(g.n_blocks), dim3(CONV_WAVES * 64), lds,
                           stream, g, kernels, in, out);
    else
        hipLaunchKernelGGL((tidas_fwd_kernel<CONV_RZ, CONV_WAVES>), dim3(g.n_blocks), dim3(CONV_WAVES * 64), lds,
                           stream, g, kernels, in, out);
    return check_launch(name);
}

// Full prepared form of a bank: [two-block images, forward | adjoint] then,
// when K allows the four-block tile, [four-block images, forward | adjoint].
static size_t full_prepared_bytes(int32_t K, int32_t Z) {
    return prepared_bytes(K, Z, 2) + (b4_image_ok(K) ? b4_bytes(K, Z, 2) : 0);
}
static void prepare_full(const float* kernels, int32_t K, int32_t Z, uint16_t* buf, hipStream_t stream) {
    launch_prepare(kernels, K, Z, 0, 2, buf, stream);
    if (b4_image_ok(K)) launch_b4_prepare(kernels, K, Z, 0, 2, buf + prepared_bytes(K, Z, 2) / 2, stream);
}

// The split-bfloat16 operator on a full prepared form.
static int32_t conv_launch_images(bool adj, const char* name, const uint16_t* prepared, int32_t K, const float* in,
                                  int32_t B, int32_t Z, int32_t X, float alpha, float beta, const float* base,
                                  float* out, hipStream_t stream) {
    int32_t st = conv_validate(name, prepared, K, in, B, Z, X, alpha, beta, base, out);
    if (st) return st;
    if (b4_path(K, B, Z, X)) {
        const uint16_t* img = prepared + prepared_bytes(K, Z, 2) / 2 + (adj ? b4_bytes(K, Z, 1) / 2 : 0);
        launch_b4(adj, img, K, in, B, Z, X, alpha, beta, base, out, stream);
        return check_launch(name);
    }
    if (!bx_path(K, B, Z, X))
        return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": K or the frame size is outside the prepared path");
    const uint16_t* img = prepared + (adj ? prepared_bytes(K, Z, 1) / 2 : 0);
    launch_bx6(adj, vec_ok(X, in, out, base), img, K, in, B, Z, X, alpha, beta, base, out, stream);
    return check_launch(name);
}

// Step operator of the Tikhonov gradient iteration, N = (1 - eta lam) I -
// eta A^T A, as a line-model bank of 2K - 1 taps (offsets m = i - j from
// -(K - 1) to K - 1): Nb[i][m + K - 1] = N[i][i - m], with
//   (A^T A)[i][j] = sum_k A[k][i] A[k][j],  A[k][i] = K[k][k - i + h],
// k over the rows both columns reach (|k - i| <= h, |k - j| <= h, 0 <= k < Z);
// entries with j outside [0, Z) are 0.  Float64 sums; `nd` keeps the float64
// bank for the squared operator, `nf` the float32 bank of N + shift I.
__global__ __launch_bounds__(256) void normal_bank_kernel(const float* __restrict__ kb, int32_t K, int32_t Z,
                                                          double eta, double lam, double shift,
                                                          double* __restrict__ nd, float* __restrict__ nf) {
    const int KN = 2 * K - 1, h = (K - 1) / 2;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)Z * KN) return;
    const int i = (int)(idx / KN);
    const int m = (int)(idx % KN) - (K - 1);
    const int j = i - m;
    double v = 0.0;
    if (j >= 0 && j < Z) {
        const int k0 = max(max(i, j) - h, 0), k1 = min(min(i, j) + h, Z - 1);
        double acc = 0.0;
        for (int k = k0; k <= k1; ++k)
            acc += (double)kb[(size_t)k * K + (k - i + h)] * (double)kb[(size_t)k * K + (k - j + h)];
        v = -eta * acc + (i == j ? 1.0 - eta * lam : 0.0);
    }
    if (nd) nd[idx] = v;
    nf[idx] = (float)(v + (m == 0 && j < Z ? shift : 0.0));
}

// N^2 from the float64 bank of N (K1 = 2K - 1 taps, H1 = K1 / 2): a bank of
// 2 K1 - 1 taps, N2[i][j] = sum_k N[i][k] N[k][j] in float64, rounded once.
__global__ __launch_bounds__(256) void square_bank_kernel(const double* __restrict__ nd, int32_t K1, int32_t Z,
                                                          float* __restrict__ n2) {
    const int K2 = 2 * K1 - 1, H1 = (K1 - 1) / 2, H2 = (K2 - 1) / 2;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)Z * K2) return;
    const int i = (int)(idx / K2);
    const int m = (int)(idx % K2) - H2;
    const int j = i - m;
    double acc = 0.0;
    if (j >= 0 && j < Z) {
        const int k0 = max(max(i, j) - H1, 0), k1 = min(min(i, j) + H1, Z - 1);
        for (int k = k0; k <= k1; ++k)
            acc += nd[(size_t)i * K1 + (i - k) + H1] * nd[(size_t)k * K1 + (k - j) + H1];
    }
    n2[idx] = (float)acc;
}

__global__ __launch_bounds__(256) void fill_kernel(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

// Single-workgroup: norm of v (length n), v /= norm, *out_norm = norm.
__global__ __launch_bounds__(1024) void normalize_kernel(float* __restrict__ v, int32_t n, double* __restrict__ out_norm) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += (double)v[i] * (double)v[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += red[w];
        red[0] = sqrt(t);
        *out_norm = red[0];
    }
    __syncthreads();
    const double nrm = red[0];
    const float inv = nrm > 0.0 ? (float)(1.0 / nrm) : 0.0f;
    for (int i = threadIdx.x; i < n; i += 1024) v[i] *= inv;
}

// Band images of the allocation-free forward operator (tidas_apply_noalloc):
// a file-scope device array, one copy on every GPU the library runs on, held
// until the process ends and shared by every call on that GPU.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept in g_scratch.
constexpr size_t NOALLOC_SCRATCH_BYTES = TIDAS_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) uint8_t noalloc_scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mutex;
static void* g_scratch[NOALLOC_MAX_DEVICES] = {};

static int32_t noalloc_scratch_ptr(void** out) {
    int dev = -1;
    if (int32_t st = check_hip(hipGetDevice(&dev), "tidas_apply_noalloc: current device")) return st;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(TIDAS_EUNSUPPORTED, "tidas_apply_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (int32_t st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)),
                                   "tidas_apply_noalloc: scratch address"))
            return st;
        if (!p) return fail(TIDAS_EHIP, "tidas_apply_noalloc: scratch address is null");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TIDAS_OK;
}

}  // namespace tidas

using namespace tidas;

extern "C" int32_t tidas_apply_noalloc(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z,
                                       int32_t X, float* image, void* stream) {
    if (int32_t st = conv_validate("tidas_apply_noalloc", kernels, K, refl, B, Z, X, 1.0f, 0.0f, nullptr, image))
        return st;
    void* scratch = nullptr;
    if (int32_t st = noalloc_scratch_ptr(&scratch)) return st;
    return conv_launch(false, "tidas_apply_noalloc", kernels, K, refl, B, Z, X, 1.0f, 0.0f, nullptr, image,
                       (hipStream_t)stream, scratch, NOALLOC_SCRATCH_BYTES);
}

extern "C" int32_t tidas_apply(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z,
                               int32_t X, float* image, void* stream) {
    return conv_launch(false, "tidas_apply", kernels, K, refl, B, Z, X, 1.0f, 0.0f, nullptr, image,
                       (hipStream_t)stream);
}

extern "C" int32_t tidas_adjoint(const float* kernels, int32_t K, const float* image_bar, int32_t B, int32_t Z,
                                 int32_t X, float* refl_bar, void* stream) {
    return conv_launch(true, "tidas_adjoint", kernels, K, image_bar, B, Z, X, 1.0f, 0.0f, nullptr, refl_bar,
                       (hipStream_t)stream);
}

extern "C" int32_t tidas_apply_ex(const float* kernels, int32_t K, const float* refl, int32_t B, int32_t Z, int32_t X,
                                  float alpha, float beta, const float* base, float* image, void* stream) {
    return conv_launch(false, "tidas_apply_ex", kernels, K, refl, B, Z, X, alpha, beta, base, image,
                       (hipStream_t)stream);
}

extern "C" int32_t tidas_adjoint_ex(const float* kernels, int32_t K, const float* image_bar, int32_t B, int32_t Z,
                                    int32_t X, float alpha, float beta, const float* base, float* refl_bar,
                                    void* stream) {
    return conv_launch(true, "tidas_adjoint_ex", kernels, K, image_bar, B, Z, X, alpha, beta, base, refl_bar,
                       (hipStream_t)stream);
}

extern "C" int32_t tidas_line_kernel(int32_t K, int32_t B, int32_t Z, int32_t X) {
    if (K < 1 || (K % 2) == 0 || B < 1 || Z < 1 || X < 1)
        return fail(TIDAS_EINVAL, "tidas_line_kernel: K must be odd, K, B, Z, X >= 1");
    if (b4_path(K, B, Z, X)) return TIDAS_LINE_FOUR_BLOCK;
    if (bx_path(K, B, Z, X)) return TIDAS_LINE_TWO_BLOCK;
    if (mfma_fits(K, Z, X) && (int64_t)((Z + MF_TZ - 1) / MF_TZ) * ((X + MF_TN - 1) / MF_TN) * B <= INT32_MAX)
        return TIDAS_LINE_FP32_MATRIX;
    const size_t lds = (size_t)(CONV_RZ + CONV_RZ * CONV_WAVES + K - 1) * 64 * sizeof(float);
    return lds <= LDS_LIMIT ? TIDAS_LINE_VECTOR : fail(TIDAS_EUNSUPPORTED, "tidas_line_kernel: K too large");
}

extern "C" size_t tidas_prepared_bytes(int32_t K, int32_t Z) {
    if (K < 1 || (K % 2) == 0 || Z < 1 || bx_lds_bytes(K) > 160 * 1024) return 0;
    return full_prepared_bytes(K, Z);
}

extern "C" int32_t tidas_prepare(const float* kernels, int32_t K, int32_t Z, void* prepared, size_t bytes,
                                 void* stream) {
    if (!kernels || !prepared) return fail(TIDAS_EINVAL, "tidas_prepare: null pointer");
    if (K < 1 || (K % 2) == 0 || Z < 1) return fail(TIDAS_EINVAL, "tidas_prepare: K odd >= 1 and Z >= 1 required");
    if (bx_lds_bytes(K) > 160 * 1024) return fail(TIDAS_EUNSUPPORTED, "tidas_prepare: K too large for the prepared path");
    if (bytes < full_prepared_bytes(K, Z)) return fail(TIDAS_EINVAL, "tidas_prepare: buffer smaller than tidas_prepared_bytes");
    if ((reinterpret_cast<uintptr_t>(prepared) & 15) != 0) return fail(TIDAS_EINVAL, "tidas_prepare: buffer not 16-byte aligned");
    if ((const void*)kernels == prepared) return fail(TIDAS_EINVAL, "tidas_prepare: output aliases the bank");
    prepare_full(kernels, K, Z, (uint16_t*)prepared, (hipStream_t)stream);
    return check_launch("tidas_prepare");
}

extern "C" int32_t tidas_apply_prepared(const void* prepared, int32_t K, const float* refl, int32_t B, int32_t Z,
                                        int32_t X, float alpha, float beta, const float* base, float* image,
                                        void* stream) {
    return conv_launch_images(false, "tidas_apply_prepared", (const uint16_t*)prepared, K, refl, B, Z, X, alpha, beta,
                              base, image, (hipStream_t)stream);
}

extern "C" int32_t tidas_adjoint_prepared(const void* prepared, int32_t K, const float* image_bar, int32_t B,
                                          int32_t Z, int32_t X, float alpha, float beta, const float* base,
                                          float* refl_bar, void* stream) {
    return conv_launch_images(true, "tidas_adjoint_prepared", (const uint16_t*)prepared, K, image_bar, B, Z, X, alpha,
                              beta, base, refl_bar, (hipStream_t)stream);
}

// Scratch of one deconvolution: [N in float64 (two steps per launch) | N
// (or N + I) | N^2 | band images of the launch's bank | c | c2]; total 0 when
// the kernels are too long for the step-operator path.
struct DeconvLayout {
    bool one, two;
    int KN, KN2, KP;
    size_t off_nd, off_n1, off_np, off_img, off_c, off_c2, total;
};

static DeconvLayout deconv_layout(int32_t K, int32_t B, int32_t Z, int32_t X) {
    DeconvLayout L{};
    L.KN = 2 * K - 1;
    L.KN2 = 2 * L.KN - 1;
    L.two = bx_path(L.KN2, B, Z, X) && bx_lds_bytes(L.KN2) <= 160 * 1024;
    L.one = bx_path(L.KN, B, Z, X) && bx_lds_bytes(L.KN) <= 160 * 1024;
    if (!L.one) return L;
    L.KP = L.two ? L.KN2 : L.KN;
    const size_t frame_bytes = (size_t)B * Z * X * sizeof(float);
    L.off_nd = 0;
    L.off_n1 = L.off_nd + (L.two ? align_up((size_t)Z * L.KN * sizeof(double), 256) : 0);
    L.off_np = L.off_n1 + align_up((size_t)Z * L.KN * sizeof(float), 256);
    L.off_img = L.off_np + (L.two ? align_up((size_t)Z * L.KP * sizeof(float), 256) : 0);
    L.off_c = L.off_img + align_up(prepared_bytes(L.KP, Z, 1), 256);
    L.off_c2 = L.off_c + align_up(frame_bytes, 256);
    L.total = L.off_c2 + (L.two ? align_up(frame_bytes, 256) : 0);
    return L;
}

extern "C" size_t tidas_deconvolve_workspace_bytes(int32_t K, int32_t B, int32_t Z, int32_t X) {
    if (K < 1 || (K % 2) == 0 || B < 1 || Z < 1 || X < 1) return 0;
    return deconv_layout(K, B, Z, X).total;
}

extern "C" int32_t tidas_deconvolve(const float* kernels, int32_t K, const float* y, int32_t B, int32_t Z, int32_t X,
                                    float lam, float eta, int32_t iters, float* r, float* work, void* workspace,
                                    size_t workspace_bytes, void* stream) {
    if (!y || !r || !work || !kernels) return fail(TIDAS_EINVAL, "tidas_deconvolve: null pointer");
    if (iters < 0) return fail(TIDAS_EINVAL, "tidas_deconvolve: iters must be >= 0");
    if (!(lam >= 0.0f) || !std::isfinite(lam) || !(eta > 0.0f) || !std::isfinite(eta))
        return fail(TIDAS_EINVAL, "tidas_deconvolve: need finite lam >= 0 and eta > 0");
    if (K < 1 || (K % 2) == 0 || B < 1 || Z < 1 || X < 1)
        return fail(TIDAS_EINVAL, "tidas_deconvolve: K odd >= 1 and B, Z, X >= 1 required");
    const void* ptrs[4] = {kernels, y, r, work};
    for (int a = 0; a < 4; ++a)
        for (int c = a + 1; c < 4; ++c)
            if (ptrs[a] == ptrs[c]) return fail(TIDAS_EINVAL, "tidas_deconvolve: buffers must be distinct");
    const DeconvLayout L = deconv_layout(K, B, Z, X);
    if (int32_t st = workspace_check("tidas_deconvolve", workspace, workspace_bytes, L.total)) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)B * Z * X;
    if (iters == 0) {
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0, s, r,
                           n, 0.0f);
        return check_launch("tidas_deconvolve(zero)");
    }
    // r_{t+1} = N r_t + c with N = (1 - eta lam) I - eta A^T A and c = eta A^T y
    // (the same step, regrouped), r_1 = c; with N^2 and c2 = N c + c two steps
    // per launch: r_{t+2} = N^2 r_t + c2.  The step operator's bank has 2K - 1
    // taps (N^2: 4K - 3); both run on the split-bfloat16 two-block tile.
    const int KN = L.KN, KN2 = L.KN2;
    const bool two = L.two;
    if (!L.one) {
        // large kernels: two fused launches per step (residual, update)
        hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0, s, r,
                           n, 0.0f);
        int32_t st = check_launch("tidas_deconvolve(zero)");
        const float decay = 1.0f - eta * lam;
        for (int it = 0; it < iters && !st; ++it) {
            st = conv_launch(false, "tidas_deconvolve(residual)", kernels, K, r, B, Z, X, 1.0f, -1.0f, y, work, s);
            if (!st) st = conv_launch(true, "tidas_deconvolve(update)", kernels, K, work, B, Z, X, -eta, decay, r, r, s);
        }
        return st;
    }
    const int KP = L.KP;  // bank of one launch
    const size_t frame_bytes = (size_t)n * sizeof(float);
    Workspace ws;
    int32_t st = workspace_acquire("tidas_deconvolve: temporaries", workspace, L.total, s, ws);
    if (st) return st;
    char* tmp = ws.ptr;
    double* nd = two ? (double*)(tmp + L.off_nd) : nullptr;
    float* n1 = (float*)(tmp + L.off_n1);  // N, or N + I with two steps per launch
    float* np = two ? (float*)(tmp + L.off_np) : n1;
    uint16_t* img = (uint16_t*)(tmp + L.off_img);
    float* c = (float*)(tmp + L.off_c);
    float* c2 = two ? (float*)(tmp + L.off_c2) : nullptr;
    const int64_t e1 = (int64_t)Z * KN;
    // with two steps per launch n1 is N + I (for c2 = (N + I) c), else N
    hipLaunchKernelGGL(normal_bank_kernel, dim3((unsigned)((e1 + 255) / 256)), dim3(256), 0, s, kernels, K, Z,
                       (double)eta, (double)lam, two ? 1.0 : 0.0, nd, n1);
    st = check_launch("tidas_deconvolve(step operator)");
    if (!st && two) {
        const int64_t e2 = (int64_t)Z * KN2;
        hipLaunchKernelGGL(square_bank_kernel, dim3((unsigned)((e2 + 255) / 256)), dim3(256), 0, s, nd, KN, Z, np);
        st = check_launch("tidas_deconvolve(squared step operator)");
    }
    if (!st) {
        launch_prepare(np, KP, Z, 0, 1, img, s);
        st = check_launch("tidas_deconvolve(prepare)");
    }
    // c = eta A^T y
    if (!st) st = conv_launch(true, "tidas_deconvolve(c)", kernels, K, y, B, Z, X, eta, 0.0f, nullptr, c, s);
    // iterate from x = r_1 = c (or, two per launch with an even count, x = r_2 = c2)
    const float* x = c;
    int left = iters - 1;  // steps still to take
    const float* base = c;
    if (!st && two) {
        st = conv_launch(false, "tidas_deconvolve(c2)", n1, KN, c, B, Z, X, 1.0f, 0.0f, nullptr, c2, s);
        base = c2;
        if (iters % 2 == 0) {
            x = c2;
            left = iters - 2;
        }
    }
    const int per = two ? 2 : 1;
    int launches = left / per;
    // the last launch writes r, so launches alternate between work and r backwards from it
    float* bufs[2] = {r, work};
    for (int q = 0; q < launches && !st; ++q) {
        float* out = bufs[(launches - 1 - q) % 2];
        launch_bx6(false, vec_ok(X, x, out, base), img, KP, x, B, Z, X, 1.0f, 1.0f, base, out, s);
        st = check_launch("tidas_deconvolve(step)");
        x = out;
    }
    if (!st && launches == 0) {
        // iters = 1 (r = c), or iters = 2 with two steps per launch (r = c2)
        st = check_hip(hipMemcpyAsync(r, x, frame_bytes, hipMemcpyDeviceToDevice, s), "tidas_deconvolve: copy");
    }
    const int32_t st2 = workspace_release("tidas_deconvolve: temporaries", ws, s);
    return st ? st : st2;
}

extern "C" size_t tidas_operator_norm_sq_workspace_bytes(int32_t K, int32_t Z) {
    if (K < 1 || (K % 2) == 0 || Z < 1 || !bx_path(K, 1, Z, 1)) return 0;
    return full_prepared_bytes(K, Z);
}

extern "C" int32_t tidas_operator_norm_sq(const float* kernels, int32_t K, int32_t Z, int32_t iters, float* work,
                                          double* out, void* workspace, size_t workspace_bytes, void* stream) {
    if (!kernels || !work || !out) return fail(TIDAS_EINVAL, "tidas_operator_norm_sq: null pointer");
    if (K < 1 || (K % 2) == 0 || Z < 1 || iters < 1)
        return fail(TIDAS_EINVAL, "tidas_operator_norm_sq: K odd >= 1, Z >= 1, iters >= 1 required");
    const bool bx = bx_path(K, 1, Z, 1);
    const size_t need = bx ? full_prepared_bytes(K, Z) : 0;
    if (int32_t st = workspace_check("tidas_operator_norm_sq", workspace, workspace_bytes, need)) return st;
    hipStream_t s = (hipStream_t)stream;
    // work layout: v [Z] | Av [Z] | w [Z] | norm (double, 8-byte aligned); v and w swap roles
    float* v = work;
    float* av = work + Z;
    float* w = work + 2 * (size_t)Z;
    double* nrm = reinterpret_cast<double*>(work + 3 * (size_t)Z + ((3 * (size_t)Z) & 1));
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<int64_t>((Z + 255) / 256, 65536)), dim3(256), 0, s, v,
                       (int64_t)Z, 1.0f);
    int32_t st = check_launch("tidas_operator_norm_sq(init)");
    Workspace ws;
    if (!st && bx && !(st = workspace_acquire("tidas_operator_norm_sq: bands", workspace, need, s, ws))) {
        prepare_full(kernels, K, Z, (uint16_t*)ws.ptr, s);
        st = check_launch("tidas_operator_norm_sq(prepare)");
    }
    const uint16_t* prep = (const uint16_t*)ws.ptr;
    for (int it = 0; it < iters && !st; ++it) {
        // v <- A^T A v / ||A^T A v||; the last norm is the largest eigenvalue of A^T A
        if (bx) {
            st = conv_launch_images(false, "tidas_operator_norm_sq", prep, K, v, 1, Z, 1, 1.0f, 0.0f, nullptr, av, s);
            if (!st) st = conv_launch_images(true, "tidas_operator_norm_sq", prep, K, av, 1, Z, 1, 1.0f, 0.0f, nullptr, w, s);
        } else {
            st = conv_launch(false, "tidas_operator_norm_sq", kernels, K, v, 1, Z, 1, 1.0f, 0.0f, nullptr, av, s);
            if (!st) st = conv_launch(true, "tidas_operator_norm_sq", kernels, K, av, 1, Z, 1, 1.0f, 0.0f, nullptr, w, s);
        }
        if (!st) {
            hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, w, Z, nrm);
            st = check_launch("tidas_operator_norm_sq(normalize)");
        }
        std::swap(v, w);
    }
    const int32_t st2 = workspace_release("tidas_operator_norm_sq: bands", ws, s);
    if (!st) st = st2;
    if (!st) st = check_hip(hipMemcpyAsync(out, nrm, sizeof(double), hipMemcpyDeviceToHost, s), "norm download");
    if (!st) st = check_hip(hipStreamSynchronize(s), "tidas_operator_norm_sq: synchronize");
    return st;
}

// Four-block ragged batch: byte offset of every frame's forward band images
// after the frame table, and the total (0 when K does not fit the tile or
// there are too many 128-row tiles for one launch).
static size_t b4_batch_layout(const tidas_frame* frames, int32_t n_frames, int32_t K, std::vector<int64_t>* offs,
                              int64_t* tiles) {
    if (!b4_image_ok(K) || n_frames < 1) return 0;
    size_t off = tidas_batch_workspace_bytes(n_frames);
    int64_t t = 0;
    for (int f = 0; f < n_frames; ++f) {
        const int Z = frames[f].grid.nz;
        if (Z < 1 || frames[f].grid.nx < 1) return 0;
        if (offs) offs->push_back((int64_t)off);
        off += b4_bytes(K, Z, 1);
        t += (Z + B4_TZ - 1) / B4_TZ;
    }
    if (t > 65535) return 0;
    if (tiles) *tiles = t;
    return off;
}

extern "C" size_t tidas_apply_batch_workspace_bytes(const tidas_frame* frames, int32_t n_frames, int32_t K) {
    if (!frames || n_frames < 1 || K < 1 || (K % 2) == 0) return 0;
    const size_t four = b4_batch_layout(frames, n_frames, K, nullptr, nullptr);
    return std::max(four, tidas_batch_workspace_bytes(n_frames));
}

// Four-block batch, step 1: validate, upload the frame table (tile_start in
// 128-row tiles, img_off the frame's band images) and prepare every frame's
// forward band images in the workspace.  *tiles receives the tile count.
static int32_t b4_batch_prepare(const char* name, const tidas_frame* frames, int32_t n_frames, int32_t K,
                                void* workspace, size_t workspace_bytes, int64_t* tiles, hipStream_t s) {
    std::vector<int64_t> offs;
    const size_t need = b4_batch_layout(frames, n_frames, K, &offs, tiles);
    if (need == 0)
        return fail(TIDAS_EUNSUPPORTED,
                    std::string(name) + ": the four-block batch needs K <= 161 and at most 65535 tiles of 128 rows");
    if (workspace_bytes < need)
        return fail(TIDAS_EINVAL, std::string(name) + ": workspace too small for the four-block batch "
                                                      "(see tidas_apply_batch_workspace_bytes)");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(TIDAS_EINVAL, std::string(name) + ": the four-block batch needs a 256-byte aligned workspace");
    std::vector<ConvFrameDev> tab(n_frames);
    int64_t t0 = 0;
    for (int f = 0; f < n_frames; ++f) {
        const tidas_frame& fr = frames[f];
        const int Z = fr.grid.nz, X = fr.grid.nx;
        if (!b4_fits(K, Z, X)) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": frame too large for the tile path");
        if (fr.in == fr.out || (const void*)fr.kernels == (const void*)fr.out)
            return fail(TIDAS_EINVAL, std::string(name) + ": output aliases an input");
        tab[f] = ConvFrameDev{fr.kernels, fr.in, fr.out, Z, X, 0, 0, t0, offs[f]};
        t0 += (Z + B4_TZ - 1) / B4_TZ;
    }
    // hipMemcpyAsync from pageable memory returns once the source is staged
    int32_t st = check_hip(hipMemcpyAsync(workspace, tab.data(), sizeof(ConvFrameDev) * n_frames,
                                          hipMemcpyHostToDevice, s),
                           "four-block batch: table upload");
    if (st) return st;
    const int nsb = b4_nsb(K);
    const int per_tile = 4 * 32 * b4_lstride(nsb);
    hipLaunchKernelGGL(b4_batch_prepare_kernel, dim3((unsigned)((per_tile + 255) / 256), (unsigned)*tiles), dim3(256),
                       0, s, (const ConvFrameDev*)workspace, n_frames, K, nsb, (uint16_t*)workspace);
    return check_launch(name);
}

// Four-block batch, step 2: one workgroup per 128-row tile of every frame.
static int32_t b4_batch_launch(const char* name, int32_t n_frames, int32_t K, const void* workspace, int64_t tiles,
                               hipStream_t s) {
    B4Geom g{};
    g.K = K;
    g.n_blocks = (int32_t)tiles;
    g.alpha = 1.0f;
    g.beta = 0.0f;
    const dim3 grid((unsigned)tiles), block(B4_THREADS);
    const int nsb = b4_nsb(K);
    const size_t lds = b4_image_bytes(nsb);
    const ConvFrameDev* d = (const ConvFrameDev*)workspace;
    const uint16_t* img = (const uint16_t*)workspace;
    switch (nsb) {
        case 4: hipLaunchKernelGGL((tidas_b4_kernel<false, 4, true, true>), grid, block, lds, s, g, img, nullptr, nullptr, d, n_frames); break;
        case 6: hipLaunchKernelGGL((tidas_b4_kernel<false, 6, true, true>), grid, block, lds, s, g, img, nullptr, nullptr, d, n_frames); break;
        case 8: hipLaunchKernelGGL((tidas_b4_kernel<false, 8, true, true>), grid, block, lds, s, g, img, nullptr, nullptr, d, n_frames); break;
        case 10: hipLaunchKernelGGL((tidas_b4_kernel<false, 10, true, true>), grid, block, lds, s, g, img, nullptr, nullptr, d, n_frames); break;
        default: hipLaunchKernelGGL((tidas_b4_kernel<false, 12, true, true>), grid, block, lds, s, g, img, nullptr, nullptr, d, n_frames); break;
    }
    return check_launch(name);
}

extern "C" int32_t tidas_apply_batch_prepare(const tidas_frame* frames, int32_t n_frames, int32_t K, void* workspace,
                                             size_t workspace_bytes, void* stream) {
    int32_t st = validate_batch("tidas_apply_batch_prepare", frames, n_frames, workspace, workspace_bytes, false, true);
    if (st) return st;
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_apply_batch_prepare: K must be odd and >= 1");
    int64_t tiles = 0;
    return b4_batch_prepare("tidas_apply_batch_prepare", frames, n_frames, K, workspace, workspace_bytes, &tiles,
                            (hipStream_t)stream);
}

extern "C" int32_t tidas_apply_batch_prepared(const tidas_frame* frames, int32_t n_frames, int32_t K,
                                              const void* workspace, size_t workspace_bytes, void* stream) {
    int32_t st = validate_batch("tidas_apply_batch_prepared", frames, n_frames, const_cast<void*>(workspace),
                                workspace_bytes, false, true);
    if (st) return st;
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_apply_batch_prepared: K must be odd and >= 1");
    int64_t tiles = 0;
    const size_t need = b4_batch_layout(frames, n_frames, K, nullptr, &tiles);
    if (need == 0)
        return fail(TIDAS_EUNSUPPORTED, "tidas_apply_batch_prepared: the four-block batch needs K <= 161 and at "
                                        "most 65535 tiles of 128 rows");
    if (workspace_bytes < need) return fail(TIDAS_EINVAL, "tidas_apply_batch_prepared: workspace too small");
    return b4_batch_launch("tidas_apply_batch_prepared", n_frames, K, workspace, tiles, (hipStream_t)stream);
}

extern "C" int32_t tidas_apply_batch(const tidas_frame* frames, int32_t n_frames, int32_t K, void* workspace,
                                     size_t workspace_bytes, int32_t variant, void* stream) {
    int32_t st = validate_batch("tidas_apply_batch", frames, n_frames, workspace, workspace_bytes, false, true);
    if (st) return st;
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_apply_batch: K must be odd and >= 1");
    if (variant < 0 || variant >= TIDAS_APPLY_BATCH_VARIANTS)
        return fail(TIDAS_EINVAL, "tidas_apply_batch: variant out of range");
    if (variant == TIDAS_APPLY_BATCH_FOUR_BLOCK) {
        int64_t tiles = 0;
        if ((st = b4_batch_prepare("tidas_apply_batch", frames, n_frames, K, workspace, workspace_bytes, &tiles,
                                   (hipStream_t)stream)))
            return st;
        return b4_batch_launch("tidas_apply_batch", n_frames, K, workspace, tiles, (hipStream_t)stream);
    }
    // the same arithmetic as tidas_apply on each frame: the split-bfloat16
    // tiles when the band fits (a visit = one 64-row tile, all its columns),
    // else the float32 matrix-core tiles
    const bool bx = bx_lds_bytes(K) <= 160 * 1024;
    const int TZ = bx ? BX_TZ : MF_TZ, TN = bx ? INT32_MAX / 2 : MF_TN;
    std::vector<ConvFrameDev> tab(n_frames);
    int64_t total = 0;
    for (int f = 0; f < n_frames; ++f) {
        const tidas_frame& fr = frames[f];
        const int Z = fr.grid.nz, X = fr.grid.nx;
        if (!(bx ? bx_fits(K, Z, X) : mfma_fits(K, Z, X)))
            return fail(TIDAS_EUNSUPPORTED, "tidas_apply_batch: frame too large for the tile path");
        if (fr.in == fr.out || (const void*)fr.kernels == (const void*)fr.out)
            return fail(TIDAS_EINVAL, "tidas_apply_batch: output aliases an input");
        tab[f].kernels = fr.kernels;
        tab[f].in = fr.in;
        tab[f].out = fr.out;
        tab[f].Z = Z;
        tab[f].X = X;
        tab[f].vec = (X % 4) == 0 && aligned16(fr.in) && aligned16(fr.out);
        tab[f].pad = 0;
        tab[f].tile_start = total;
        tab[f].img_off = 0;
        total += (int64_t)((Z + TZ - 1) / TZ) * ((X + TN - 1) / TN);
    }
    hipStream_t s = (hipStream_t)stream;
    // hipMemcpyAsync from pageable memory returns once the source is staged
    if ((st = check_hip(hipMemcpyAsync(workspace, tab.data(), sizeof(ConvFrameDev) * n_frames, hipMemcpyHostToDevice, s),
                        "tidas_apply_batch: table upload")))
        return st;
    const int n_cu = device_cu_count();
    const ConvFrameDev* d = (const ConvFrameDev*)workspace;
    if (bx) {
        // variants: workgroups per compute unit
        static const int bx_per_cu[TIDAS_APPLY_BATCH_FOUR_BLOCK] = {1, 2, 3, 4, 6, 8};
        auto grid_for = [&](int64_t t) {
            const int64_t nb = std::max<int64_t>(8, std::min<int64_t>(t, (int64_t)n_cu * bx_per_cu[variant]));
            return (unsigned)((nb + 7) / 8 * 8);
        };
        hipLaunchKernelGGL(tidas_bx6_batch_kernel, dim3(grid_for(total)), dim3(BX_THREADS), bx_lds_bytes(K), s, d,
                           n_frames, total, K);
        return check_launch("tidas_apply_batch");
    }
    const int pd_sel = variant % 3, per_cu = (variant / 3) == 0 ? 2 : 4;
    // a multiple of 8 workgroups: the tile list is cut into 8 chunks, one per
    // residue of the block id, and every chunk needs at least one workgroup
    const int64_t nb = std::max<int64_t>(8, std::min<int64_t>(total, (int64_t)n_cu * per_cu));
    const unsigned nblk = (unsigned)((nb + 7) / 8 * 8);
    const size_t lds = mf_lds_bytes(K);
    if (pd_sel == 0) hipLaunchKernelGGL(tidas_batch_kernel<4>, dim3(nblk), dim3(MF_THREADS), lds, s, d, n_frames, total, K);
    else if (pd_sel == 1) hipLaunchKernelGGL(tidas_batch_kernel<8>, dim3(nblk), dim3(MF_THREADS), lds, s, d, n_frames, total, K);
    else hipLaunchKernelGGL(tidas_batch_kernel<16>, dim3(nblk), dim3(MF_THREADS), lds, s, d, n_frames, total, K);
    return check_launch("tidas_apply_batch");
}
