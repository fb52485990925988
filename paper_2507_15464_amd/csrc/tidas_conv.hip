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
#include <algorithm>
#include <utility>
#include <vector>

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

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Validate, pick the matrix-core or the VALU kernel, launch.  Enqueues nothing
// when it returns TIDAS_EINVAL / TIDAS_EUNSUPPORTED.
static int32_t conv_launch(bool adj, const char* name, const float* kernels, int32_t K, const float* in, int32_t B,
                           int32_t Z, int32_t X, float alpha, float beta, const float* base, float* out,
                           hipStream_t stream) {
    if (!kernels || !in || !out) return fail(TIDAS_EINVAL, std::string(name) + ": null pointer");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, std::string(name) + ": K must be odd and >= 1");
    if (B < 1 || Z < 1 || X < 1) return fail(TIDAS_EINVAL, std::string(name) + ": B, Z, X must be >= 1");
    if ((const void*)in == (const void*)out || (const void*)kernels == (const void*)out)
        return fail(TIDAS_EINVAL, std::string(name) + ": output aliases an input");
    if (base && ((const void*)base == (const void*)in || (const void*)base == (const void*)kernels))
        return fail(TIDAS_EINVAL, std::string(name) + ": base aliases an input");
    if (!std::isfinite(alpha) || !std::isfinite(beta))
        return fail(TIDAS_EINVAL, std::string(name) + ": alpha and beta must be finite");
    const bool use_mfma = mfma_fits(K, Z, X) && (int64_t)((Z + MF_TZ - 1) / MF_TZ) * ((X + MF_TN - 1) / MF_TN) * B <= INT32_MAX;
    if (use_mfma) {
        const bool vec = (X % 4) == 0 && aligned16(in) && aligned16(out) && (!base || aligned16(base));
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

}  // namespace tidas

using namespace tidas;

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

extern "C" int32_t tidas_deconvolve(const float* kernels, int32_t K, const float* y, int32_t B, int32_t Z, int32_t X,
                                    float lam, float eta, int32_t iters, float* r, float* work, void* stream) {
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
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)B * Z * X;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 65536)), dim3(256), 0, s, r, n,
                       0.0f);
    int32_t st = check_launch("tidas_deconvolve(zero)");
    const float decay = 1.0f - eta * lam;
    for (int it = 0; it < iters && !st; ++it) {
        // work = A r - y ;  r = -eta A^T work + (1 - eta lam) r
        st = conv_launch(false, "tidas_deconvolve(residual)", kernels, K, r, B, Z, X, 1.0f, -1.0f, y, work, s);
        if (!st)
            st = conv_launch(true, "tidas_deconvolve(update)", kernels, K, work, B, Z, X, -eta, decay, r, r, s);
    }
    return st;
}

extern "C" int32_t tidas_operator_norm_sq(const float* kernels, int32_t K, int32_t Z, int32_t iters, float* work,
                                          double* out, void* stream) {
    if (!kernels || !work || !out) return fail(TIDAS_EINVAL, "tidas_operator_norm_sq: null pointer");
    if (K < 1 || (K % 2) == 0 || Z < 1 || iters < 1)
        return fail(TIDAS_EINVAL, "tidas_operator_norm_sq: K odd >= 1, Z >= 1, iters >= 1 required");
    hipStream_t s = (hipStream_t)stream;
    // work layout: v [Z] | Av [Z] | w [Z] | norm (double, 8-byte aligned); v and w swap roles
    float* v = work;
    float* av = work + Z;
    float* w = work + 2 * (size_t)Z;
    double* nrm = reinterpret_cast<double*>(work + 3 * (size_t)Z + ((3 * (size_t)Z) & 1));
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<int64_t>((Z + 255) / 256, 65536)), dim3(256), 0, s, v,
                       (int64_t)Z, 1.0f);
    int32_t st = check_launch("tidas_operator_norm_sq(init)");
    for (int it = 0; it < iters && !st; ++it) {
        // v <- A^T A v / ||A^T A v||; the last norm is the largest eigenvalue of A^T A
        st = conv_launch(false, "tidas_operator_norm_sq", kernels, K, v, 1, Z, 1, 1.0f, 0.0f, nullptr, av, s);
        if (!st) st = conv_launch(true, "tidas_operator_norm_sq", kernels, K, av, 1, Z, 1, 1.0f, 0.0f, nullptr, w, s);
        if (!st) {
            hipLaunchKernelGGL(normalize_kernel, dim3(1), dim3(1024), 0, s, w, Z, nrm);
            st = check_launch("tidas_operator_norm_sq(normalize)");
        }
        std::swap(v, w);
    }
    if (!st) st = check_hip(hipMemcpyAsync(out, nrm, sizeof(double), hipMemcpyDeviceToHost, s), "norm download");
    if (!st) st = check_hip(hipStreamSynchronize(s), "tidas_operator_norm_sq: synchronize");
    return st;
}

extern "C" int32_t tidas_apply_batch(const tidas_frame* frames, int32_t n_frames, int32_t K, void* workspace,
                                     size_t workspace_bytes, int32_t variant, void* stream) {
    int32_t st = validate_batch("tidas_apply_batch", frames, n_frames, workspace, workspace_bytes, false, true);
    if (st) return st;
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_apply_batch: K must be odd and >= 1");
    if (variant < 0 || variant >= TIDAS_APPLY_BATCH_VARIANTS)
        return fail(TIDAS_EINVAL, "tidas_apply_batch: variant out of range");
    std::vector<ConvFrameDev> tab(n_frames);
    int64_t total = 0;
    for (int f = 0; f < n_frames; ++f) {
        const tidas_frame& fr = frames[f];
        const int Z = fr.grid.nz, X = fr.grid.nx;
        if (!mfma_fits(K, Z, X)) return fail(TIDAS_EUNSUPPORTED, "tidas_apply_batch: frame too large for the tile path");
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
        total += (int64_t)((Z + MF_TZ - 1) / MF_TZ) * ((X + MF_TN - 1) / MF_TN);
    }
    hipStream_t s = (hipStream_t)stream;
    // hipMemcpyAsync from pageable memory returns once the source is staged
    if ((st = check_hip(hipMemcpyAsync(workspace, tab.data(), sizeof(ConvFrameDev) * n_frames, hipMemcpyHostToDevice, s),
                        "tidas_apply_batch: table upload")))
        return st;
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
    }
    const int pd_sel = variant % 3, per_cu = (variant / 3) == 0 ? 2 : 4;
    // a multiple of 8 workgroups: the tile list is cut into 8 chunks, one per
    // residue of the block id, and every chunk needs at least one workgroup
    const int64_t nb = std::max<int64_t>(8, std::min<int64_t>(total, (int64_t)n_cu * per_cu));
    const unsigned nblk = (unsigned)((nb + 7) / 8 * 8);
    const size_t lds = mf_lds_bytes(K);
    const ConvFrameDev* d = (const ConvFrameDev*)workspace;
    if (pd_sel == 0) hipLaunchKernelGGL(tidas_batch_kernel<4>, dim3(nblk), dim3(MF_THREADS), lds, s, d, n_frames, total, K);
    else if (pd_sel == 1) hipLaunchKernelGGL(tidas_batch_kernel<8>, dim3(nblk), dim3(MF_THREADS), lds, s, d, n_frames, total, K);
    else hipLaunchKernelGGL(tidas_batch_kernel<16>, dim3(nblk), dim3(MF_THREADS), lds, s, d, n_frames, total, K);
    return check_launch("tidas_apply_batch");
}
