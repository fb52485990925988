// Kernel-surrogate MLP on matrix cores: 4 -> 256 -> 256 -> 256 -> K with
// GELU, bfloat16 operands and float32 accumulation (v_mfma_f32_16x16x32_bf16),
// trained by the library's own forward, backward and Adam kernels.
//
// Parameters are one flat float32 buffer, layer by layer: W_l [out][in] then
// b_l [out].  A bfloat16 copy of the same buffer feeds the GEMMs.  Rounding
// points (round to nearest even): the input features, every weight matrix,
// each hidden activation before the next GEMM, and each back-propagated
// gradient before its GEMMs; sums, biases, GELU and its derivative stay in
// float32.
//
// One GEMM kernel serves every product: C[m][n] = sum_k A(m, k) B(k, n) with
// A(m, k) = A[m sam + k sak] and B(k, n) = B[k sbk + n sbn] (bfloat16), so the
// forward (H W^T), data-gradient (G W) and weight-gradient (G^T H) products
// differ only in strides.  Tiles of 32 x 32 outputs, 4 waves, each wave a
// 16 x 16 block (one MFMA 16x16x32 accumulator): the 1024 x 256 products of
// a training step then take 256 workgroups, one per compute unit, where 64 x
// 64 tiles took 64 and left the launches to four times the latency.  The k
// dimension is staged in LDS in blocks of 128 with operands stored
// k-contiguous, and multiplied in chunks of 32, so each lane's 8 bfloat16
// operand values are one 16-byte LDS read.
//   A operand (16 x 32): lane l holds A[l % 16][8 (l / 16) .. +7]
//   B operand (32 x 16): lane l holds B[8 (l / 16) .. +7][l % 16]
//   D (16 x 16): register r of lane l holds D[4 (l / 16) + r][l % 16]
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace tidas {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS_SCALE = 2, EPI_GELU_GRAD = 3 };

struct GemmArgs {
    const uint16_t* A;
    int64_t sam, sak;
    const uint16_t* B;
    int64_t sbk, sbn;
    int32_t M, N, K;
    float* c32;     // float32 output (all epilogues)
    int64_t ldc;
    uint16_t* c16;  // bfloat16 copy of the activation / gradient (GELU epilogues)
    int64_t ldc16;
    const float* bias;   // [N]
    const float* scale;  // [M] row scale (EPI_BIAS_SCALE) or null
    const float* zin;    // pre-activations for GELU' (EPI_GELU_GRAD)
    int64_t ldz;
};

// output tiles of GM x GN per workgroup (four waves, each GM / 2 x GN / 2 in
// 16 x 16 blocks)
constexpr int GM = 32, GN = 32, GK = 32, GPAD = 8;
constexpr int GW = GM / 2, GSUB = GW / 16;
constexpr int GKB = 128;  // k staged in LDS at once
static_assert(GM == GN, "operand staging assumes square tiles");

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[GM][GKB + GPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[GN][GKB + GPAD];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * GM, n0 = blockIdx.y * GN;
    const int wr = (wave >> 1) * GW, wc = (wave & 1) * GW;
    const int li = lane & 15, lq = lane >> 4;
    // split-K: slice blockIdx.z of gridDim.z covers [kbeg, kend), a whole number of GK chunks
    const int kper = ((g.K + (int)gridDim.z - 1) / (int)gridDim.z + GK - 1) / GK * GK;
    const int kbeg = blockIdx.z * kper;
    const int kend = min(g.K, kbeg + kper);
    floatx4 acc[GSUB][GSUB];
#pragma unroll
    for (int a = 0; a < GSUB; ++a)
#pragma unroll
        for (int b = 0; b < GSUB; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    // The slice's k moves through LDS in blocks of GKB = 128: every load of a block
    // is issued before the first is awaited (one memory latency per block, not
    // one per 32-wide chunk: these products are small and latency-bound),
    // then its chunks of GK are multiplied in ascending order, as a chunk-by-
    // chunk walk would.  Each thread stages PER elements of each operand:
    // element j of thread t is (row, k) = (t / GKB + j * 256 / GKB, t % GKB)
    // when the operand is k-contiguous in memory and (t % GM, t / GM + j *
    // 256 / GM) otherwise, so neighbouring threads read neighbouring
    // addresses in both layouts.  Rows past the operand and k past the slice
    // read a clamped (valid) address; such rows only feed outputs that are
    // not stored, and the k past the slice up to the chunk's end are set to
    // zero in LDS in both operands before the products.
    constexpr int PER = (GM * GKB) / 256;
    struct Walk {
        int r0, k0, dr, dk;
    };
    auto walk = [&](bool kfast) {
        return kfast ? Walk{tid / GKB, tid % GKB, 256 / GKB, 0} : Walk{tid % GM, tid / GM, 0, 256 / GM};
    };
    const Walk wa_ = walk(g.sak == 1), wb_ = walk(g.sbk == 1);
    // byte offsets (32-bit: the host checks the operands' extents) through
    // buffer records over each operand
    const int sam = (int)g.sam * 2, sak = (int)g.sak * 2, sbk = (int)g.sbk * 2, sbn = (int)g.sbn * 2;
    const auto rsa = make_rsrc(g.A, 0x7fffffff), rsb = make_rsrc(g.B, 0x7fffffff);
    for (int kb = kbeg; kb < kend; kb += GKB) {
        const int kn = min(GKB, kend - kb);
        uint16_t ra[PER], rb[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int ma = min(m0 + wa_.r0 + j * wa_.dr, g.M - 1), ka = kb + min(wa_.k0 + j * wa_.dk, kn - 1);
            const int nb = min(n0 + wb_.r0 + j * wb_.dr, g.N - 1), kb_ = kb + min(wb_.k0 + j * wb_.dk, kn - 1);
            ra[j] = __builtin_amdgcn_raw_buffer_load_b16(rsa, ma * sam + ka * sak, 0, 0);
            rb[j] = __builtin_amdgcn_raw_buffer_load_b16(rsb, kb_ * sbk + nb * sbn, 0, 0);
        }
        if (kb > kbeg) __syncthreads();  // the previous block's reads are done
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            As[wa_.r0 + j * wa_.dr][wa_.k0 + j * wa_.dk] = ra[j];
            Bs[wb_.r0 + j * wb_.dr][wb_.k0 + j * wb_.dk] = rb[j];
        }
        const int kpad = (kn + GK - 1) / GK * GK;
        if (kpad > kn) {
            __syncthreads();  // the staged values are in place before the padding overwrites them
            const int w = kpad - kn;
            for (int e = tid; e < GM * w; e += 256) {
                As[e / w][kn + e % w] = 0;
                Bs[e / w][kn + e % w] = 0;
            }
        }
        __syncthreads();
        const int nch = (kn + GK - 1) / GK;
        for (int c = 0; c < nch; ++c) {
            bf16x8 af[GSUB], bfr[GSUB];
#pragma unroll
            for (int a = 0; a < GSUB; ++a)
                af[a] = *reinterpret_cast<const bf16x8*>(&As[wr + 16 * a + li][GK * c + 8 * lq]);
#pragma unroll
            for (int b = 0; b < GSUB; ++b)
                bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[wc + 16 * b + li][GK * c + 8 * lq]);
#pragma unroll
            for (int a = 0; a < GSUB; ++a)
#pragma unroll
                for (int b = 0; b < GSUB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        }
    }

    // split-K partials go to slice blockIdx.z of c32 (reduced afterwards)
    float* c32 = g.c32 + (int64_t)blockIdx.z * g.M * g.ldc;
#pragma unroll
    for (int a = 0; a < GSUB; ++a)
#pragma unroll
        for (int b = 0; b < GSUB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr + 16 * a + 4 * lq + r;
                const int n = n0 + wc + 16 * b + li;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[a][b][r];
                if (EPI == EPI_STORE) {
                    c32[(int64_t)m * g.ldc + n] = v;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float z = v + g.bias[n];
                    g.c32[(int64_t)m * g.ldc + n] = z;
                    g.c16[(int64_t)m * g.ldc16 + n] = to_bf16(gelu(z));
                } else if (EPI == EPI_BIAS_SCALE) {
                    float y = v + g.bias[n];
                    if (g.scale) y *= g.scale[m];
                    g.c32[(int64_t)m * g.ldc + n] = y;
                } else {  // EPI_GELU_GRAD
                    const float d = v * gelu_grad(g.zin[(int64_t)m * g.ldz + n]);
                    g.c32[(int64_t)m * g.ldc + n] = d;
                    g.c16[(int64_t)m * g.ldc16 + n] = to_bf16(d);
                }
            }
}

static void gemm(int epi, const GemmArgs& g, hipStream_t s, int splits = 1) {
    const dim3 grid((g.M + GM - 1) / GM, (g.N + GN - 1) / GN, splits), block(256);
    switch (epi) {
        case EPI_STORE: hipLaunchKernelGGL(gemm_bf16_kernel<EPI_STORE>, grid, block, 0, s, g); break;
        case EPI_BIAS_GELU: hipLaunchKernelGGL(gemm_bf16_kernel<EPI_BIAS_GELU>, grid, block, 0, s, g); break;
        case EPI_BIAS_SCALE: hipLaunchKernelGGL(gemm_bf16_kernel<EPI_BIAS_SCALE>, grid, block, 0, s, g); break;
        default: hipLaunchKernelGGL(gemm_bf16_kernel<EPI_GELU_GRAD>, grid, block, 0, s, g); break;
    }
}

// x16[b][i] = bf16(x[row(b)][i]); t32[b][o] = t[row(b)][o] (rows gathered through idx when given)
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ x, int32_t in, const float* __restrict__ t,
                                                     int32_t out, const int32_t* __restrict__ idx, int32_t n_rows,
                                                     int32_t N, uint16_t* __restrict__ x16, float* __restrict__ t32) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nx = (int64_t)N * in, nt = t ? (int64_t)N * out : 0;
    if (e < nx) {
        const int b = (int)(e / in), i = (int)(e % in);
        const int64_t row = idx ? min(max(idx[b], 0), n_rows - 1) : b;
        x16[e] = to_bf16(x[row * in + i]);
    } else if (e < nx + nt) {
        const int64_t f = e - nx;
        const int b = (int)(f / out), o = (int)(f % out);
        const int64_t row = idx ? min(max(idx[b], 0), n_rows - 1) : b;
        t32[f] = t[row * out + o];
    }
}

// g = 2 (y - t) / (N K), its bfloat16 copy, and per-block partial sums of (y - t)^2
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                        int64_t n, float inv_n, float* __restrict__ g32,
                                                        uint16_t* __restrict__ g16, double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const float d = y[e] - t[e];
        const float gg = 2.0f * d * inv_n;
        g32[e] = gg;
        g16[e] = to_bf16(gg);
        acc += (double)d * (double)d;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one workgroup adds the per-block partial sums (tree order fixed: deterministic)
__global__ __launch_bounds__(256) void loss_finish_kernel(const double* __restrict__ partial, int32_t nblk, double inv_n,
                                                          float* __restrict__ loss) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += partial[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *loss = (float)((red[0] + red[1] + red[2] + red[3]) * inv_n);
}

// db[o] = sum_b g[b][o]: 64 columns per workgroup, 16 row lanes each summing a
// strided subset, then the 16 partial sums added in lane order (deterministic)
// The end of a layer's weight gradient, one launch: blocks [0, nr) add the
// split-K slices (out[e] = sum_s part[s][e], slices in order; nr = 0 without
// split-K) and blocks [nr, nr + ceil(O / 8)) the bias gradient's column sums
// db[o] = sum_b g[b][o], 8 columns per block: thread (r, c) sums rows r, r +
// 32, ... of column c, then one thread per column adds the 32 partials in
// order (fixed order throughout: bit-reproducible).
__global__ __launch_bounds__(256) void wgrad_finish_kernel(const float* __restrict__ part, int32_t S, int64_t mn,
                                                           float* __restrict__ out, int32_t nr,
                                                           const float* __restrict__ g, int32_t N, int32_t O,
                                                           float* __restrict__ db) {
    __shared__ float cs[32][9];
    if ((int)blockIdx.x < nr) {
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mn; e += (int64_t)nr * 256) {
            float sum = 0.0f;
            for (int i = 0; i < S; ++i) sum += part[(int64_t)i * mn + e];
            out[e] = sum;
        }
        return;
    }
    const int c = threadIdx.x & 7, r = threadIdx.x >> 3;
    const int o = ((int)blockIdx.x - nr) * 8 + c;
    float sum = 0.0f;
    if (o < O) {
#pragma unroll 8
        for (int b = r; b < N; b += 32) sum += g[(int64_t)b * O + o];
    }
    cs[r][c] = sum;
    __syncthreads();
    if (threadIdx.x < 8 && o < O) {
        float t = 0.0f;
        for (int i = 0; i < 32; ++i) t += cs[i][c];
        db[o] = t;
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ gr,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   uint16_t* __restrict__ p16, int64_t n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const float g = gr[e];
        const float mm = b1 * m[e] + (1.0f - b1) * g;
        const float vv = b2 * v[e] + (1.0f - b2) * g * g;
        m[e] = mm;
        v[e] = vv;
        const float np = p[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        p[e] = np;
        p16[e] = to_bf16(np);
    }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ p, int64_t n, uint16_t* __restrict__ q) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) q[e] = to_bf16(p[e]);
}

// x[b][j] = 2 (p[b][j] - lo_j) / (hi_j - lo_j) - 1
struct FeatRange {
    double lo[4], hi[4];
};
__global__ __launch_bounds__(256) void features_kernel(const double* __restrict__ params, int32_t N, const FeatRange r,
                                                       float* __restrict__ x) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)N * 4) return;
    const int j = (int)(e & 3);
    x[e] = (float)(2.0 * (params[e] - r.lo[j]) / (r.hi[j] - r.lo[j]) - 1.0);
}

// sums of (a - b)^2 and b^2 in float64 (atomics: order-free, used for error reports only)
__global__ __launch_bounds__(256) void sq_norms_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                       int64_t n, double* __restrict__ out) {
    __shared__ double red[2][4];
    double d2 = 0.0, b2 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const double d = (double)a[e] - (double)b[e];
        d2 += d * d;
        b2 += (double)b[e] * (double)b[e];
    }
    for (int off = 32; off > 0; off >>= 1) {
        d2 += __shfl_down(d2, off, 64);
        b2 += __shfl_down(b2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = d2;
        red[1][threadIdx.x >> 6] = b2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(out, red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        unsafeAtomicAdd(out + 1, red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    }
}

__global__ void zero2_kernel(double* p) {
    if (threadIdx.x < 2) p[threadIdx.x] = 0.0;
}

// ---------------------------------------------------------------- layout ----
struct MlpLayout {
    int32_t w[5];
    int64_t off_w[4], off_b[4];
    int64_t P;
};

static bool make_layout(const int32_t* widths, MlpLayout& L) {
    if (!widths) return false;
    int64_t off = 0;
    for (int i = 0; i < 5; ++i) {
        if (widths[i] < 1 || widths[i] > 65536) return false;
        L.w[i] = widths[i];
    }
    for (int l = 0; l < 4; ++l) {
        L.off_w[l] = off;
        off += (int64_t)L.w[l + 1] * L.w[l];
        L.off_b[l] = off;
        off += L.w[l + 1];
    }
    L.P = off;
    return true;
}

// Workspace carve-up for a batch of N rows (all offsets 256-byte aligned).
struct MlpWork {
    uint16_t* x16;
    float* z[3];
    uint16_t* h16[3];
    float* y;
    float* t;
    float* g32[4];
    uint16_t* g16[4];
    double* partial;
    float* splitk;  // split-K partial products of the weight gradients
    size_t bytes;
};

constexpr int LOSS_BLOCKS = 256;

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// weight-gradient products run over the batch: one k-slice per 256 rows (at most 8)
static int wgrad_splits(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>(8, N / 256)); }

static MlpWork carve(const MlpLayout& L, int64_t N, void* base) {
    MlpWork w{};
    char* p = (char*)base;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* q = p ? (void*)(p + off) : nullptr;
        off += align256(bytes);
        return q;
    };
    w.x16 = (uint16_t*)take(2 * N * L.w[0]);
    for (int l = 0; l < 3; ++l) {
        w.z[l] = (float*)take(4 * N * L.w[l + 1]);
        w.h16[l] = (uint16_t*)take(2 * N * L.w[l + 1]);
    }
    w.y = (float*)take(4 * N * L.w[4]);
    w.t = (float*)take(4 * N * L.w[4]);
    for (int l = 0; l < 4; ++l) {
        w.g32[l] = (float*)take(4 * N * L.w[l + 1]);
        w.g16[l] = (uint16_t*)take(2 * N * L.w[l + 1]);
    }
    w.partial = (double*)take(8 * LOSS_BLOCKS);
    int64_t mn = 0;
    for (int l = 0; l < 4; ++l) mn = std::max<int64_t>(mn, (int64_t)L.w[l] * L.w[l + 1]);
    w.splitk = (float*)take(4 * (size_t)wgrad_splits(N) * mn);
    w.bytes = off;
    return w;
}

// forward through the four layers; rows of x (and t) gathered through idx
static void forward(const MlpLayout& L, const uint16_t* p16, const float* p32, const float* x, const float* t,
                    const int32_t* idx, int32_t n_rows, int32_t N, const float* scale, const MlpWork& w,
                    float* y_out, hipStream_t s) {
    const int64_t ng = (int64_t)N * L.w[0] + (t ? (int64_t)N * L.w[4] : 0);
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, x, L.w[0], t, L.w[4], idx,
                       n_rows, N, w.x16, w.t);
    const uint16_t* in = w.x16;
    for (int l = 0; l < 4; ++l) {
        GemmArgs g{};
        g.A = in;
        g.sam = L.w[l];
        g.sak = 1;
        g.B = p16 + L.off_w[l];  // B(k, n) = W[n][k]
        g.sbk = 1;
        g.sbn = L.w[l];
        g.M = N;
        g.N = L.w[l + 1];
        g.K = L.w[l];
        g.bias = p32 + L.off_b[l];
        if (l < 3) {
            g.c32 = w.z[l];
            g.ldc = L.w[l + 1];
            g.c16 = w.h16[l];
            g.ldc16 = L.w[l + 1];
            gemm(EPI_BIAS_GELU, g, s);
            in = w.h16[l];
        } else {
            g.c32 = y_out;
            g.ldc = L.w[4];
            g.scale = scale;
            gemm(EPI_BIAS_SCALE, g, s);
        }
    }
}

}  // namespace tidas

using namespace tidas;

extern "C" int64_t tidas_mlp_param_count(const int32_t* widths) {
    MlpLayout L;
    return make_layout(widths, L) ? L.P : -1;
}

extern "C" size_t tidas_mlp_workspace_bytes(const int32_t* widths, int32_t N) {
    MlpLayout L;
    if (!make_layout(widths, L) || N < 1) return 0;
    return carve(L, N, nullptr).bytes;
}

static int32_t mlp_common(const char* name, const int32_t* widths, int32_t N, void* work, size_t work_bytes,
                          MlpLayout& L) {
    if (!make_layout(widths, L)) return fail(TIDAS_EINVAL, std::string(name) + ": widths must be 5 values in [1, 65536]");
    if (N < 1) return fail(TIDAS_EINVAL, std::string(name) + ": N must be >= 1");
    if (!work || work_bytes < carve(L, N, nullptr).bytes)
        return fail(TIDAS_EINVAL, std::string(name) + ": workspace missing or too small");
    if ((reinterpret_cast<uintptr_t>(work) & 255) != 0)
        return fail(TIDAS_EINVAL, std::string(name) + ": workspace must be 256-byte aligned");
    if (N > (1 << 22)) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": batch too large");
    // the GEMMs address their bfloat16 operands with 32-bit byte offsets
    int64_t widest = 1;
    for (int i = 0; i < 5; ++i) widest = std::max<int64_t>(widest, L.w[i]);
    if ((int64_t)N * widest * 2 >= ((int64_t)1 << 31) || widest * widest * 2 >= ((int64_t)1 << 31))
        return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": operands beyond 2 GiB");
    return TIDAS_OK;
}

extern "C" int32_t tidas_mlp_forward(const int32_t* widths, const uint16_t* params16, const float* params,
                                     const float* x, int32_t N, const float* scale, float* y, void* work,
                                     size_t work_bytes, void* stream) {
    MlpLayout L;
    int32_t st = mlp_common("tidas_mlp_forward", widths, N, work, work_bytes, L);
    if (st) return st;
    if (!params16 || !params || !x || !y) return fail(TIDAS_EINVAL, "tidas_mlp_forward: null pointer");
    const MlpWork w = carve(L, N, work);
    forward(L, params16, params, x, nullptr, nullptr, N, N, scale, w, y, (hipStream_t)stream);
    return check_launch("tidas_mlp_forward");
}

extern "C" int32_t tidas_mlp_train_step(const int32_t* widths, const uint16_t* params16, const float* params,
                                        const float* x, const float* target, int32_t n_rows, const int32_t* idx,
                                        int32_t N, float* grad, float* loss, void* work, size_t work_bytes,
                                        void* stream) {
    MlpLayout L;
    int32_t st = mlp_common("tidas_mlp_train_step", widths, N, work, work_bytes, L);
    if (st) return st;
    if (!params16 || !params || !x || !target || !grad || !loss)
        return fail(TIDAS_EINVAL, "tidas_mlp_train_step: null pointer");
    if (n_rows < 1 || (!idx && n_rows < N))
        return fail(TIDAS_EINVAL, "tidas_mlp_train_step: n_rows must be >= 1 (and >= N without idx)");
    hipStream_t s = (hipStream_t)stream;
    const MlpWork w = carve(L, N, work);
    forward(L, params16, params, x, target, idx, n_rows, N, nullptr, w, w.y, s);
    const int64_t ny = (int64_t)N * L.w[4];
    hipLaunchKernelGGL(loss_grad_kernel, dim3(LOSS_BLOCKS), dim3(256), 0, s, w.y, w.t, ny, (float)(1.0 / (double)ny),
                       w.g32[3], w.g16[3], w.partial);
    hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(256), 0, s, w.partial, LOSS_BLOCKS, 1.0 / (double)ny, loss);
    for (int l = 3; l >= 0; --l) {
        const uint16_t* h_in = (l == 0) ? w.x16 : w.h16[l - 1];
        const int in = L.w[l], out = L.w[l + 1];
        // dW_l[o][i] = sum_b g_l[b][o] h_in[b][i]
        GemmArgs gw{};
        gw.A = w.g16[l];
        gw.sam = 1;
        gw.sak = out;
        gw.B = h_in;
        gw.sbk = in;
        gw.sbn = 1;
        gw.M = out;
        gw.N = in;
        gw.K = N;
        gw.ldc = in;
        const int S = wgrad_splits(N);
        const int64_t mn = (int64_t)out * in;
        int nr = 0;
        if (S > 1) {
            gw.c32 = w.splitk;
            gemm(EPI_STORE, gw, s, S);
            nr = (int)std::min<int64_t>((mn + 255) / 256, 1024);
        } else {
            gw.c32 = grad + L.off_w[l];
            gemm(EPI_STORE, gw, s);
        }
        hipLaunchKernelGGL(wgrad_finish_kernel, dim3((unsigned)(nr + (out + 7) / 8)), dim3(256), 0, s, w.splitk, S, mn,
                           grad + L.off_w[l], nr, w.g32[l], N, out, grad + L.off_b[l]);
        if (l > 0) {
            // g_{l-1}[b][i] = (sum_o g_l[b][o] W_l[o][i]) * GELU'(z_{l-1}[b][i])
            GemmArgs gd{};
            gd.A = w.g16[l];
            gd.sam = out;
            gd.sak = 1;
            gd.B = params16 + L.off_w[l];
            gd.sbk = in;
            gd.sbn = 1;
            gd.M = N;
            gd.N = in;
            gd.K = out;
            gd.c32 = w.g32[l - 1];
            gd.ldc = in;
            gd.c16 = w.g16[l - 1];
            gd.ldc16 = in;
            gd.zin = w.z[l - 1];
            gd.ldz = in;
            gemm(EPI_GELU_GRAD, gd, s);
        }
    }
    return check_launch("tidas_mlp_train_step");
}

extern "C" int32_t tidas_mlp_adam(const int32_t* widths, float* params, const float* grad, float* m, float* v,
                                  uint16_t* params16, float lr, float beta1, float beta2, float eps, int32_t step,
                                  void* stream) {
    MlpLayout L;
    if (!make_layout(widths, L)) return fail(TIDAS_EINVAL, "tidas_mlp_adam: bad widths");
    if (!params || !grad || !m || !v || !params16) return fail(TIDAS_EINVAL, "tidas_mlp_adam: null pointer");
    if (step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(TIDAS_EINVAL, "tidas_mlp_adam: need step >= 1, lr >= 0, betas in [0, 1), eps > 0");
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    const unsigned nb = (unsigned)std::min<int64_t>((L.P + 255) / 256, 4096);
    hipLaunchKernelGGL(adam_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, params16, L.P, lr,
                       beta1, beta2, eps, c1, c2);
    return check_launch("tidas_mlp_adam");
}

extern "C" int32_t tidas_mlp_to_bf16(const float* params, int64_t n, uint16_t* params16, void* stream) {
    if (!params || !params16 || n < 0) return fail(TIDAS_EINVAL, "tidas_mlp_to_bf16: bad arguments");
    if (n == 0) return TIDAS_OK;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, params, n, params16);
    return check_launch("tidas_mlp_to_bf16");
}

extern "C" int32_t tidas_mlp_features(const double* params, int32_t N, const double* lo, const double* hi, float* x,
                                      void* stream) {
    if (!params || !lo || !hi || !x || N < 1) return fail(TIDAS_EINVAL, "tidas_mlp_features: bad arguments");
    FeatRange r;
    for (int j = 0; j < 4; ++j) {
        if (!(hi[j] > lo[j]) || !std::isfinite(lo[j]) || !std::isfinite(hi[j]))
            return fail(TIDAS_EINVAL, "tidas_mlp_features: need finite lo < hi");
        r.lo[j] = lo[j];
        r.hi[j] = hi[j];
    }
    const int64_t n = (int64_t)N * 4;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, params, N,
                       r, x);
    return check_launch("tidas_mlp_features");
}

extern "C" int32_t tidas_sq_norms(const float* a, const float* b, int64_t n, double* work, double* out,
                                  void* stream) {
    if (!a || !b || !work || !out || n < 0) return fail(TIDAS_EINVAL, "tidas_sq_norms: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(64), 0, s, work);
    if (n > 0) {
        const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
        hipLaunchKernelGGL(sq_norms_kernel, dim3(nb), dim3(256), 0, s, a, b, n, work);
    }
    int32_t st = check_launch("tidas_sq_norms");
    if (!st) st = check_hip(hipMemcpyAsync(out, work, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "tidas_sq_norms");
    if (!st) st = check_hip(hipStreamSynchronize(s), "tidas_sq_norms: synchronize");
    return st;
}
