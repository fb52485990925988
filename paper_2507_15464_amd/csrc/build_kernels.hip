// Per-depth-row kernel banks of the line model, derived from DAS, and the
// Born RF synthesis that feeds the path.  All arithmetic here is float64:
// these run once per geometry (or once per phantom), not per frame.
//
// Exact mode (Sec. 2.2, eq:PSF): K[i][m+h] = DAS, at pixel (0, z_i + m dz), of
// the echo of a unit scatterer at (0, z_i).  The echo is evaluated
// analytically where DAS reads it: RF1[a][n][k] = p(t0 + k/fs - tau_n) for
// 0 <= k < T, zero outside the record.
//
// Lateral mode (the separable 2-D extension; the conclusion, Sec. 4, leaves a
// 2-D model for future work): Kx[i][m+h] = DAS, at pixel (m dx, z_i), of the
// same unit echo, divided by its value at (0, z_i): the lateral profile of row
// i's PSF through the scatterer, for tidas_apply_lateral.
//
// Paper mode (Sec. 2.3 eqn:tDAS / eqn:theta; Sec. 3.1-3.2): receive delays and
// apodization frozen at a reference depth z_r; the kernel is the fixed-delay
// response h_r scaled by the least-squares weight theta_i fitted inside a
// window as wide as the FWHM of the DAS PSF envelope at z_r.  Two launches:
//   paper_ref_kernel  one workgroup per distinct reference row: h_r, the PSF on
//                     a fine axis, its envelope by a direct DFT (analytic
//                     signal), and the FWHM;
//   paper_row_kernel  one workgroup per row: a_i and b_i on the window, the
//                     two dot products, theta_i, and the scaled kernel row.
//
// Line mode (Sec. 2.4, eqn:line_conv read literally: Theta times the
// fixed-delay beamformer of the RF): same theta_i and reference rows as paper
// mode, but tap m of row i is theta_i times the fixed-delay response, read at
// z_i, of a unit scatterer at the source row's depth z_i - m dz (Born
// linearity turns the RF-domain model into this gather on the reflectivity).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "envelope.hpp"

namespace tidas {

constexpr int BK_MAX_ANGLES = 32;

struct Setup64 {
    int32_t C, T, A;
    double pitch, c, fs, t0, fc, sigma, fnumber, x_first;
    double sin_a[BK_MAX_ANGLES];
    double cos_a[BK_MAX_ANGLES];
};

__device__ __forceinline__ double pulse_d(double t, double fc, double sigma) {
    if (fabs(t) > 4.0 * sigma) return 0.0;
    return exp(-t * t / (2.0 * sigma * sigma)) * cospi(2.0 * fc * t);
}

__device__ __forceinline__ double hann_d(double d, double z, double F) {
    const double a = z / (2.0 * F);
    if (!(a > 0.0) || fabs(d) > a) return 0.0;
    return 0.5 * (1.0 + cospi(d / a));
}

// Linear-interpolation read at fractional index u of the unit echo whose
// arrival time is tau.
__device__ __forceinline__ double unit_echo_read(const Setup64& s, double u, double tau) {
    const double q = floor(u);
    const double f = u - q;
    double s0 = 0.0, s1 = 0.0;
    if (q >= 0.0 && q < (double)s.T) s0 = pulse_d(s.t0 + q / s.fs - tau, s.fc, s.sigma);
    if (q + 1.0 >= 0.0 && q + 1.0 < (double)s.T) s1 = pulse_d(s.t0 + (q + 1.0) / s.fs - tau, s.fc, s.sigma);
    return (1.0 - f) * s0 + f * s1;
}

__device__ __forceinline__ double arrival(const Setup64& s, int a, double x, double z, double xn) {
    const double dx = x - xn;
    return (x * s.sin_a[a] + z * s.cos_a[a]) / s.c + sqrt(dx * dx + z * z) / s.c;
}

// DAS at pixel (x, z) of a unit scatterer at (0, zs).
__device__ double unit_das(const Setup64& s, double x, double z, double zs) {
    double acc = 0.0;
    for (int a = 0; a < s.A; ++a) {
        for (int n = 0; n < s.C; ++n) {
            const double xn = s.x_first + (double)n * s.pitch;
            const double w = hann_d(x - xn, z, s.fnumber);
            if (w == 0.0) continue;
            const double u = (arrival(s, a, x, z, xn) - s.t0) * s.fs;
            acc += w * unit_echo_read(s, u, arrival(s, a, 0.0, zs, xn));
        }
    }
    return acc;
}

// Fixed-delay line F_r[unit echo at zs](z): delays and weights of depth zr.
__device__ double fixed_delay(const Setup64& s, double z, double zr, double zs) {
    double acc = 0.0;
    for (int a = 0; a < s.A; ++a) {
        const double t_centre = z * s.cos_a[a] / s.c + z / s.c;
        for (int n = 0; n < s.C; ++n) {
            const double xn = s.x_first + (double)n * s.pitch;
            const double w = hann_d(-xn, zr, s.fnumber);
            if (w == 0.0) continue;
            const double D = (zr - sqrt(xn * xn + zr * zr)) / s.c;  // eqn:delay
            const double u = (t_centre - D - s.t0) * s.fs;
            acc += w * unit_echo_read(s, u, arrival(s, a, 0.0, zs, xn));
        }
    }
    return acc;
}

// ------------------------------------------------------------ exact mode ----
__global__ __launch_bounds__(256) void exact_kernel(const Setup64 s, int32_t Z, int32_t K, double z0, double dz,
                                                    float* __restrict__ kb, float* __restrict__ theta) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)Z * K) return;
    const int i = (int)(idx / K);
    const int t = (int)(idx % K);
    const int h = (K - 1) / 2;
    const double zi = z0 + (double)i * dz;
    kb[idx] = (float)unit_das(s, 0.0, zi + (double)(t - h) * dz, zi);
    if (theta && t == 0) theta[i] = 1.0f;
}

// ---------------------------------------------------------- lateral mode ----
// Row i's lateral kernel: the DAS response of the unit scatterer at (0, z_i)
// along its own row, divided by its value at the scatterer (0 if that is 0).
__global__ __launch_bounds__(256) void lateral_kernel(const Setup64 s, int32_t Z, int32_t K, double z0, double dz,
                                                      double dx, float* __restrict__ kb, float* __restrict__ theta) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)Z * K) return;
    const int i = (int)(idx / K);
    const int t = (int)(idx % K);
    const int h = (K - 1) / 2;
    const double zi = z0 + (double)i * dz;
    const double centre = unit_das(s, 0.0, zi, zi);
    kb[idx] = centre != 0.0 ? (float)(unit_das(s, (double)(t - h) * dx, zi, zi) / centre) : 0.0f;
    if (theta && t == 0) theta[i] = 1.0f;
}

// ------------------------------------------------------------ paper mode ----
constexpr int PAPER_THREADS = 256;
constexpr int FINE_MAX = ENV_MAX;  // max fine-axis length 2 Qf + 1 (DFT length <= 2 FINE_MAX)

__device__ double block_sum(double v, double* red) {
    // wave reduction then LDS across the 4 waves
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < PAPER_THREADS / 64; ++w) tot += red[w];
        red[0] = tot;
    }
    __syncthreads();
    tot = red[0];
    __syncthreads();
    return tot;
}

// One workgroup per distinct reference row.  Outputs h_ref[u][K] and
// width[u] (metres).
__global__ __launch_bounds__(PAPER_THREADS) void paper_ref_kernel(const Setup64 s, int32_t K, double z0, double dz,
                                                                  int32_t Qf, const int32_t* __restrict__ refs,
                                                                  double* __restrict__ h_ref,
                                                                  double* __restrict__ width) {
    __shared__ double b[FINE_MAX];
    __shared__ double env[FINE_MAX];
    __shared__ double Xr[FINE_MAX + 1];  // bins 0 .. N/2, N <= 2 FINE_MAX
    __shared__ double Xi[FINE_MAX + 1];
    __shared__ double tc[2 * FINE_MAX];  // twiddles of the DFT length N <= 2 FINE_MAX
    __shared__ double ts[2 * FINE_MAX];
    const int u = blockIdx.x;
    const int r = refs[u];
    const double zr = z0 + (double)r * dz;
    const int h = (K - 1) / 2;
    const double dzf = s.c / (2.0 * s.fs);
    const int L = 2 * Qf + 1;

    for (int t = threadIdx.x; t < K; t += PAPER_THREADS)
        h_ref[(size_t)u * K + t] = fixed_delay(s, zr + (double)(t - h) * dz, zr, zr);
    for (int q = threadIdx.x; q < L; q += PAPER_THREADS) b[q] = unit_das(s, 0.0, zr + (double)(q - Qf) * dzf, zr);
    __syncthreads();
    block_envelope<PAPER_THREADS>(b, L, env, Xr, Xi, tc, ts);
    if (threadIdx.x == 0) width[u] = env_fwhm(env, L) * dzf;
}

// One workgroup per row i.
__global__ __launch_bounds__(PAPER_THREADS) void paper_row_kernel(const Setup64 s, int32_t K, double z0, double dz,
                                                                  const int32_t* __restrict__ ref_of_row,
                                                                  const int32_t* __restrict__ refs,
                                                                  const double* __restrict__ h_ref,
                                                                  const double* __restrict__ width, int32_t line,
                                                                  float* __restrict__ kb, float* __restrict__ theta) {
    __shared__ double red[PAPER_THREADS / 64];
    const int i = blockIdx.x;
    const int u = ref_of_row[i];
    const double zr = z0 + (double)refs[u] * dz;
    const double zi = z0 + (double)i * dz;
    const double dzf = s.c / (2.0 * s.fs);
    // width <= 2 Qf dzf by construction; the clamp only guards non-finite input
    const double wq = 0.5 * width[u] / dzf;
    const int qmax = (wq >= 0.0 && wq <= (double)FINE_MAX) ? (int)floor(wq) : 0;
    double ab = 0.0, aa = 0.0;
    for (int q = -qmax + (int)threadIdx.x; q <= qmax; q += PAPER_THREADS) {
        const double z = zi + (double)q * dzf;
        const double a = fixed_delay(s, z, zr, zi);
        const double bb = unit_das(s, 0.0, z, zi);
        ab += a * bb;
        aa += a * a;
    }
    ab = block_sum(ab, red);
    aa = block_sum(aa, red);
    const double th = (aa > 0.0) ? ab / aa : 0.0;
    const int h = (K - 1) / 2;
    for (int t = threadIdx.x; t < K; t += PAPER_THREADS) {
        const double k = line ? fixed_delay(s, zi, zr, zi - (double)(t - h) * dz) : h_ref[(size_t)u * K + t];
        kb[(size_t)i * K + t] = (float)(th * k);
    }
    if (theta && threadIdx.x == 0) theta[i] = (float)th;
}

// ------------------------------------------------------------ RF synthesis ----
// Order-independent accumulation: every contribution amp * p(t) is rounded
// once to a fixed-point integer with 2^e units per unit of amplitude and the
// integers are summed with 64-bit integer atomics.  Integer addition is exact
// and associative, so the sum (and the float32 record) does not depend on the
// order in which threads add.  e is the largest exponent with
// n_scat * max|amp| * 2^e < 2^61 (no sum can overflow, since |p| <= 1), so
// each contribution carries an absolute error below 2^-(e+1): relative to the
// largest possible sample, under n_scat * 2^-62.
__global__ __launch_bounds__(256) void amp_scale_kernel(const double* __restrict__ scat, int32_t S,
                                                        double* __restrict__ scale) {
    __shared__ double red[4];
    double m = 0.0;
    for (int i = threadIdx.x; i < S; i += 256) m = fmax(m, fabs(scat[3 * (int64_t)i + 2]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double top = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * (double)max(S, 1);
        // 2^e with top * 2^e < 2^61; amplitudes of 0 (or none): any scale
        int e = 0;
        if (top > 0.0 && isfinite(top)) e = 60 - ilogb(top);
        scale[0] = ldexp(1.0, max(min(e, 1000), -1000));
    }
}

__global__ __launch_bounds__(256) void simulate_kernel(const Setup64 s, const double* __restrict__ scat, int32_t S,
                                                       int32_t width, const double* __restrict__ scale,
                                                       unsigned long long* __restrict__ acc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;  // over (a, n, scatterer)
    const int64_t total = (int64_t)s.A * s.C * S;
    if (idx >= total) return;
    const int sc = (int)(idx % S);
    const int n = (int)((idx / S) % s.C);
    const int a = (int)(idx / ((int64_t)S * s.C));
    const double x = scat[3 * (int64_t)sc], z = scat[3 * (int64_t)sc + 1], amp = scat[3 * (int64_t)sc + 2];
    const double xn = s.x_first + (double)n * s.pitch;
    const double tau = arrival(s, a, x, z, xn);
    const double half = 4.0 * s.sigma;
    const double sc_amp = amp * scale[0];
    const int64_t k_lo = (int64_t)ceil((tau - half - s.t0) * s.fs);
    unsigned long long* row = acc + ((int64_t)a * s.C + n) * s.T;
    for (int w = 0; w < width; ++w) {
        const int64_t k = k_lo + w;
        if (k < 0 || k >= s.T) continue;
        const long long v = __double2ll_rn(sc_amp * pulse_d(s.t0 + (double)k / s.fs - tau, s.fc, s.sigma));
        // two's complement: adding the bit pattern of a negative value modulo
        // 2^64 is adding the value
        if (v != 0) atomicAdd(row + k, (unsigned long long)v);
    }
}

__global__ __launch_bounds__(256) void round_kernel(const unsigned long long* __restrict__ acc, int64_t n,
                                                    const double* __restrict__ scale, float* __restrict__ rf) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) rf[idx] = (float)((double)(long long)acc[idx] / scale[0]);
}

__global__ __launch_bounds__(256) void zero_kernel(double* __restrict__ p, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx < n) p[idx] = 0.0;
}

// ------------------------------------------------------- per-row draws ----
// Exact-mode kernels for independent rows, each with its own depth, F-number,
// plane-wave angle and centre frequency (single angle per row); the training
// data and error judge of the kernel surrogate.
struct RowDrawArgs {
    int32_t C, T, K;
    double pitch, c, fs, t0, cycles, dz, x_first;
};

__device__ double unit_das_row(const RowDrawArgs& e, double z, double zs, double fnumber, double sa, double ca,
                               double fc, double sigma) {
    double acc = 0.0;
    for (int n = 0; n < e.C; ++n) {
        const double xn = e.x_first + (double)n * e.pitch;
        const double w = hann_d(-xn, z, fnumber);
        if (w == 0.0) continue;
        const double u = ((z * ca) / e.c + sqrt(xn * xn + z * z) / e.c - e.t0) * e.fs;
        const double tau = (zs * ca) / e.c + sqrt(xn * xn + zs * zs) / e.c;
        const double q = floor(u);
        const double f = u - q;
        double s0 = 0.0, s1 = 0.0;
        if (q >= 0.0 && q < (double)e.T) s0 = pulse_d(e.t0 + q / e.fs - tau, fc, sigma);
        if (q + 1.0 >= 0.0 && q + 1.0 < (double)e.T) s1 = pulse_d(e.t0 + (q + 1.0) / e.fs - tau, fc, sigma);
        acc += w * ((1.0 - f) * s0 + f * s1);
    }
    return acc;
}

__global__ __launch_bounds__(256) void kernels_at_kernel(const RowDrawArgs e, const double* __restrict__ params,
                                                         int32_t N, int32_t normalise, float* __restrict__ out,
                                                         float* __restrict__ scale) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)N * e.K) return;
    const int i = (int)(idx / e.K);
    const int t = (int)(idx % e.K);
    const int h = (e.K - 1) / 2;
    const double z = params[4 * (int64_t)i], F = params[4 * (int64_t)i + 1];
    const double alpha = params[4 * (int64_t)i + 2], fc = params[4 * (int64_t)i + 3];
    const double sigma = (e.cycles / fc) / (2.0 * sqrt(2.0 * log(2.0)));
    double sa, ca;
    sincos(alpha, &sa, &ca);
    double sw = 1.0;
    if (normalise || (scale && t == 0)) {
        sw = 0.0;
        for (int n = 0; n < e.C; ++n) sw += hann_d(-(e.x_first + (double)n * e.pitch), z, F);
        sw = fmax(sw, 1.0);
    }
    const double v = unit_das_row(e, z + (double)(t - h) * e.dz, z, F, sa, ca, fc, sigma);
    out[idx] = (float)(normalise ? v / sw : v);
    if (scale && t == 0) scale[i] = (float)sw;
}

static int32_t fill_setup(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx, int32_t T, Setup64& s) {
    if (tx->n_angles > BK_MAX_ANGLES) return fail(TIDAS_EUNSUPPORTED, "at most 32 plane-wave angles");
    s.C = array->n_elem;
    s.T = T;
    s.A = tx->n_angles;
    s.pitch = array->pitch;
    s.c = array->c;
    s.fs = tx->fs;
    s.t0 = tx->t0;
    s.fc = tx->fc;
    s.sigma = (tx->cycles / tx->fc) / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    s.fnumber = rx ? rx->fnumber : 1.0;
    s.x_first = -0.5 * (double)(s.C - 1) * s.pitch;
    for (int a = 0; a < s.A; ++a) {
        s.sin_a[a] = std::sin(tx->angles[a]);
        s.cos_a[a] = std::cos(tx->angles[a]);
    }
    return TIDAS_OK;
}

}  // namespace tidas

using namespace tidas;

// Paper and line modes: [reference responses nref x K doubles | widths nref
// doubles | row -> slot map Z ints | reference rows nref ints], sized for
// nref = Z (every row its own reference).
static size_t paper_workspace_bytes(int64_t Z, int64_t K) {
    return (size_t)(8 * Z * K + 8 * Z + 4 * Z + 4 * Z + 16);
}

extern "C" size_t tidas_build_kernels_workspace_bytes(int32_t nz, int32_t K, int32_t mode) {
    if (nz < 1 || K < 1 || (mode != TIDAS_MODE_PAPER && mode != TIDAS_MODE_LINE)) return 0;
    return paper_workspace_bytes(nz, K);
}

static void free_staging(void* p) { delete static_cast<std::vector<int32_t>*>(p); }

extern "C" int32_t tidas_build_kernels(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                                       const tidas_grid* grid, int32_t n_samples, int32_t K, int32_t mode,
                                       const int32_t* ref_row, float* kernels, float* theta, void* workspace,
                                       size_t workspace_bytes, void* stream) {
    int32_t st;
    if ((st = validate_array(array)) || (st = validate_tx(tx, true)) || (st = validate_rx(rx)) ||
        (st = validate_grid(grid)))
        return st;
    if (!kernels) return fail(TIDAS_EINVAL, "tidas_build_kernels: null kernels pointer");
    if (n_samples < 2) return fail(TIDAS_EINVAL, "tidas_build_kernels: n_samples must be >= 2");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_build_kernels: K must be odd and >= 1");
    if (mode != TIDAS_MODE_EXACT && mode != TIDAS_MODE_PAPER && mode != TIDAS_MODE_LINE && mode != TIDAS_MODE_LATERAL)
        return fail(TIDAS_EINVAL, "tidas_build_kernels: mode must be 0 (exact), 1 (paper), 2 (line) or 3 (lateral)");
    if ((void*)kernels == (void*)theta) return fail(TIDAS_EINVAL, "tidas_build_kernels: theta aliases kernels");
    const int Z = grid->nz;
    const bool paper = mode == TIDAS_MODE_PAPER || mode == TIDAS_MODE_LINE;
    if ((st = workspace_check("tidas_build_kernels", workspace, workspace_bytes,
                              paper ? paper_workspace_bytes(Z, K) : 0)))
        return st;
    if (ref_row)
        for (int i = 0; i < Z; ++i)
            if (ref_row[i] < 0 || ref_row[i] >= Z)
                return fail(TIDAS_EINVAL, "tidas_build_kernels: ref_row entries must lie in [0, nz)");
    Setup64 s;
    if ((st = fill_setup(array, tx, rx, n_samples, s))) return st;
    hipStream_t strm = (hipStream_t)stream;

    if (mode == TIDAS_MODE_EXACT) {
        const int64_t n = (int64_t)Z * K;
        hipLaunchKernelGGL(exact_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, strm, s, Z, K, grid->z0,
                           grid->dz, kernels, theta);
        return check_launch("tidas_build_kernels(exact)");
    }
    if (mode == TIDAS_MODE_LATERAL) {
        const int64_t n = (int64_t)Z * K;
        hipLaunchKernelGGL(lateral_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, strm, s, Z, K, grid->z0,
                           grid->dz, grid->dx, kernels, theta);
        return check_launch("tidas_build_kernels(lateral)");
    }

    // paper and line modes: distinct reference rows and the row -> reference map
    const int Qf = (int)std::ceil(8.0 * s.sigma * s.fs);
    if (2 * Qf + 1 > FINE_MAX) return fail(TIDAS_EUNSUPPORTED, "tidas_build_kernels: pulse too long for the fine axis");
    std::vector<int32_t> refs;
    std::vector<int32_t> map(Z);
    {
        std::vector<int32_t> slot(Z, -1);
        for (int i = 0; i < Z; ++i) {
            const int r = ref_row ? ref_row[i] : i;
            if (slot[r] < 0) {
                slot[r] = (int32_t)refs.size();
                refs.push_back(r);
            }
            map[i] = slot[r];
        }
    }
    const size_t nref = refs.size();
    const size_t bytes = sizeof(int32_t) * (Z + nref) + sizeof(double) * (nref * (K + 1)) + 16;
    Workspace ws;
    if ((st = workspace_acquire("tidas_build_kernels: temporary buffer", workspace, bytes, strm, ws))) return st;
    double* h_ref = (double*)ws.ptr;
    double* width = h_ref + nref * K;
    int32_t* d_map = (int32_t*)(width + nref);
    int32_t* d_refs = d_map + Z;
    // host staging of the map, released by a host function queued after the
    // copy (the call does not wait for the stream)
    auto* host_ints = new std::vector<int32_t>(map);
    host_ints->insert(host_ints->end(), refs.begin(), refs.end());
    st = check_hip(hipMemcpyAsync(d_map, host_ints->data(), sizeof(int32_t) * host_ints->size(), hipMemcpyHostToDevice,
                                  strm),
                   "tidas_build_kernels: upload");
    if (check_hip(hipLaunchHostFunc(strm, free_staging, host_ints), "tidas_build_kernels: staging release")) {
        // the host function could not be queued: wait for the copy instead
        const hipError_t e = hipStreamSynchronize(strm);
        delete host_ints;
        if (!st) st = check_hip(e, "tidas_build_kernels: synchronize");
    }
    if (!st) {
        hipLaunchKernelGGL(paper_ref_kernel, dim3((unsigned)nref), dim3(PAPER_THREADS), 0, strm, s, K, grid->z0,
                           grid->dz, Qf, d_refs, h_ref, width);
        st = check_launch("tidas_build_kernels(paper, reference rows)");
    }
    if (!st) {
        hipLaunchKernelGGL(paper_row_kernel, dim3((unsigned)Z), dim3(PAPER_THREADS), 0, strm, s, K, grid->z0, grid->dz,
                           d_map, d_refs, h_ref, width, (int32_t)(mode == TIDAS_MODE_LINE), kernels, theta);
        st = check_launch("tidas_build_kernels(paper, rows)");
    }
    const int32_t st2 = workspace_release("tidas_build_kernels: free", ws, strm);
    return st ? st : st2;
}

extern "C" size_t tidas_simulate_rf_workspace_bytes(int32_t n_angles, int32_t n_elem, int32_t n_samples) {
    if (n_angles < 1 || n_elem < 1 || n_samples < 1) return 0;
    return sizeof(double) * ((size_t)n_angles * n_elem * n_samples + 1);
}

extern "C" int32_t tidas_simulate_rf(const tidas_array* array, const tidas_tx* tx, const double* scat, int32_t n_scat,
                                     int32_t n_samples, float* rf, void* workspace, size_t workspace_bytes,
                                     void* stream) {
    int32_t st;
    if ((st = validate_array(array)) || (st = validate_tx(tx, true))) return st;
    if (!rf || (n_scat > 0 && !scat)) return fail(TIDAS_EINVAL, "tidas_simulate_rf: null pointer");
    if (n_samples < 1) return fail(TIDAS_EINVAL, "tidas_simulate_rf: n_samples must be >= 1");
    if (n_scat < 0) return fail(TIDAS_EINVAL, "tidas_simulate_rf: n_scat must be >= 0");
    Setup64 s;
    if ((st = fill_setup(array, tx, nullptr, n_samples, s))) return st;
    hipStream_t strm = (hipStream_t)stream;
    const int64_t n = (int64_t)s.A * s.C * s.T;
    const size_t need = sizeof(double) * ((size_t)n + 1);
    if ((st = workspace_check("tidas_simulate_rf", workspace, workspace_bytes, need))) return st;
    // [fixed-point accumulator n x 8 bytes | scale (8 bytes)]
    Workspace ws;
    if ((st = workspace_acquire("tidas_simulate_rf: accumulator", workspace, need, strm, ws))) return st;
    void* buf = ws.ptr;
    unsigned long long* acc = (unsigned long long*)buf;
    double* scale = (double*)buf + n;
    // the all-zero bit pattern is the integer 0
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, strm, (double*)buf, n);
    st = check_launch("tidas_simulate_rf(zero)");
    if (!st) {
        hipLaunchKernelGGL(amp_scale_kernel, dim3(1), dim3(256), 0, strm, scat, n_scat, scale);
        st = check_launch("tidas_simulate_rf(scale)");
    }
    const int width = (int)std::ceil(2.0 * 4.0 * s.sigma * s.fs) + 2;
    const int64_t work = (int64_t)s.A * s.C * n_scat;
    if (!st && work > 0) {
        hipLaunchKernelGGL(simulate_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, strm, s, scat, n_scat,
                           width, scale, acc);
        st = check_launch("tidas_simulate_rf(accumulate)");
    }
    if (!st) {
        hipLaunchKernelGGL(round_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, strm, acc, n, scale, rf);
        st = check_launch("tidas_simulate_rf(round)");
    }
    const int32_t st2 = workspace_release("tidas_simulate_rf: free", ws, strm);
    return st ? st : st2;
}

extern "C" int32_t tidas_kernels_at(const tidas_array* array, double fs, double t0, double cycles, int32_t n_samples,
                                    double dz, const double* params, int32_t N, int32_t K, int32_t normalise,
                                    float* out, float* scale, void* stream) {
    int32_t st;
    if ((st = validate_array(array))) return st;
    if (!params || !out || N < 1) return fail(TIDAS_EINVAL, "tidas_kernels_at: null pointer or N < 1");
    if (K < 1 || (K % 2) == 0) return fail(TIDAS_EINVAL, "tidas_kernels_at: K must be odd and >= 1");
    if (!finite_pos(fs) || !std::isfinite(t0) || !finite_pos(cycles) || !finite_pos(dz) || n_samples < 2)
        return fail(TIDAS_EINVAL, "tidas_kernels_at: need fs, cycles, dz > 0, finite t0, n_samples >= 2");
    if ((void*)out == (void*)scale) return fail(TIDAS_EINVAL, "tidas_kernels_at: scale aliases out");
    RowDrawArgs e;
    e.C = array->n_elem;
    e.T = n_samples;
    e.K = K;
    e.pitch = array->pitch;
    e.c = array->c;
    e.fs = fs;
    e.t0 = t0;
    e.cycles = cycles;
    e.dz = dz;
    e.x_first = -0.5 * (double)(e.C - 1) * e.pitch;
    const int64_t n = (int64_t)N * K;
    hipLaunchKernelGGL(kernels_at_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, e,
                       params, N, normalise, out, scale);
    return check_launch("tidas_kernels_at");
}
