// The paper's single-point study (Sec. 3.1-3.3) on the device, float64
// throughout: it is an analysis of the approximation, run once per setting,
// and float64 keeps every weight and error at the oracle's precision.
//
// A linear probe transmits one beam focused on its axis at the depth of one
// of P axial points (Sec. 2.1: an unsteered beam focused on the axis; Sec.
// 3.1: one of the points is the transmit focus).  The n_tx centremost
// elements fire at T_m = (z_f - sqrt(x_m^2 + z_f^2)) / c so that every wave
// reaches the focus at z_f / c.  For a unit scatterer at every point s the
// echo RF_s[n][k] = sum_m p(t0 + k/fs - T_m - rho_m(z_s)/c - rho_n(z_s)/c) is
// synthesised once; on the fine axis z_s + q dzf (dzf = c / (2 fs), |q| <=
// Ql) the DAS line b_s (transmit arrival z / c, dynamic receive law) and, for
// every point r, the time-invariant line a_rs (receive delays D_n(z_r) of
// eqn:delay and the aperture of depth z_r frozen: read time 2 z / c - D_n(z_r))
// give
//   Theta[r][s]      = sum_B a b / sum_B a^2                (eqn:theta, line 1)
//   err_local[r][s]  = ||Theta a - b||^2_B / ||b||^2_B      (window B: |q| <= W / (2 dzf))
//   err_global[r][s] = ||Theta a - b||^2 / ||b||^2          (the whole line)
// with W the FWHM of the envelope of the focal point's DAS line (Sec. 3.1-3.2,
// measured as for the paper-mode kernels on |q| <= Qf = ceil(8 sigma fs)).
//
// Kernels, in launch order:
//   study_echo_kernel    echoes RF_s [P][C][T] and each one's sample support
//   study_das_kernel     DAS lines b_s [P][2 Ql + 1]
//   study_window_kernel  W and the window half length Qw (one workgroup)
//   study_pair_kernel    a_rs for four delay curves r per workgroup and one s,
//                        the six sums over B and over the line, then Theta and
//                        both errors
//   study_stats_kernel   per s: DAS and Theta-scaled time-invariant line of the
//                        focal point's curve on |q| <= Qh, envelope peaks and
//                        FWHMs (Sec. 3.2)
#include <algorithm>

#include "common.hpp"
#include "envelope.hpp"

namespace tidas {

TIDAS_DEBUG_FLAGS_DEFINE(study)
namespace {

constexpr int ST_THREADS = 256;
constexpr int ST_RB = 4;          // delay curves per pair workgroup
constexpr int ST_ECHO_PER_THREAD = 4;  // echo samples per thread (the arrival table and receive path shared)
constexpr int ST_MAX_ELEM = 512;  // pair-kernel LDS: ST_RB x C x 20 + C x 8 bytes (45 KB at 512) + 8 KB of lists

struct StudyGeom {
    int32_t C, T, P, n_tx, Ql, Qh, Qf, focal;
    double pitch, c, fs, t0, fc, sigma, fnumber, x_first, z_first, z_step, dzf;
};

__device__ __forceinline__ double st_pulse(double t, double fc, double sigma) {
    if (fabs(t) > 4.0 * sigma) return 0.0;
    return exp(-t * t / (2.0 * sigma * sigma)) * cospi(2.0 * fc * t);
}

__device__ __forceinline__ double st_hann(double d, double z, double F) {
    const double a = z / (2.0 * F);
    if (!(a > 0.0) || fabs(d) > a) return 0.0;
    return 0.5 * (1.0 + cospi(d / a));
}

__device__ __forceinline__ double st_point(const StudyGeom& g, int s) { return g.z_first + (double)s * g.z_step; }

__device__ __forceinline__ double st_elem(const StudyGeom& g, int n) { return g.x_first + (double)n * g.pitch; }

// L(RF row, u): linear interpolation, zero outside [0, T - 1].
__device__ __forceinline__ double st_read(const double* row, int T, double u) {
    const double qf = floor(u);
    const double f = u - qf;
    if (!(qf >= -1.0 && qf <= (double)(T - 1))) return 0.0;
    const int k = (int)qf;
    const double s0 = k >= 0 ? row[k] : 0.0;
    const double s1 = k + 1 <= T - 1 ? row[k + 1] : 0.0;
    return (1.0 - f) * s0 + f * s1;
}

// DAS of RF_s on the probe axis at depth z.
__device__ double st_das(const StudyGeom& g, const double* rf_s, double z) {
    double acc = 0.0;
    for (int n = 0; n < g.C; ++n) {
        const double xn = st_elem(g, n);
        const double w = st_hann(-xn, z, g.fnumber);
        if (w == 0.0) continue;
        const double u = (z / g.c + sqrt(xn * xn + z * z) / g.c - g.t0) * g.fs;
        acc += w * st_read(rf_s + (size_t)n * g.T, g.T, u);
    }
    return acc;
}

// The time-invariant line of delay curve zr read on RF_s at depth z.
__device__ double st_fixed(const StudyGeom& g, const double* rf_s, double z, double zr) {
    double acc = 0.0;
    for (int n = 0; n < g.C; ++n) {
        const double xn = st_elem(g, n);
        const double w = st_hann(-xn, zr, g.fnumber);
        if (w == 0.0) continue;
        const double D = (zr - sqrt(xn * xn + zr * zr)) / g.c;  // eqn:delay
        const double u = (2.0 * z / g.c - D - g.t0) * g.fs;
        acc += w * st_read(rf_s + (size_t)n * g.T, g.T, u);
    }
    return acc;
}

// grid (ceil(T / (256 ST_ECHO_PER_THREAD)), C, P), each thread taking
// ST_ECHO_PER_THREAD samples 256 apart.  The transmit arrival of every element at z_s
// is staged in LDS, with the earliest and the latest of them (a min / max
// reduction, exact in any order); a sample more than 4 sigma after the latest
// or before the earliest is more than 4 sigma from every arrival, so every
// pulse gives exactly 0 there and the sample is stored as 0 without the loop
// over the arrivals (most of the record: an echo spans a few hundred
// samples).  Block x = 0, thread 0 also stores the echo's sample support
// [lo, hi] (a superset: a margin of two samples each side).
__global__ __launch_bounds__(ST_THREADS) void study_echo_kernel(const StudyGeom g, double* __restrict__ rf,
                                                                int2* __restrict__ span) {
    extern __shared__ double tx_arrival[];  // [n_tx]
    __shared__ double ext[2][ST_THREADS / 64];
    const int n = blockIdx.y, s = blockIdx.z;
    const double zs = st_point(g, s);
    const double zf = st_point(g, g.focal);
    const int first = (g.C - g.n_tx) / 2;
    double lo_t = INFINITY, hi_t = -INFINITY;
    for (int m = threadIdx.x; m < g.n_tx; m += ST_THREADS) {
        const double xm = st_elem(g, first + m);
        const double Tm = (zf - sqrt(xm * xm + zf * zf)) / g.c;
        const double arr = Tm + sqrt(xm * xm + zs * zs) / g.c;
        tx_arrival[m] = arr;
        lo_t = fmin(lo_t, arr);
        hi_t = fmax(hi_t, arr);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo_t = fmin(lo_t, __shfl_xor(lo_t, off, 64));
        hi_t = fmax(hi_t, __shfl_xor(hi_t, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        ext[0][threadIdx.x >> 6] = lo_t;
        ext[1][threadIdx.x >> 6] = hi_t;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < ST_THREADS / 64; ++w) {
        lo_t = fmin(lo_t, ext[0][w]);
        hi_t = fmax(hi_t, ext[1][w]);
    }
    const double xn = st_elem(g, n);
    const double rx = sqrt(xn * xn + zs * zs) / g.c;
    for (int e = 0; e < ST_ECHO_PER_THREAD; ++e) {
        const int k = (blockIdx.x * ST_ECHO_PER_THREAD + e) * ST_THREADS + threadIdx.x;
        if (k < g.T) {
            const double t = g.t0 + (double)k / g.fs - rx;
            double acc = 0.0;
            if (!(t - hi_t > 4.0 * g.sigma || lo_t - t > 4.0 * g.sigma))
                for (int m = 0; m < g.n_tx; ++m) acc += st_pulse(t - tx_arrival[m], g.fc, g.sigma);
            rf[((size_t)s * g.C + n) * g.T + k] = acc;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double u_lo = (lo_t + rx - 4.0 * g.sigma - g.t0) * g.fs - 2.0;
        const double u_hi = (hi_t + rx + 4.0 * g.sigma - g.t0) * g.fs + 2.0;
        // clamped in float64 before the conversion: an echo wholly outside
        // the record gives lo > hi (an empty support)
        const int lo = (int)fmin(fmax(0.0, floor(u_lo)), (double)g.T);
        const int hi = (int)fmax(fmin((double)(g.T - 1), ceil(u_hi)), -1.0);
        span[(size_t)s * g.C + n] = make_int2(lo, hi);
    }
}

// grid (ceil((2 Ql + 1) / 256), P): b_s(z_s + q dzf).
__global__ __launch_bounds__(ST_THREADS) void study_das_kernel(const StudyGeom g, const double* __restrict__ rf,
                                                               double* __restrict__ bline) {
    const int L = 2 * g.Ql + 1;
    const int s = blockIdx.y;
    const int i = blockIdx.x * ST_THREADS + threadIdx.x;
    if (i >= L) return;
    const double z = st_point(g, s) + (double)(i - g.Ql) * g.dzf;
    bline[(size_t)s * L + i] = st_das(g, rf + (size_t)s * g.C * g.T, z);
}

// One workgroup: W (metres) and Qw = floor(W / (2 dzf)) into `win`.
__global__ __launch_bounds__(ST_THREADS) void study_window_kernel(const StudyGeom g, const double* __restrict__ rf,
                                                                  double* __restrict__ win) {
    __shared__ double b[ENV_MAX];
    __shared__ double env[ENV_MAX];
    __shared__ double Xr[ENV_MAX + 1];
    __shared__ double Xi[ENV_MAX + 1];
    __shared__ double tc[2 * ENV_MAX];
    __shared__ double ts[2 * ENV_MAX];
    const int L = 2 * g.Qf + 1;
    const double zf = st_point(g, g.focal);
    const double* rf_f = rf + (size_t)g.focal * g.C * g.T;
    for (int q = threadIdx.x; q < L; q += ST_THREADS) b[q] = st_das(g, rf_f, zf + (double)(q - g.Qf) * g.dzf);
    __syncthreads();
    block_envelope<ST_THREADS>(b, L, env, Xr, Xi, tc, ts);
    if (threadIdx.x == 0) {
        const double W = env_fwhm(env, L) * g.dzf;
        win[0] = W;
        win[1] = floor(0.5 * W / g.dzf);
    }
}

// grid (ceil(P / ST_RB), P).  Workgroup (rb, s): delay curves r = ST_RB rb ..
// +ST_RB-1 on scatterer s.  Each thread owns the line samples q = -Ql + t +
// 256 j and, per sample, sums the channels of all ST_RB curves: the read
// position of channel n for curve r is u = u0[r][n] + q, so its integer part
// kq + q and fraction f are fixed per (r, n) and staged in LDS with the
// weights; reads outside the echo's support are skipped (they are zeros).
// The samples are taken 256 at a time: for each such chunk the workgroup
// first lists, in order of r then n, the (r, n) with a non-zero weight whose
// support meets the chunk's read positions (an interval of q per (r, n)), so
// a thread visits only those (an echo's support spans a few hundred samples
// of a line of thousands, so most (r, n) reach no sample of a chunk), and a
// wave passes over the listed entries that reach none of its own 64 samples;
// each curve's channels are still summed in increasing n, as in a plain loop
// over the aperture, so the bits do not depend on the lists.
// The line's sums go through a fixed-order workgroup reduction, then thread
// 0 forms Theta and both errors from them:
//   ||t a - b||^2 = t^2 sum a^2 - 2 t sum a b + sum b^2  (clamped at 0).
__global__ __launch_bounds__(ST_THREADS) void study_pair_kernel(const StudyGeom g, const double* __restrict__ rf,
                                                                const int2* __restrict__ span,
                                                                const double* __restrict__ bline,
                                                                const double* __restrict__ win,
                                                                double* __restrict__ theta,
                                                                double* __restrict__ err_local,
                                                                double* __restrict__ err_global) {
    extern __shared__ double lds[];
    double* w_rn = lds;                                    // [ST_RB][C]
    double* f_rn = w_rn + ST_RB * g.C;                     // [ST_RB][C]
    int* k_rn = (int*)(f_rn + ST_RB * g.C);                // [ST_RB][C]
    int2* sp = (int2*)(k_rn + ST_RB * g.C);                // [C]
    __shared__ double red[ST_THREADS / 64][2 + 4 * ST_RB];
    __shared__ double tot[2 + 4 * ST_RB];
    __shared__ int n_range[2];
    __shared__ int lst[ST_RB * ST_MAX_ELEM];
    __shared__ int seg[ST_RB + 1];
    __shared__ int wcnt[ST_THREADS / 64];
    const int s = blockIdx.y;
    const int r0 = blockIdx.x * ST_RB;
    const double zs = st_point(g, s);
    const double* rf_s = rf + (size_t)s * g.C * g.T;
    const int Qw = (int)win[1];
    int n_lo = g.C, n_hi = -1;
    for (int e = threadIdx.x; e < ST_RB * g.C; e += ST_THREADS) {
        const int j = e / g.C, n = e % g.C;
        const int r = min(r0 + j, g.P - 1);
        const double zr = st_point(g, r);
        const double xn = st_elem(g, n);
        const double w = (r0 + j < g.P) ? st_hann(-xn, zr, g.fnumber) : 0.0;
        const double D = (zr - sqrt(xn * xn + zr * zr)) / g.c;
        const double u0 = (2.0 * zs / g.c - D - g.t0) * g.fs;
        const double kf = floor(u0);
        w_rn[e] = w;
        f_rn[e] = u0 - kf;
        k_rn[e] = (int)kf;
    }
    for (int n = threadIdx.x; n < g.C; n += ST_THREADS) sp[n] = span[(size_t)s * g.C + n];
    if (threadIdx.x == 0) {
        n_range[0] = g.C;
        n_range[1] = -1;
    }
    __syncthreads();
    // channels with a non-zero weight for some curve of the block: the
    // apertures are symmetric intervals, so their union is one interval
    for (int e = threadIdx.x; e < ST_RB * g.C; e += ST_THREADS)
        if (w_rn[e] != 0.0) {
            n_lo = min(n_lo, e % g.C);
            n_hi = max(n_hi, e % g.C);
        }
    if (n_hi >= 0) {
        atomicMin(&n_range[0], n_lo);
        atomicMax(&n_range[1], n_hi);
    }
    __syncthreads();
    n_lo = n_range[0];
    n_hi = n_range[1];

    double ab[ST_RB], aa[ST_RB], abB[ST_RB], aaB[ST_RB];
    double bb = 0.0, bbB = 0.0;
#pragma unroll
    for (int j = 0; j < ST_RB; ++j) ab[j] = aa[j] = abB[j] = aaB[j] = 0.0;
    const int L = 2 * g.Ql + 1;
    // entries (j, n), j-major over the channels n_lo .. n_hi (none if no
    // channel has a weight)
    const int Cr = n_hi - n_lo + 1;
    const int E = Cr > 0 ? ST_RB * Cr : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = -g.Ql; c0 <= g.Ql; c0 += ST_THREADS) {
        const int c1 = c0 + ST_THREADS - 1;
        // the chunk's list: lst[seg[j] .. seg[j + 1]) holds, in increasing n,
        // the channels of curve j whose read positions k_rn + q, q in
        // [c0, c1], meet the support [su.x - 1, su.y] (an ordered compaction:
        // per pass over 256 entries a ballot per wave and the waves' counts)
        if (threadIdx.x <= ST_RB) seg[threadIdx.x] = 0;
        int base = 0;
        for (int t0 = 0; t0 < E; t0 += ST_THREADS) {
            const int idx = t0 + threadIdx.x;
            bool keep = false;
            int j = 0, n = 0;
            if (idx < E) {
                j = idx / Cr;
                n = n_lo + idx - j * Cr;
                const int e = j * g.C + n;
                const int2 su = sp[n];
                keep = w_rn[e] != 0.0 && su.x - 1 - k_rn[e] <= c1 && su.y - k_rn[e] >= c0;
            }
            const uint64_t m = __ballot(keep);
            if (lane == 0) wcnt[wave] = __popcll(m);
            __syncthreads();
            int pos = base, tot = 0;
#pragma unroll
            for (int w = 0; w < ST_THREADS / 64; ++w) {
                pos += w < wave ? wcnt[w] : 0;
                tot += wcnt[w];
            }
            pos += __popcll(m & ((1ull << lane) - 1ull));
            if (idx < E && n == n_lo) seg[j] = pos;  // entries listed before curve j's first
            if (keep) lst[pos] = n;
            base += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) seg[ST_RB] = base;
        __syncthreads();

        const int q = c0 + threadIdx.x;
        const int wq0 = c0 + 64 * wave, wq1 = wq0 + 63;  // this wave's samples
        if (q <= g.Ql) {
            double a[ST_RB];
#pragma unroll
            for (int j = 0; j < ST_RB; ++j) {
                a[j] = 0.0;
                const int t_end = seg[j + 1];
                for (int t = seg[j]; t < t_end; ++t) {
                    const int n = lst[t];
                    const int e = j * g.C + n;
                    const int2 su = sp[n];
                    const int kr = k_rn[e];
                    // the same for every lane of the wave: an entry whose
                    // reads miss the wave's 64 samples adds nothing to them
                    if (su.x - 1 - kr > wq1 || su.y - kr < wq0) continue;
                    // reads at positions clamped into the record (every one in
                    // bounds), added where the sample lies in the support
                    const int k = kr + q;
                    const double* row = rf_s + (size_t)n * g.T;
                    const double r0 = row[min(max(k, 0), g.T - 1)];
                    const double r1 = row[min(max(k + 1, 0), g.T - 1)];
                    if (k >= su.x - 1 && k <= su.y) {
                        const double f = f_rn[e];
                        const double s0 = k >= su.x ? r0 : 0.0;
                        const double s1 = k + 1 <= su.y ? r1 : 0.0;
                        a[j] += w_rn[e] * ((1.0 - f) * s0 + f * s1);
                    }
                }
            }
#ifdef TIDAS_DEBUG
            // the support table: samples it leaves out are zero
            for (int n = n_lo; n <= n_hi; ++n) {
                const int2 su = sp[n];
                const double* row = rf_s + (size_t)n * g.T;
                for (int j = 0; j < ST_RB; ++j) {
                    const int e = j * g.C + n;
                    const int k = k_rn[e] + q;
                    if (k >= 0 && k < g.T && (k < su.x || k > su.y))
                        TIDAS_DCHECK(w_rn[e] == 0.0 || row[k] == 0.0, TIDAS_DBG_STUDY_SPAN);
                }
            }
#endif
            const double b = bline[(size_t)s * L + (q + g.Ql)];
            const bool inB = q >= -Qw && q <= Qw;
            bb += b * b;
            if (inB) bbB += b * b;
#pragma unroll
            for (int j = 0; j < ST_RB; ++j) {
                ab[j] += a[j] * b;
                aa[j] += a[j] * a[j];
                if (inB) {
                    abB[j] += a[j] * b;
                    aaB[j] += a[j] * a[j];
                }
            }
        }
        __syncthreads();  // the next chunk rewrites the list
    }
    // the 2 + 4 ST_RB sums over the workgroup, each in a fixed order: a
    // shuffle tree within each wave, then the waves' partial sums in order
    constexpr int NS = 2 + 4 * ST_RB;
    double v[NS];
    v[0] = bb;
    v[1] = bbB;
#pragma unroll
    for (int j = 0; j < ST_RB; ++j) {
        v[2 + 4 * j] = ab[j];
        v[3 + 4 * j] = aa[j];
        v[4 + 4 * j] = abB[j];
        v[5 + 4 * j] = aaB[j];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i)
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NS; ++i) red[wave][i] = v[i];
    __syncthreads();
    // thread i adds the waves' parts of sum i (thread 0 reading all of them
    // at once held them all in registers: 144 of them)
    if (threadIdx.x < NS) {
        double t = 0.0;
        for (int w = 0; w < ST_THREADS / 64; ++w) t += red[w][threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sbb = tot[0], sbbB = tot[1];
#pragma unroll
        for (int j = 0; j < ST_RB; ++j) {
            const int r = r0 + j;
            if (r >= g.P) break;
            const double sab = tot[2 + 4 * j], saa = tot[3 + 4 * j], sabB = tot[4 + 4 * j], saaB = tot[5 + 4 * j];
            const double t = saaB > 0.0 ? sabB / saaB : 0.0;
            const double el = t * t * saaB - 2.0 * t * sabB + sbbB;
            const double eg = t * t * saa - 2.0 * t * sab + sbb;
            const size_t o = (size_t)r * g.P + s;
            theta[o] = t;
            err_local[o] = sbbB > 0.0 ? fmax(el, 0.0) / sbbB : 0.0;
            err_global[o] = sbb > 0.0 ? fmax(eg, 0.0) / sbb : 0.0;
        }
    }
}

// grid (P): stats[s] = (DAS peak, tiDAS peak, DAS FWHM, tiDAS FWHM) of the
// DAS line and of Theta[focal][s] times the focal curve's time-invariant
// line on |q| <= Qh (envelope maxima and envelope FWHMs in metres).
__global__ __launch_bounds__(ST_THREADS) void study_stats_kernel(const StudyGeom g, const double* __restrict__ rf,
                                                                 const double* __restrict__ theta,
                                                                 double* __restrict__ stats) {
    __shared__ double b[ENV_MAX];
    __shared__ double a[ENV_MAX];
    __shared__ double env[ENV_MAX];
    __shared__ double Xr[ENV_MAX + 1];
    __shared__ double Xi[ENV_MAX + 1];
    __shared__ double tc[2 * ENV_MAX];
    __shared__ double ts[2 * ENV_MAX];
    const int s = blockIdx.x;
    const int L = 2 * g.Qh + 1;
    const double zs = st_point(g, s);
    const double zf = st_point(g, g.focal);
    const double t = theta[(size_t)g.focal * g.P + s];
    const double* rf_s = rf + (size_t)s * g.C * g.T;
    for (int q = threadIdx.x; q < L; q += ST_THREADS) {
        const double z = zs + (double)(q - g.Qh) * g.dzf;
        b[q] = st_das(g, rf_s, z);
        a[q] = t * st_fixed(g, rf_s, z, zf);
    }
    __syncthreads();
    block_envelope<ST_THREADS>(b, L, env, Xr, Xi, tc, ts);
    if (threadIdx.x == 0) {
        stats[(size_t)s * 4 + 0] = env[env_peak(env, L)];
        stats[(size_t)s * 4 + 2] = env_fwhm(env, L) * g.dzf;
    }
    __syncthreads();
    block_envelope<ST_THREADS>(a, L, env, Xr, Xi, tc, ts);
    if (threadIdx.x == 0) {
        stats[(size_t)s * 4 + 1] = env[env_peak(env, L)];
        stats[(size_t)s * 4 + 3] = env_fwhm(env, L) * g.dzf;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct StudyLayout {
    size_t rf, span, bline, win, total;
};

StudyLayout study_layout(int64_t C, int64_t P, int64_t T, int64_t Ql) {
    StudyLayout l;
    l.rf = 0;
    l.span = l.rf + align256((size_t)(P * C * T) * sizeof(double));
    l.bline = l.span + align256((size_t)(P * C) * sizeof(int2));
    l.win = l.bline + align256((size_t)(P * (2 * Ql + 1)) * sizeof(double));
    l.total = l.win + 256;
    return l;
}

int fine_half(double fs, double sigma) { return (int)std::ceil(8.0 * sigma * fs); }

}  // namespace
}  // namespace tidas

using namespace tidas;

extern "C" int32_t tidas_kossoff_tx_count(const tidas_array* array, double fc, double z_focus, double ratio) {
    if (int32_t st = validate_array(array)) return st;
    if (!finite_pos(fc) || !finite_pos(z_focus) || !finite_pos(ratio))
        return fail(TIDAS_EINVAL, "tidas_kossoff_tx_count: fc, z_focus and ratio must be > 0");
    const double lam = array->c / fc;
    const double width = std::sqrt(4.0 * lam * z_focus / ratio);
    const int par = array->n_elem % 2;
    const double half = (width / array->pitch - par) / 2.0 + 0.5;
    if (!(half < 1e9)) return array->n_elem;
    const int n = par + 2 * (int)std::floor(half);
    return std::min(std::max(n, par ? 1 : 2), (int)array->n_elem);
}

extern "C" size_t tidas_point_study_workspace_bytes(int32_t n_elem, int32_t n_points, int32_t n_samples,
                                                     int32_t line_half) {
    if (n_elem < 1 || n_points < 1 || n_samples < 2 || line_half < 0) return 0;
    return study_layout(n_elem, n_points, n_samples, line_half).total;
}

extern "C" int32_t tidas_point_study(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                                     int32_t n_tx, int32_t n_samples, int32_t n_points, double z_first,
                                     double z_step, int32_t focal_index, int32_t line_half, int32_t stats_half,
                                     double* theta, double* err_local, double* err_global, double* stats,
                                     double* window, void* workspace, size_t workspace_bytes, void* stream) {
    if (int32_t st = validate_array(array)) return st;
    if (int32_t st = validate_tx(tx, true)) return st;
    if (int32_t st = validate_rx(rx)) return st;
    if (tx->n_angles != 1 || tx->angles[0] != 0.0)
        return fail(TIDAS_EINVAL, "tidas_point_study: the focused transmit is unsteered (one angle, 0)");
    const int32_t C = array->n_elem;
    if (C > ST_MAX_ELEM) return fail(TIDAS_EUNSUPPORTED, "tidas_point_study: at most 512 elements");
    if (n_tx < 1 || n_tx > C || ((C - n_tx) % 2) != 0)
        return fail(TIDAS_EINVAL, "tidas_point_study: n_tx must be in [1, C] with C - n_tx even");
    if (n_samples < 2) return fail(TIDAS_EINVAL, "tidas_point_study: n_samples must be >= 2");
    if (n_points < 1) return fail(TIDAS_EINVAL, "tidas_point_study: n_points must be >= 1");
    if (!std::isfinite(z_first) || z_first <= 0.0 || !std::isfinite(z_step) || (n_points > 1 && z_step <= 0.0))
        return fail(TIDAS_EINVAL, "tidas_point_study: z_first and z_step must be > 0");
    if (focal_index < 0 || focal_index >= n_points)
        return fail(TIDAS_EINVAL, "tidas_point_study: focal_index outside the points");
    if (line_half < 0) return fail(TIDAS_EINVAL, "tidas_point_study: line_half must be >= 0");
    if (!theta || !err_local || !err_global || !workspace)
        return fail(TIDAS_EINVAL, "tidas_point_study: null pointer");
    if (theta == err_local || theta == err_global || err_local == err_global ||
        (stats && (stats == theta || stats == err_local || stats == err_global)))
        return fail(TIDAS_EINVAL, "tidas_point_study: outputs overlap");
    if (stats && (stats_half < 0 || 2 * stats_half + 1 > ENV_MAX))
        return fail(TIDAS_EINVAL, "tidas_point_study: stats_half must be in [0, 511]");
    StudyGeom g;
    g.C = C;
    g.T = n_samples;
    g.P = n_points;
    g.n_tx = n_tx;
    g.Ql = line_half;
    g.Qh = stats ? stats_half : 0;
    g.focal = focal_index;
    g.pitch = array->pitch;
    g.c = array->c;
    g.fs = tx->fs;
    g.t0 = tx->t0;
    g.fc = tx->fc;
    g.sigma = (tx->cycles / tx->fc) / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    g.fnumber = rx->fnumber;
    g.x_first = -0.5 * (double)(C - 1) * g.pitch;
    g.z_first = z_first;
    g.z_step = z_step;
    g.dzf = g.c / (2.0 * g.fs);
    g.Qf = fine_half(g.fs, g.sigma);
    if (2 * (int64_t)g.Qf + 1 > ENV_MAX)
        return fail(TIDAS_EUNSUPPORTED, "tidas_point_study: the FWHM axis (8 pulse sigmas) exceeds 1023 samples");
    if ((int64_t)n_points * (2 * (int64_t)line_half + 1) > ((int64_t)1 << 40) || (int64_t)n_points > 65535 ||
        (int64_t)C * n_samples > ((int64_t)1 << 31))
        return fail(TIDAS_EUNSUPPORTED, "tidas_point_study: sizes too large");
    const StudyLayout lay = study_layout(C, n_points, n_samples, line_half);
    if (workspace_bytes < lay.total) return fail(TIDAS_EINVAL, "tidas_point_study: workspace too small");
    char* ws = (char*)workspace;
    double* rf = (double*)(ws + lay.rf);
    int2* span = (int2*)(ws + lay.span);
    double* bline = (double*)(ws + lay.bline);
    double* win = (double*)(ws + lay.win);
    hipStream_t s = (hipStream_t)stream;

    hipLaunchKernelGGL(study_echo_kernel,
                       dim3((uint32_t)((n_samples + ST_THREADS * ST_ECHO_PER_THREAD - 1) / (ST_THREADS * ST_ECHO_PER_THREAD)),
                            C, n_points),
                       dim3(ST_THREADS), (size_t)n_tx * sizeof(double), s, g, rf, span);
    if (int32_t st = check_launch("tidas_point_study(echo)")) return st;
    const int64_t L = 2 * (int64_t)line_half + 1;
    hipLaunchKernelGGL(study_das_kernel, dim3((uint32_t)((L + ST_THREADS - 1) / ST_THREADS), n_points),
                       dim3(ST_THREADS), 0, s, g, rf, bline);
    if (int32_t st = check_launch("tidas_point_study(das)")) return st;
    hipLaunchKernelGGL(study_window_kernel, dim3(1), dim3(ST_THREADS), 0, s, g, rf, win);
    if (int32_t st = check_launch("tidas_point_study(window)")) return st;
    const size_t pair_lds = (size_t)ST_RB * C * (2 * sizeof(double) + sizeof(int)) + (size_t)C * sizeof(int2);
    hipLaunchKernelGGL(study_pair_kernel, dim3((uint32_t)((n_points + ST_RB - 1) / ST_RB), n_points),
                       dim3(ST_THREADS), pair_lds, s, g, rf, span, bline, win, theta, err_local, err_global);
    if (int32_t st = check_launch("tidas_point_study(pairs)")) return st;
    if (stats) {
        hipLaunchKernelGGL(study_stats_kernel, dim3(n_points), dim3(ST_THREADS), 0, s, g, rf, theta, stats);
        if (int32_t st = check_launch("tidas_point_study(stats)")) return st;
    }
    if (window) {
        if (int32_t st = check_hip(hipMemcpyAsync(window, win, sizeof(double), hipMemcpyDeviceToDevice, s),
                                   "tidas_point_study: window"))
            return st;
    }
    return TIDAS_OK;
}
