// Envelope and FWHM of a sampled depth profile, shared by the paper-mode
// kernel build and the single-point study (Sec. 3.1-3.2: the FWHM of the
// DAS PSF's envelope sets the correction window).  Float64 throughout.
#pragma once

#include <hip/hip_runtime.h>

namespace tidas {

constexpr int ENV_MAX = 1024;  // longest profile (the DFT length is at most 2 ENV_MAX)

// env[n] = |analytic signal of b|[n], n < L <= ENV_MAX: DFT of b zero-padded
// to N (the first power of two >= 2 L) at bins 0 .. N/2, weighted 1 at 0 and
// N/2 and 2 in between (the analytic signal keeps those bins), then the
// inverse DFT at n < L.  Xr, Xi hold N/2 + 1 entries; tc, ts (2 ENV_MAX
// entries each) take the N twiddles cos, sin of 2 pi m / N, evaluated once per
// call and read by both transforms (each term used to evaluate its own: the
// same values, so the same sums).  All THREADS threads of the workgroup call
// it; b must be complete (a barrier before the call) and env is complete on
// return.
template <int THREADS>
__device__ void block_envelope(const double* b, int L, double* env, double* Xr, double* Xi, double* tc, double* ts) {
    int N = 1;
    while (N < 2 * L) N *= 2;
    for (int m = threadIdx.x; m < N; m += THREADS) sincospi(2.0 * (double)m / (double)N, &ts[m], &tc[m]);
    __syncthreads();
    for (int k = threadIdx.x; k <= N / 2; k += THREADS) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < L; ++n) {
            const int m = (int)(((int64_t)k * n) & (N - 1));
            re += b[n] * tc[m];
            im -= b[n] * ts[m];
        }
        const double wgt = (k == 0 || k == N / 2) ? 1.0 : 2.0;
        Xr[k] = wgt * re;
        Xi[k] = wgt * im;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < L; n += THREADS) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= N / 2; ++k) {
            const int m = (int)(((int64_t)k * n) & (N - 1));
            const double cs = tc[m], sn = ts[m];
            re += Xr[k] * cs - Xi[k] * sn;
            im += Xr[k] * sn + Xi[k] * cs;
        }
        env[n] = sqrt(re * re + im * im) / (double)N;
    }
    __syncthreads();
}

// Index of the (first) maximum of env[0..L).
__device__ __forceinline__ int env_peak(const double* env, int L) {
    int p = 0;
    for (int n = 1; n < L; ++n)
        if (env[n] > env[p]) p = n;
    return p;
}

// Full width at half maximum of env[0..L) in samples: from the first maximum
// walk outwards to the first samples below half of it and interpolate the
// crossings linearly; an end of the axis with no crossing counts as the
// crossing.  One thread.
__device__ __forceinline__ double env_fwhm(const double* env, int L) {
    const int p = env_peak(env, L);
    const double half = 0.5 * env[p];
    int lo = p;
    while (lo > 0 && env[lo - 1] >= half) --lo;
    const double xl = (lo == 0) ? 0.0 : (lo - 1) + (half - env[lo - 1]) / (env[lo] - env[lo - 1]);
    int hi = p;
    while (hi < L - 1 && env[hi + 1] >= half) ++hi;
    const double xr = (hi == L - 1) ? (double)(L - 1) : hi + (env[hi] - half) / (env[hi] - env[hi + 1]);
    return xr - xl;
}

}  // namespace tidas
