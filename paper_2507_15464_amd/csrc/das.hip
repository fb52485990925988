// Exact Delay-and-Sum beamformer for plane-wave transmits (Sec. 2, eqn:appF).
//
// Mapping on gfx950: one wavefront = a tile of 2 depth rows x 32 consecutive
// image columns (lane l: row l % 2, column l / 2); a workgroup stacks 4 such
// tiles in depth (8 rows x 32 columns).  For a fixed element n the lanes read
// a short, monotone window of that element's channel: along a row the sample
// index changes by at most dx fs / (c F') per column (~1.5 samples here),
// down a column by 2 dz fs / c (~3.8), so the tile spans ~55 samples (a row of
// 64 pixels ~100, a column of 64 ~250).  The channel gathers, not the
// arithmetic, bound this kernel; measured on the benchmark workload (64
// frames, with the paired 8-byte reads below): 0.57 ms as 2 x 32 tiles, 0.60
// as 1 x 64 and as 4 x 16, 0.72 as 8 x 8 (wider tiles also waste lanes on
// elements outside their own aperture).
//
// Delay precision.  The fractional sample index is split:
//   u = fs (tau_tx(x_j, z_i; a) + z_i / c - t0)      [per pixel, float64]
//     + (fs / c) * dx^2 / (rho + z_i)                 [per pixel and element, float32]
// The first term (up to ~8000 samples) is split once per pixel into an
// integer and a float fraction; the second is the receive excess rho - z,
// written without cancellation, so float32 only has to carry a quantity of
// at most a few hundred samples.  Plain float32 evaluation of the whole
// index would lose ~2e-4 samples, i.e. ~1e-4 relative error per term.
//
// The element loop runs over the union of the tile's apertures with a
// branch-free body: a lane outside its own aperture gets weight 0 (its reads
// are in range or read 0, and add exactly 0), so loads of consecutive
// elements can be in flight together.
//
// Each thread can beamform FB frames that share the geometry: delays and
// apodization are computed once per (pixel, element) and reused.  Eight or
// more frames (one angle, or the 11-angle compounding) are first copied into
// a frame-interleaved layout, [group of 4][angle][channel][sample][frame], so
// that one 16-byte load returns a sample of four frames: the gathers then
// issue half the load instructions, which the texture address unit (~16
// cycles per load instruction, whatever its width) bounds.  Measured on the
// benchmark workload: 0.57-0.60 ms per 64 frames with one 8-byte load per
// frame and pair, 0.37-0.43 ms with the copy (39 us of it).
#include <algorithm>
#include <climits>
#include <vector>

#include "common.hpp"

namespace tidas {

TIDAS_DEBUG_FLAGS_DEFINE(das)

typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int DAS_MAX_ANGLES = 32;

struct DasArgs {
    int32_t C, T, A, n_frames;
    double pitch, fs, t0, fnumber, c;
    double x_first;    // x of element 0
    float kappa;       // fs / c
    double sin_a[DAS_MAX_ANGLES];
    double cos_a[DAS_MAX_ANGLES];
};

// Grid of one frame (or of every frame of a uniform batch).
struct DasGrid {
    int32_t nz, nx;
    double z0, dz, x0, dx;
};

// Wave tile: WZ depth rows x 64 / WZ columns.  One angle: 2 x 32 (the
// narrowest sample windows); several angles: 1 x 64 (a steered transmit adds
// x sin(alpha) to the index, so rows of pixels spread less than two-row tiles
// over the angles' windows; measured on the 11-angle batch: 5.5 ms as 1 x 64,
// 9.2 ms as 2 x 32).
__host__ __device__ constexpr int das_wz(int na) { return na == 1 ? 2 : 1; }
__host__ __device__ constexpr int das_wx(int na) { return 64 / das_wz(na); }
constexpr int DAS_BZ = 4;   // wave tiles per workgroup, stacked in depth

// One wave: the WZ x WX pixel tile at rows i_base.., columns j_base.., for FB
// frames sharing the geometry.  rf points at the first frame's [A][C][T]
// record, img at its [nz][nx] image; frame f of the group is rf + f *
// frame_rf, img + f * frame_img.  IL (FB a multiple of 4): rf points at the
// group's frame-interleaved record [A][C][T][FB] instead (das_interleave_kernel),
// so one 16-byte load returns a sample of four frames.
template <int FB, int NA, int WZ = das_wz(NA), bool IL = false>
__device__ __forceinline__ void das_wave(const DasArgs& p, const DasGrid& gr, int i_base, int j_base, int nfr,
                                         const float* __restrict__ rf, size_t frame_rf, float* img,
                                         size_t frame_img) {
    static_assert(WZ == 1 || WZ == 2 || WZ == 4, "wave tiles of 1 x 64, 2 x 32 or 4 x 16 pixels");
    constexpr int WX = 64 / WZ;
    const int lane = threadIdx.x & 63;
    const int i = i_base + (lane % WZ);
    const int j = j_base + (lane / WZ);
    const int A = (NA > 0) ? NA : p.A;

    const double xd = gr.x0 + (double)min(j, gr.nx - 1) * gr.dx;
    // lateral offset to element n: x_j - x_n = (x_j - x_0) - n pitch with the
    // origin and the pitch as float32 pairs (hi + lo): fma(-n, pitch_hi,
    // origin_hi) is rounded once from its exact value, and the lo terms carry
    // the rest, so dx keeps float32 accuracy relative to its own size (as the
    // float64 difference rounded to float32 would), not to the origin's
    const double ox = xd - p.x_first;
    const float dx0 = (float)ox, dx0_lo = (float)(ox - (double)dx0);
    const float pitch_f = (float)p.pitch, pitch_lo = (float)(p.pitch - (double)pitch_f);
    const double zd = gr.z0 + (double)min(i, gr.nz - 1) * gr.dz;
    const bool active = (i < gr.nz) && (j < gr.nx) && (zd > 0.0);
    const float zf = (float)zd;
    const float z2 = (float)(zd * zd);
    const float inv_az = active ? (float)(2.0 * p.fnumber / zd) : 0.0f;

    // per-angle integer and fractional parts of fs (tau_tx + z/c - t0)
    int q_a[(NA > 0) ? NA : DAS_MAX_ANGLES];
    float f_a[(NA > 0) ? NA : DAS_MAX_ANGLES];
#pragma unroll
    for (int a = 0; a < ((NA > 0) ? NA : DAS_MAX_ANGLES); ++a) {
        if (a < A) {
            const double U = p.fs * ((xd * p.sin_a[a] + zd * p.cos_a[a]) / p.c + zd / p.c - p.t0);
            const double Uf = floor(U);
            q_a[a] = (int)Uf;
            f_a[a] = (float)(U - Uf);
        }
    }

    // element range covering the widest aperture among the tile's pixels
    const int i_last = min(i_base + WZ - 1, gr.nz - 1);
    const double z_last = gr.z0 + (double)i_last * gr.dz;
    const double x_lo = gr.x0 + (double)j_base * gr.dx;
    const double x_hi = gr.x0 + (double)min(j_base + WX - 1, gr.nx - 1) * gr.dx;
    int n_lo = 0, n_hi = -1;
    if (z_last > 0.0) {
        const double a_max = z_last / (2.0 * p.fnumber);
        n_lo = max(0, (int)floor((fmin(x_lo, x_hi) - a_max - p.x_first) / p.pitch));
        n_hi = min(p.C - 1, (int)ceil((fmax(x_lo, x_hi) + a_max - p.x_first) / p.pitch));
    }

    float acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = 0.0f;

    const uint32_t row_bytes = (uint32_t)p.T * 4u;
    const int last_pair = (p.T - 2) * 4;  // byte offset of the last sample pair
    // two elements' loads in flight together, except for the interleaved
    // compounding, whose angles already hold 22 16-byte loads per element
    constexpr int UNR = (IL && NA > 1) ? 1 : 2;
#pragma unroll UNR
    for (int n = n_lo; n <= n_hi; ++n) {
        const float nf = (float)n;
        const float dx = fmaf(-nf, pitch_f, dx0) + fmaf(-nf, pitch_lo, dx0_lo);
        const float t = fabsf(dx) * inv_az;
        const float wh = hann_weight(fminf(t, 1.0f));
        const float w = (active && t <= 1.0f) ? wh : 0.0f;
        const float rho = __builtin_amdgcn_sqrtf(fmaf(dx, dx, z2));
        const float ke = p.kappa * (dx * dx) * __builtin_amdgcn_rcpf(rho + zf);
#pragma unroll
        for (int a = 0; a < ((NA > 0) ? NA : DAS_MAX_ANGLES); ++a) {
            if (a < A) {
                const float v = f_a[a] + ke;
                const float qf = floorf(v);
                const float fr = v - qf;
                const int off = (q_a[a] + (int)qf) * 4;
                const size_t ch = (size_t)a * p.C + n;
                if constexpr (FB > 1) {
                    // Both samples of the read come from one 8-byte load at the
                    // pair's offset clamped into [0, T - 2]; the clamp's shift d
                    // (in bytes) says which of the two loaded samples the read
                    // needs: d = 0 both, d = -4 (q = -1) the first as S[q + 1],
                    // d = +4 (q = T - 1) the second as S[q], otherwise none (the
                    // read lies outside the record and is 0).  The weights fold
                    // the interpolation, the case and the apodization, once for
                    // the FB frames.
                    const int oc = min(max(off, 0), last_pair);
                    const int d = off - oc;
                    const float wa = d == 0 ? w * (1.0f - fr) : (d == -4 ? w * fr : 0.0f);
                    const float wb = d == 0 ? w * fr : (d == 4 ? w * (1.0f - fr) : 0.0f);
                    if constexpr (IL) {
                        // channel ch of the group: T samples x FB frames; sample
                        // q of frames 4k..4k+3 at byte 16 (FB / 4 q + k)
                        static_assert(FB % 4 == 0, "interleaved records hold frames in fours");
                        constexpr int NQ = FB / 4;
                        const auto rs = make_rsrc(rf + ch * p.T * FB, row_bytes * FB);
                        floatx4 s0[NQ], s1[NQ];
#pragma unroll
                        for (int k = 0; k < NQ; ++k) {
                            s0[k] = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, oc * FB + 16 * k, 0, 0));
                            s1[k] = __builtin_bit_cast(floatx4,
                                                       __builtin_amdgcn_raw_buffer_load_b128(rs, (oc + 4) * FB + 16 * k, 0, 0));
                        }
#pragma unroll
                        for (int f = 0; f < FB; ++f) {
                            const float a0 = s0[f / 4][f % 4], a1 = s1[f / 4][f % 4];
                            TIDAS_DCHECK((wa == 0.0f || __builtin_isfinite(a0)) && (wb == 0.0f || __builtin_isfinite(a1)),
                                         TIDAS_DBG_NONFINITE_IN);
                            acc[f] = fmaf(wb, a1, fmaf(wa, a0, acc[f]));
                        }
                    } else {
#pragma unroll
                        for (int f = 0; f < FB; ++f) {
                            // every frame slot loads (a slot past the group's last
                            // frame has an empty record: it reads 0 and is never
                            // stored), so the loads of all slots and of the next
                            // element are in flight together
                            const bool fv = f < nfr;
                            const auto rs = make_rsrc(rf + (fv ? f : 0) * frame_rf + ch * p.T, fv ? row_bytes : 0u);
                            const floatx2 sp =
                                __builtin_bit_cast(floatx2, __builtin_amdgcn_raw_buffer_load_b64(rs, oc, 0, 0));
                            TIDAS_DCHECK((wa == 0.0f || __builtin_isfinite(sp[0])) && (wb == 0.0f || __builtin_isfinite(sp[1])),
                                         TIDAS_DBG_NONFINITE_IN);
                            acc[f] = fmaf(wb, sp[1], fmaf(wa, sp[0], acc[f]));
                        }
                    }
                } else {
                    // one frame (per-angle work not shared): two dword reads, each
                    // range-checked on its own.  The neighbour's offset is computed
                    // apart (not off + 4) so that the two loads are not merged into
                    // one 8-byte load, whose range check at sample -1 (offset -4,
                    // huge unsigned) would also discard the in-range sample 0.
                    const int off1 = (q_a[a] + (int)(qf + 1.0f)) * 4;
                    const auto rs = make_rsrc(rf + ch * p.T, nfr > 0 ? row_bytes : 0u);
                    const float s0 = buffer_load_f32(rs, off);
                    const float s1 = buffer_load_f32(rs, off1);
                    TIDAS_DCHECK(w == 0.0f || (__builtin_isfinite(s0) && __builtin_isfinite(s1)), TIDAS_DBG_NONFINITE_IN);
                    acc[0] = fmaf(w, fmaf(fr, s1 - s0, s0), acc[0]);
                }
            }
        }
    }
    // the image is not read again: stored non-temporally, so that the L2
    // keeps the channel windows that neighbouring tiles read (measured on the
    // benchmark's 64 frames: 369-421 -> 357-385 us)
    if (i < gr.nz && j < gr.nx) {
#pragma unroll
        for (int f = 0; f < FB; ++f)
            if (f < nfr) __builtin_nontemporal_store(acc[f], &img[f * frame_img + (size_t)i * gr.nx + j]);
    }
}

// workgroup = DAS_BZ wave tiles stacked in depth
// (IL: rf is the frame-interleaved copy, group g's [A][C][T][FB] record at
// the same offset, g FB frame_rf, as its first frame in the plain layout)
template <int FB, int NA, bool IL = false>
__global__ __launch_bounds__(256) void das_kernel(const DasArgs p, const DasGrid gr, const float* __restrict__ rf,
                                                  float* __restrict__ img) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int fr0 = blockIdx.z * FB;
    const size_t frame_rf = (size_t)p.A * p.C * p.T;
    const size_t frame_img = (size_t)gr.nz * gr.nx;
    das_wave<FB, NA, das_wz(NA), IL>(p, gr, (blockIdx.x * DAS_BZ + wave) * das_wz(NA), blockIdx.y * das_wx(NA),
                                     min(FB, p.n_frames - fr0), rf + fr0 * frame_rf, frame_rf, img + fr0 * frame_img,
                                     frame_img);
}

// Frame-interleaved copy of the RF for das_kernel<FB, NA, true>: frames
// 0..B-1 of [B][E] (E = A C T samples per frame) -> [G][E][FB], G = ceil(B /
// FB), frames past B zero.  A thread takes samples e + 256 k (k < S) of its
// block's 256 S: per sample FB dword reads (each coalesced over the wave) and
// FB / 4 16-byte writes (a wave writes 64 FB contiguous floats).
template <int FB, int S>
__global__ __launch_bounds__(256) void das_interleave_kernel(const float* __restrict__ rf, int32_t B, int64_t E,
                                                             float* __restrict__ out) {
    const int g = blockIdx.y;
    const int64_t e0 = (int64_t)blockIdx.x * 256 * S + threadIdx.x;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int64_t e = e0 + 256 * k;
        if (e < E) {
            float v[FB];
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const int b = g * FB + f;
                v[f] = b < B ? rf[(size_t)b * E + e] : 0.0f;
            }
            floatx4* dst = reinterpret_cast<floatx4*>(out + ((size_t)g * E + e) * FB);
#pragma unroll
            for (int q = 0; q < FB / 4; ++q) dst[q] = floatx4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
        }
    }
}

// ------------------------------------------------- fixed-delay beamformer ----
// The paper's time-invariant beamformer applied to RF (Sec. 2.3 eqn:tDAS: the
// delays of one point used for a whole line; Sec. 2.4 eqn:line_conv: fixed
// parameters along the line, scaled by Theta): row i reads every element with
// the receive law (delay and Hann weight) of its reference row r(i) in the
// same column, and is scaled by theta_i,
//   u = fs (tau_tx(x_j, z_i; a) + z_i / c - t0) + (fs / c) dx^2 / (rho_r + z_r),
// rho_r = sqrt(dx^2 + z_r^2), the receive excess written as in the DAS kernel.
// The wave tiles are DAS's, and each lane walks FD_RB rows (stride WZ) of its
// column: when every row of a wave shares one reference (the paper's one law
// per neighbourhood or per line), the law of an element is computed once and
// serves FD_RB rows, so a pair costs its index, its reads and its FMAs only;
// a wave whose rows have different references evaluates the law per row.
template <int FB, int NA, int FD_RB, bool IL = false>
__device__ __forceinline__ void fd_wave(const DasArgs& p, const DasGrid& gr, int i_base, int j_base, int nfr,
                                        const int32_t* __restrict__ ref, const float* __restrict__ theta,
                                        const float* __restrict__ rf, size_t frame_rf, float* img, size_t frame_img) {
    constexpr int WZ = das_wz(NA), WX = das_wx(NA);
    constexpr int NAM = (NA > 0) ? NA : DAS_MAX_ANGLES;
    const int lane = threadIdx.x & 63;
    const int j = j_base + lane / WZ;
    const int i_first = i_base + lane % WZ;  // the lane's rows: i_first + WZ k
    const int A = (NA > 0) ? NA : p.A;

    const double xd = gr.x0 + (double)min(j, gr.nx - 1) * gr.dx;
    const double ox = xd - p.x_first;
    const float dx0 = (float)ox, dx0_lo = (float)(ox - (double)dx0);
    const float pitch_f = (float)p.pitch, pitch_lo = (float)(p.pitch - (double)pitch_f);

    // reference row of each of the lane's rows (rows past the image, never
    // stored, take the tile's first reference), clamped into the image
    auto ref_of = [&](int i) {
        const int ii = i < gr.nz ? i : i_base;
        const int r = ref ? ref[ii] : ii;
        return min(max(r, 0), gr.nz - 1);
    };
    int rk[FD_RB];
    bool same = true;
    const int r_wave = __builtin_amdgcn_readfirstlane(ref_of(i_base));
#pragma unroll
    for (int k = 0; k < FD_RB; ++k) {
        rk[k] = ref_of(i_first + WZ * k);
        same = same && rk[k] == r_wave;
    }
    const bool uniform = __builtin_amdgcn_ballot_w64(!same) == 0;

    float acc[FD_RB][FB];
#pragma unroll
    for (int k = 0; k < FD_RB; ++k)
#pragma unroll
        for (int f = 0; f < FB; ++f) acc[k][f] = 0.0f;

    const uint32_t row_bytes = (uint32_t)p.T * 4u;
    const int last_pair = (p.T - 2) * 4;

    // the frozen law of element offset dx at reference depth zr: weight and
    // receive excess in samples
    struct Law {
        float zr, z2, inv_az;
        bool on;
    };
    auto law_at = [&](int r) {
        const double zr = gr.z0 + (double)r * gr.dz;
        Law L;
        L.zr = (float)zr;
        L.z2 = (float)(zr * zr);
        L.on = (j < gr.nx) && (zr > 0.0);
        L.inv_az = L.on ? (float)(2.0 * p.fnumber / zr) : 0.0f;
        return L;
    };
    auto weight_excess = [&](const Law& L, float dx, float& w, float& ke) {
        const float t = fabsf(dx) * L.inv_az;
        const float wh = hann_weight(fminf(t, 1.0f));
        w = (L.on && t <= 1.0f) ? wh : 0.0f;
        const float rho = __builtin_amdgcn_sqrtf(fmaf(dx, dx, L.z2));
        ke = p.kappa * (dx * dx) * __builtin_amdgcn_rcpf(rho + L.zr);
    };
    // one pair: element n's channel of angle a read at q + v for the FB frames
    auto accumulate = [&](int k, size_t ch, int q, float v, float w) {
        const float qf = floorf(v);
        const float fr = v - qf;
        const int off = (q + (int)qf) * 4;
        if constexpr (FB > 1) {
            const int oc = min(max(off, 0), last_pair);
            const int d = off - oc;
            const float wa = d == 0 ? w * (1.0f - fr) : (d == -4 ? w * fr : 0.0f);
            const float wb = d == 0 ? w * fr : (d == 4 ? w * (1.0f - fr) : 0.0f);
            if constexpr (IL) {
                // the frame-interleaved record, as in das_wave
                static_assert(FB == 4, "interleaved records hold frames in fours");
                const auto rs = make_rsrc(rf + ch * p.T * FB, row_bytes * FB);
                const floatx4 s0 = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, oc * FB, 0, 0));
                const floatx4 s1 =
                    __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, (oc + 4) * FB, 0, 0));
#pragma unroll
                for (int f = 0; f < FB; ++f) acc[k][f] = fmaf(wb, s1[f], fmaf(wa, s0[f], acc[k][f]));
            } else {
#pragma unroll
                for (int f = 0; f < FB; ++f) {
                    const bool fv = f < nfr;
                    const auto rs = make_rsrc(rf + (fv ? f : 0) * frame_rf + ch * p.T, fv ? row_bytes : 0u);
                    const floatx2 sp =
                        __builtin_bit_cast(floatx2, __builtin_amdgcn_raw_buffer_load_b64(rs, oc, 0, 0));
                    acc[k][f] = fmaf(wb, sp[1], fmaf(wa, sp[0], acc[k][f]));
                }
            }
        } else {
            const int off1 = (q + (int)(qf + 1.0f)) * 4;
            const auto rs = make_rsrc(rf + ch * p.T, nfr > 0 ? row_bytes : 0u);
            const float s0 = buffer_load_f32(rs, off);
            const float s1 = buffer_load_f32(rs, off1);
            acc[k][0] = fmaf(w, fmaf(fr, s1 - s0, s0), acc[k][0]);
        }
    };

    const double x_lo = gr.x0 + (double)j_base * gr.dx;
    const double x_hi = gr.x0 + (double)min(j_base + WX - 1, gr.nx - 1) * gr.dx;
    auto element_range = [&](double zr, int& n_lo, int& n_hi) {
        n_lo = 0;
        n_hi = -1;
        if (zr > 0.0) {
            const double a_max = zr / (2.0 * p.fnumber);
            n_lo = max(0, (int)floor((fmin(x_lo, x_hi) - a_max - p.x_first) / p.pitch));
            n_hi = min(p.C - 1, (int)ceil((fmax(x_lo, x_hi) + a_max - p.x_first) / p.pitch));
        }
    };

#pragma unroll 1
    for (int a = 0; a < A; ++a) {
        const double sa = p.sin_a[a], ca = p.cos_a[a];
        // per row: integer and fractional parts of fs (tau_tx + z/c - t0)
        int q[FD_RB];
        float fpart[FD_RB];
#pragma unroll
        for (int k = 0; k < FD_RB; ++k) {
            const double zd = gr.z0 + (double)min(i_first + WZ * k, gr.nz - 1) * gr.dz;
            const double U = p.fs * ((xd * sa + zd * ca) / p.c + zd / p.c - p.t0);
            const double Uf = floor(U);
            q[k] = (int)Uf;
            fpart[k] = (float)(U - Uf);
        }
        const size_t ch_a = (size_t)a * p.C;
        if (uniform) {
            const Law L = law_at(r_wave);
            int n_lo, n_hi;
            element_range(gr.z0 + (double)r_wave * gr.dz, n_lo, n_hi);
#pragma unroll 2
            for (int n = n_lo; n <= n_hi; ++n) {
                const float nf = (float)n;
                const float dx = fmaf(-nf, pitch_f, dx0) + fmaf(-nf, pitch_lo, dx0_lo);
                float w, ke;
                weight_excess(L, dx, w, ke);
#pragma unroll
                for (int k = 0; k < FD_RB; ++k) accumulate(k, ch_a + n, q[k], fpart[k] + ke, w);
            }
        } else {
            // the elements of the widest aperture among the wave's rows (the
            // deepest reference; weights vanish outside each row's own)
            int r_max = rk[0];
#pragma unroll
            for (int k = 1; k < FD_RB; ++k) r_max = max(r_max, rk[k]);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) r_max = max(r_max, __shfl_xor(r_max, o));
            r_max = __builtin_amdgcn_readfirstlane(r_max);
            int n_lo, n_hi;
            element_range(gr.z0 + (double)r_max * gr.dz, n_lo, n_hi);
#pragma unroll 2
            for (int n = n_lo; n <= n_hi; ++n) {
                const float nf = (float)n;
                const float dx = fmaf(-nf, pitch_f, dx0) + fmaf(-nf, pitch_lo, dx0_lo);
#pragma unroll
                for (int k = 0; k < FD_RB; ++k) {
                    float w, ke;
                    weight_excess(law_at(rk[k]), dx, w, ke);
                    accumulate(k, ch_a + n, q[k], fpart[k] + ke, w);
                }
            }
        }
    }
    if (j < gr.nx) {
#pragma unroll
        for (int k = 0; k < FD_RB; ++k) {
            const int i = i_first + WZ * k;
            if (i < gr.nz) {
                const float th = theta ? theta[i] : 1.0f;
#pragma unroll
                for (int f = 0; f < FB; ++f)
                    if (f < nfr) __builtin_nontemporal_store(th * acc[k][f], &img[f * frame_img + (size_t)i * gr.nx + j]);
            }
        }
    }
}

// workgroup = DAS_BZ wave tiles stacked in depth, each WZ x FD_RB rows
template <int FB, int NA, int FD_RB, bool IL = false>
__global__ __launch_bounds__(256) void fixed_das_kernel(const DasArgs p, const DasGrid gr, const int32_t* __restrict__ ref,
                                                        const float* __restrict__ theta, const float* __restrict__ rf,
                                                        float* __restrict__ img) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int fr0 = blockIdx.z * FB;
    const size_t frame_rf = (size_t)p.A * p.C * p.T;
    const size_t frame_img = (size_t)gr.nz * gr.nx;
    const int i_base = (blockIdx.x * DAS_BZ + wave) * das_wz(NA) * FD_RB;
    if (i_base >= gr.nz) return;
    fd_wave<FB, NA, FD_RB, IL>(p, gr, i_base, blockIdx.y * das_wx(NA), min(FB, p.n_frames - fr0), ref, theta,
                               rf + fr0 * frame_rf, frame_rf, img + fr0 * frame_img, frame_img);
}

// ----------------------------------------------------------------- batches ----
// Ragged batch: every frame has its own grid, RF record and image.  One
// persistent launch covers the tiles (WAVES wave tiles stacked in depth) of
// all frames.
// The tile list is cut into 8 contiguous chunks, chunk x served by the
// workgroups the hardware places on XCD x (block id = x mod 8), so each frame's
// RF stays in one XCD's L2.  Every workgroup walks its chunk with a fixed
// stride: the loop always ends.
struct BatchFrameDev {
    DasGrid grid;
    const float* rf;
    const float* kernels;
    const float* in;
    float* out;
    int64_t tile_start;  // prefix sum of tiles before this frame (op specific)
};

__device__ __forceinline__ int find_frame(const BatchFrameDev* __restrict__ fr, int n, int64_t t) {
    int lo = 0, hi = n - 1;  // largest f with tile_start[f] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fr[mid].tile_start <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NA, int WAVES, int WZ>
__global__ __launch_bounds__(WAVES * 64) void das_batch_kernel(const DasArgs p, const BatchFrameDev* __restrict__ fr,
                                                               int32_t n_frames, int64_t total) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int nblk = gridDim.x;
    const int per_xcd = (nblk - x + 7) >> 3;  // workgroups on this XCD
    const int64_t lo = total * x / 8, hi = total * (x + 1) / 8;
    for (int64_t t = lo + slot; t < hi; t += per_xcd) {
        const int f = find_frame(fr, n_frames, t);
        const DasGrid gr = fr[f].grid;
        const int64_t local = t - fr[f].tile_start;
        // tile of WAVES wave tiles (WZ x 64 / WZ pixels) stacked in depth
        const int row_tiles = (gr.nz + WAVES * WZ - 1) / (WAVES * WZ);
        const int rt = (int)(local % row_tiles);
        const int ct = (int)(local / row_tiles);
        const int i_base = (rt * WAVES + wave) * WZ;
        if (i_base < gr.nz) das_wave<1, NA, WZ>(p, gr, i_base, ct * (64 / WZ), 1, fr[f].rf, 0, fr[f].out, 0);
    }
}

template <int FB, int NA, bool IL = false>
static void launch_das(const DasArgs& p, const DasGrid& gr, const float* rf, float* img, hipStream_t s) {
    dim3 grid((gr.nz + DAS_BZ * das_wz(NA) - 1) / (DAS_BZ * das_wz(NA)), (gr.nx + das_wx(NA) - 1) / das_wx(NA),
              (p.n_frames + FB - 1) / FB);
    hipLaunchKernelGGL((das_kernel<FB, NA, IL>), grid, dim3(256), 0, s, p, gr, rf, img);
}

// Frames per interleaved group and the copy's bytes (0: the call reads the
// RF in place: one frame per thread, or several angles).
constexpr int DAS_IL_FB = 4;
static size_t das_il_bytes(int32_t A, int32_t C, int32_t T, int32_t n_frames) {
    const int64_t groups = (n_frames + DAS_IL_FB - 1) / DAS_IL_FB;
    return ((size_t)groups * DAS_IL_FB * A * C * T * sizeof(float) + 255) / 256 * 256;
}
// the interleaved channel record (T FB floats) and its byte offsets fit 31 bits
static bool das_il_fits(int32_t T) { return (int64_t)T * 4 * DAS_IL_FB + 64 < ((int64_t)1 << 31); }
// which calls read the RF through the copy: eight or more frames of one plane
// wave, or (DAS) of the 11-angle compounding the batch kernels serve
// (the groups are the launches' third grid dimension: at most 65535)
static bool das_uses_il(int32_t A, int32_t T, int32_t n_frames) {
    return (A == 1 || A == 11) && n_frames >= 8 && n_frames <= 4 * 65535 && das_il_fits(T);
}
static bool fd_uses_il(int32_t A, int32_t T, int32_t n_frames) {
    return A == 1 && n_frames >= 8 && n_frames <= 4 * 65535 && das_il_fits(T);
}
// two samples per thread: measured on 64 frames of 128 x 4096 samples, 39 us
// (6.8 TB/s of the copy's read and write) against 42 us for one and 40 us for
// four; a variant reading four samples per 16-byte load and transposing in
// registers took 62 us (its 16-byte writes strided 64 bytes apart)
static void launch_interleave(const float* rf, int32_t B, int64_t E, float* il, hipStream_t s) {
    constexpr int S = 2;
    const dim3 grid((unsigned)((E + 256 * S - 1) / (256 * S)), (unsigned)((B + DAS_IL_FB - 1) / DAS_IL_FB));
    hipLaunchKernelGGL((das_interleave_kernel<DAS_IL_FB, S>), grid, dim3(256), 0, s, rf, B, E, il);
}

template <int FB, int NA, int FD_RB>
static void launch_fixed_das(const DasArgs& p, const DasGrid& gr, const int32_t* ref, const float* theta,
                             const float* rf, float* img, hipStream_t s) {
    const int rows_per_wg = DAS_BZ * das_wz(NA) * FD_RB;
    dim3 grid((gr.nz + rows_per_wg - 1) / rows_per_wg, (gr.nx + das_wx(NA) - 1) / das_wx(NA),
              (p.n_frames + FB - 1) / FB);
    hipLaunchKernelGGL((fixed_das_kernel<FB, NA, FD_RB>), grid, dim3(256), 0, s, p, gr, ref, theta, rf, img);
}

// Shared validation and argument set-up of the DAS entry points.
static int32_t das_setup(const char* name, const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                         int32_t n_samples, DasArgs& p) {
    int32_t st;
    if ((st = validate_array(array)) || (st = validate_tx(tx, false)) || (st = validate_rx(rx))) return st;
    if (n_samples < 2) return fail(TIDAS_EINVAL, std::string(name) + ": n_samples must be >= 2");
    if (tx->n_angles > DAS_MAX_ANGLES) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": at most 32 angles");
    if ((int64_t)n_samples * 4 > INT32_MAX / 2) return fail(TIDAS_EUNSUPPORTED, std::string(name) + ": record too long");
    p = DasArgs{};
    p.C = array->n_elem;
    p.T = n_samples;
    p.A = tx->n_angles;
    p.n_frames = 1;
    p.pitch = array->pitch;
    p.c = array->c;
    p.fs = tx->fs;
    p.t0 = tx->t0;
    p.fnumber = rx->fnumber;
    p.x_first = -0.5 * (double)(p.C - 1) * p.pitch;
    p.kappa = (float)(p.fs / p.c);
    for (int a = 0; a < p.A; ++a) {
        p.sin_a[a] = std::sin(tx->angles[a]);
        p.cos_a[a] = std::cos(tx->angles[a]);
    }
    return TIDAS_OK;
}

// Every fractional sample index of the grid must stay far inside int32 (byte offsets = 4 x index).
static bool das_grid_in_range(const DasArgs& p, const tidas_grid* grid) {
    const double half_w = 0.5 * (double)(p.C - 1) * p.pitch;
    const double xmax = std::fabs(grid->x0) + std::fabs(grid->x0 + (grid->nx - 1) * grid->dx) + half_w;
    const double zmax = std::fabs(grid->z0) + std::fabs(grid->z0 + (grid->nz - 1) * grid->dz);
    const double bound = p.fs * (2.0 * xmax + 2.0 * zmax) / p.c + p.fs * std::fabs(p.t0) + 2.0;
    return bound < 268435456.0;
}

static DasGrid to_grid(const tidas_grid* g) { return DasGrid{g->nz, g->nx, g->z0, g->dz, g->x0, g->dx}; }

}  // namespace tidas

using namespace tidas;

extern "C" size_t das_beamform_workspace_bytes(int32_t n_angles, int32_t n_elem, int32_t n_samples,
                                               int32_t n_frames) {
    if (n_angles < 1 || n_elem < 1 || n_samples < 2 || n_frames < 1 || !das_uses_il(n_angles, n_samples, n_frames))
        return 0;
    return das_il_bytes(n_angles, n_elem, n_samples, n_frames);
}

extern "C" int32_t das_beamform(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                                const tidas_grid* grid, const float* rf, int32_t n_samples,
                                int32_t n_frames, float* image, void* workspace, size_t workspace_bytes,
                                void* stream) {
    DasArgs p;
    int32_t st = das_setup("das_beamform", array, tx, rx, n_samples, p);
    if (st) return st;
    if ((st = validate_grid(grid))) return st;
    if (!rf || !image) return fail(TIDAS_EINVAL, "das_beamform: null rf or image pointer");
    if (n_frames < 1) return fail(TIDAS_EINVAL, "das_beamform: n_frames must be >= 1");
    if ((const void*)rf == (const void*)image) return fail(TIDAS_EINVAL, "das_beamform: image aliases rf");
    if (!das_grid_in_range(p, grid)) return fail(TIDAS_EUNSUPPORTED, "das_beamform: sample indices exceed 2^28");
    const size_t need = das_uses_il(p.A, p.T, n_frames) ? das_il_bytes(p.A, p.C, p.T, n_frames) : 0;
    if ((st = workspace_check("das_beamform", workspace, workspace_bytes, need))) return st;
    p.n_frames = n_frames;
    const DasGrid gr = to_grid(grid);
    hipStream_t s = (hipStream_t)stream;
    // several frames per thread amortise the geometry over a batch; their
    // samples are read four frames per 16-byte load from an interleaved copy
    if (need) {
        Workspace w;
        if ((st = workspace_acquire("das_beamform", workspace, need, s, w))) return st;
        float* il = reinterpret_cast<float*>(w.ptr);
        const int64_t E = (int64_t)p.A * p.C * p.T;
        launch_interleave(rf, n_frames, E, il, s);
        if (p.A == 1) launch_das<DAS_IL_FB, 1, true>(p, gr, il, image, s);
        else launch_das<DAS_IL_FB, 11, true>(p, gr, il, image, s);
        if ((st = check_launch("das_beamform"))) {
            workspace_release("das_beamform", w, s);
            return st;
        }
        return workspace_release("das_beamform", w, s);
    }
    const bool multi = n_frames >= 8;
    if (p.A == 1) {
        if (multi) launch_das<4, 1>(p, gr, rf, image, s);
        else launch_das<1, 1>(p, gr, rf, image, s);
    } else if (p.A == 11) {
        launch_das<1, 11>(p, gr, rf, image, s);
    } else {
        launch_das<1, 0>(p, gr, rf, image, s);
    }
    return check_launch("das_beamform");
}

extern "C" size_t tidas_beamform_workspace_bytes(int32_t n_angles, int32_t n_elem, int32_t n_samples,
                                                 int32_t n_frames) {
    if (n_angles < 1 || n_elem < 1 || n_samples < 2 || n_frames < 1 || !fd_uses_il(n_angles, n_samples, n_frames))
        return 0;
    return das_il_bytes(n_angles, n_elem, n_samples, n_frames);
}

extern "C" int32_t tidas_beamform(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                                  const tidas_grid* grid, const float* rf, int32_t n_samples, int32_t n_frames,
                                  const int32_t* ref_row, const float* theta, float* image, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    DasArgs p;
    int32_t st = das_setup("tidas_beamform", array, tx, rx, n_samples, p);
    if (st) return st;
    if ((st = validate_grid(grid))) return st;
    if (!rf || !image) return fail(TIDAS_EINVAL, "tidas_beamform: null rf or image pointer");
    if (n_frames < 1) return fail(TIDAS_EINVAL, "tidas_beamform: n_frames must be >= 1");
    if ((const void*)rf == (const void*)image || (const void*)theta == (const void*)image ||
        (const void*)ref_row == (const void*)image)
        return fail(TIDAS_EINVAL, "tidas_beamform: image aliases an input");
    if (!das_grid_in_range(p, grid)) return fail(TIDAS_EUNSUPPORTED, "tidas_beamform: sample indices exceed 2^28");
    const size_t need = fd_uses_il(p.A, p.T, n_frames) ? das_il_bytes(p.A, p.C, p.T, n_frames) : 0;
    if ((st = workspace_check("tidas_beamform", workspace, workspace_bytes, need))) return st;
    p.n_frames = n_frames;
    const DasGrid gr = to_grid(grid);
    hipStream_t s = (hipStream_t)stream;
    if (need) {
        // groups of four frames read from the interleaved copy, as DAS; two
        // rows per lane share the frozen law (measured on 64 frames of 1024 x
        // 256, 128 elements: 0.39-0.45 ms with one law per 64 rows or per row,
        // one row per lane the same)
        Workspace w;
        if ((st = workspace_acquire("tidas_beamform", workspace, need, s, w))) return st;
        float* il = reinterpret_cast<float*>(w.ptr);
        launch_interleave(rf, n_frames, (int64_t)p.A * p.C * p.T, il, s);
        constexpr int RB = 2;
        const int rows_per_wg = DAS_BZ * das_wz(1) * RB;
        const dim3 grid((gr.nz + rows_per_wg - 1) / rows_per_wg, (gr.nx + das_wx(1) - 1) / das_wx(1),
                        (n_frames + DAS_IL_FB - 1) / DAS_IL_FB);
        hipLaunchKernelGGL((fixed_das_kernel<DAS_IL_FB, 1, RB, true>), grid, dim3(256), 0, s, p, gr, ref_row, theta,
                           il, image);
        if ((st = check_launch("tidas_beamform"))) {
            workspace_release("tidas_beamform", w, s);
            return st;
        }
        return workspace_release("tidas_beamform", w, s);
    }
    // one frame per thread: rows per lane share the law when their references
    // agree; measured on 64 frames of 1024 x 256, 128 elements, one law per
    // 64 rows, before the interleaved copy: 4 frames x 2 rows 0.64 ms, x 4
    // rows 0.78, x 8 rows 0.82 (166 registers)
    if (p.A == 1) {
        launch_fixed_das<1, 1, 4>(p, gr, ref_row, theta, rf, image, s);
    } else if (p.A == 11) {
        launch_fixed_das<1, 11, 4>(p, gr, ref_row, theta, rf, image, s);
    } else {
        launch_fixed_das<1, 0, 4>(p, gr, ref_row, theta, rf, image, s);
    }
    return check_launch("tidas_beamform");
}

// ------------------------------------------------------------------ batch ----
namespace tidas {


int32_t validate_batch(const char* name, const tidas_frame* frames, int32_t n_frames, void* workspace,
                       size_t workspace_bytes, bool need_rf, bool need_conv) {
    if (!frames || !workspace) return fail(TIDAS_EINVAL, std::string(name) + ": null frames or workspace");
    if (n_frames < 1) return fail(TIDAS_EINVAL, std::string(name) + ": n_frames must be >= 1");
    if (workspace_bytes < tidas_batch_workspace_bytes(n_frames))
        return fail(TIDAS_EINVAL, std::string(name) + ": workspace too small");
    if ((reinterpret_cast<uintptr_t>(workspace) & 15) != 0)
        return fail(TIDAS_EINVAL, std::string(name) + ": workspace must be 16-byte aligned");
    for (int f = 0; f < n_frames; ++f) {
        int32_t st = validate_grid(&frames[f].grid);
        if (st) return st;
        if (!frames[f].out) return fail(TIDAS_EINVAL, std::string(name) + ": null output pointer");
        if (need_rf && !frames[f].rf) return fail(TIDAS_EINVAL, std::string(name) + ": null rf pointer");
        if (need_conv && (!frames[f].kernels || !frames[f].in))
            return fail(TIDAS_EINVAL, std::string(name) + ": null kernels or input pointer");
    }
    return TIDAS_OK;
}

// Builds the device table: host staging vector -> workspace.  hipMemcpyAsync
// from pageable memory returns only once the source has been staged, so the
// vector may go out of scope when this returns.
int32_t upload_batch(const tidas_frame* frames, int32_t n_frames, int tile_rows, int tile_cols, void* workspace,
                     hipStream_t s, int64_t& total) {
    std::vector<BatchFrameDev> tab(n_frames);
    total = 0;
    for (int f = 0; f < n_frames; ++f) {
        const tidas_grid& g = frames[f].grid;
        tab[f].grid = to_grid(&g);
        tab[f].rf = frames[f].rf;
        tab[f].kernels = frames[f].kernels;
        tab[f].in = frames[f].in;
        tab[f].out = frames[f].out;
        tab[f].tile_start = total;
        total += (int64_t)((g.nz + tile_rows - 1) / tile_rows) * ((g.nx + tile_cols - 1) / tile_cols);
    }
    return check_hip(hipMemcpyAsync(workspace, tab.data(), sizeof(BatchFrameDev) * n_frames, hipMemcpyHostToDevice, s),
                     "batch table upload");
}

}  // namespace tidas

static_assert(sizeof(tidas::BatchFrameDev) <= 128, "batch table entry too large");

extern "C" size_t tidas_batch_workspace_bytes(int32_t n_frames) {
    return n_frames < 1 ? 0 : ((128 * (size_t)n_frames + 255) / 256) * 256;
}

template <int NA>
static void launch_das_batch(int wz, int waves, unsigned nblk, hipStream_t s, const DasArgs& p,
                             const BatchFrameDev* tab, int32_t n_frames, int64_t total) {
    const dim3 grid(nblk), block(waves * 64);
    if (waves == 8) {
        if (wz == 1) hipLaunchKernelGGL((das_batch_kernel<NA, 8, 1>), grid, block, 0, s, p, tab, n_frames, total);
        else if (wz == 2) hipLaunchKernelGGL((das_batch_kernel<NA, 8, 2>), grid, block, 0, s, p, tab, n_frames, total);
        else hipLaunchKernelGGL((das_batch_kernel<NA, 8, 4>), grid, block, 0, s, p, tab, n_frames, total);
    } else {
        if (wz == 1) hipLaunchKernelGGL((das_batch_kernel<NA, 4, 1>), grid, block, 0, s, p, tab, n_frames, total);
        else if (wz == 2) hipLaunchKernelGGL((das_batch_kernel<NA, 4, 2>), grid, block, 0, s, p, tab, n_frames, total);
        else hipLaunchKernelGGL((das_batch_kernel<NA, 4, 4>), grid, block, 0, s, p, tab, n_frames, total);
    }
}

extern "C" int32_t das_beamform_batch(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                                      int32_t n_samples, const tidas_frame* frames, int32_t n_frames,
                                      void* workspace, size_t workspace_bytes, int32_t variant, void* stream) {
    DasArgs p;
    int32_t st = das_setup("das_beamform_batch", array, tx, rx, n_samples, p);
    if (st) return st;
    if ((st = validate_batch("das_beamform_batch", frames, n_frames, workspace, workspace_bytes, true, false)))
        return st;
    for (int f = 0; f < n_frames; ++f)
        if (!das_grid_in_range(p, &frames[f].grid))
            return fail(TIDAS_EUNSUPPORTED, "das_beamform_batch: sample indices exceed 2^28");
    if (variant < 0 || variant >= TIDAS_DAS_BATCH_VARIANTS)
        return fail(TIDAS_EINVAL, "das_beamform_batch: variant out of range");
    // variant = 6 shape + occupancy: wave tile 1 x 64, 2 x 32 or 4 x 16 pixels;
    // 4 or 8 waves per workgroup; 2, 4 or 8 workgroups per compute unit
    const int wz = 1 << (variant / 6);
    const int waves = (variant & 1) ? 8 : 4;
    const int per_cu = ((variant % 6) >> 1) == 0 ? 2 : (((variant % 6) >> 1) == 1 ? 4 : 8);
    hipStream_t s = (hipStream_t)stream;
    int64_t total = 0;
    if ((st = upload_batch(frames, n_frames, waves * wz, 64 / wz, workspace, s, total))) return st;
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
    }
    const int64_t want = (int64_t)n_cu * per_cu;  // workgroups of the persistent launch
    // a multiple of 8 workgroups: the tile list is cut into 8 chunks, one per
    // residue of the block id, and every chunk needs at least one workgroup
    const int64_t nb = std::max<int64_t>(8, std::min<int64_t>(total, want));
    const unsigned nblk = (unsigned)((nb + 7) / 8 * 8);
    const BatchFrameDev* tab = (const BatchFrameDev*)workspace;
    if (p.A == 11) launch_das_batch<11>(wz, waves, nblk, s, p, tab, n_frames, total);
    else if (p.A == 1) launch_das_batch<1>(wz, waves, nblk, s, p, tab, n_frames, total);
    else launch_das_batch<0>(wz, waves, nblk, s, p, tab, n_frames, total);
    return check_launch("das_beamform_batch");
}
