// Exact Delay-and-Sum beamformer for plane-wave transmits (Sec. 2, eqn:appF).
//
// Mapping on gfx950: one wavefront = 64 consecutive depth rows of ONE image
// column, a workgroup = 4 columns.  For a fixed element n the 64 lanes then
// read a short, nearly contiguous window of that element's channel (the
// sample index grows by ~2 dz fs / c per row), so the channel-major RF reads
// coalesce into a few cache lines per wave, and the lateral offset
// x_j - x_n is the same for the whole wave.
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
// Each thread can beamform FB frames that share the geometry: delays and
// apodization are computed once per (pixel, element) and reused.
#include "common.hpp"

namespace tidas {

constexpr int DAS_MAX_ANGLES = 32;

struct DasArgs {
    int32_t C, T, A, nz, nx, n_frames;
    double pitch, fs, t0, fnumber, z0, dz, x0, dx, c;
    double x_first;    // x of element 0
    float kappa;       // fs / c
    double sin_a[DAS_MAX_ANGLES];
    double cos_a[DAS_MAX_ANGLES];
};

template <int FB, int NA>
__global__ __launch_bounds__(256) void das_kernel(const DasArgs p, const float* __restrict__ rf,
                                                  float* __restrict__ img) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = blockIdx.y * 4 + wave;
    if (j >= p.nx) return;
    const int i = blockIdx.x * 64 + lane;
    const int fr0 = blockIdx.z * FB;
    const int A = (NA > 0) ? NA : p.A;

    const double xd = p.x0 + (double)j * p.dx;
    const double zd = p.z0 + (double)min(i, p.nz - 1) * p.dz;
    const bool active = (i < p.nz) && (zd > 0.0);
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

    // element range covering the widest aperture among this wave's rows
    const int i_last = min((int)blockIdx.x * 64 + 63, p.nz - 1);
    const double z_last = p.z0 + (double)i_last * p.dz;
    int n_lo = 0, n_hi = -1;
    if (z_last > 0.0) {
        const double a_max = z_last / (2.0 * p.fnumber);
        n_lo = max(0, (int)floor((xd - a_max - p.x_first) / p.pitch));
        n_hi = min(p.C - 1, (int)ceil((xd + a_max - p.x_first) / p.pitch));
    }

    float acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = 0.0f;

    const uint32_t row_bytes = (uint32_t)p.T * 4u;
    for (int n = n_lo; n <= n_hi; ++n) {
        const float dx = (float)(xd - (p.x_first + (double)n * p.pitch));
        const float t = fabsf(dx) * inv_az;
        if (active && t <= 1.0f) {
            const float w = hann_weight(t);
            const float rho = __builtin_amdgcn_sqrtf(fmaf(dx, dx, z2));
            const float ke = p.kappa * (dx * dx) * __builtin_amdgcn_rcpf(rho + zf);
#pragma unroll
            for (int a = 0; a < ((NA > 0) ? NA : DAS_MAX_ANGLES); ++a) {
                if (a < A) {
                    const float v = f_a[a] + ke;
                    const float qf = floorf(v);
                    const float fr = v - qf;
                    const int off = (q_a[a] + (int)qf) * 4;
#pragma unroll
                    for (int f = 0; f < FB; ++f) {
                        if (fr0 + f < p.n_frames) {
                            const size_t ch = ((size_t)(fr0 + f) * A + a) * p.C + n;
                            const auto rs = make_rsrc(rf + ch * p.T, row_bytes);
                            const float s0 = buffer_load_f32(rs, off);
                            const float s1 = buffer_load_f32(rs, off + 4);
                            acc[f] = fmaf(w, fmaf(fr, s1 - s0, s0), acc[f]);
                        }
                    }
                }
            }
        }
    }
    if (i < p.nz) {
#pragma unroll
        for (int f = 0; f < FB; ++f)
            if (fr0 + f < p.n_frames) img[((size_t)(fr0 + f) * p.nz + i) * p.nx + j] = acc[f];
    }
}

template <int FB, int NA>
static void launch_das(const DasArgs& p, const float* rf, float* img, hipStream_t s) {
    dim3 grid((p.nz + 63) / 64, (p.nx + 3) / 4, (p.n_frames + FB - 1) / FB);
    hipLaunchKernelGGL((das_kernel<FB, NA>), grid, dim3(256), 0, s, p, rf, img);
}

}  // namespace tidas

using namespace tidas;

extern "C" int32_t das_beamform(const tidas_array* array, const tidas_tx* tx, const tidas_rx* rx,
                                const tidas_grid* grid, const float* rf, int32_t n_samples,
                                int32_t n_frames, float* image, void* stream) {
    int32_t st;
    if ((st = validate_array(array)) || (st = validate_tx(tx, false)) || (st = validate_rx(rx)) ||
        (st = validate_grid(grid)))
        return st;
    if (!rf || !image) return fail(TIDAS_EINVAL, "das_beamform: null rf or image pointer");
    if (n_samples < 2) return fail(TIDAS_EINVAL, "das_beamform: n_samples must be >= 2");
    if (n_frames < 1) return fail(TIDAS_EINVAL, "das_beamform: n_frames must be >= 1");
    if (tx->n_angles > DAS_MAX_ANGLES)
        return fail(TIDAS_EUNSUPPORTED, "das_beamform: at most 32 plane-wave angles");
    if ((const void*)rf == (const void*)image) return fail(TIDAS_EINVAL, "das_beamform: image aliases rf");
    if ((int64_t)n_samples * 4 > INT32_MAX / 2) return fail(TIDAS_EUNSUPPORTED, "das_beamform: record too long");

    {
        // every fractional sample index must stay far inside int32 (byte offsets = 4 x index)
        const double half_w = 0.5 * (double)(array->n_elem - 1) * array->pitch;
        const double xmax = std::fabs(grid->x0) + std::fabs(grid->x0 + (grid->nx - 1) * grid->dx) + half_w;
        const double zmax = std::fabs(grid->z0) + std::fabs(grid->z0 + (grid->nz - 1) * grid->dz);
        const double bound = tx->fs * (2.0 * xmax + 2.0 * zmax) / array->c + tx->fs * std::fabs(tx->t0) + 2.0;
        if (!(bound < 268435456.0)) return fail(TIDAS_EUNSUPPORTED, "das_beamform: sample indices exceed 2^28");
    }
    DasArgs p{};
    p.C = array->n_elem;
    p.T = n_samples;
    p.A = tx->n_angles;
    p.nz = grid->nz;
    p.nx = grid->nx;
    p.n_frames = n_frames;
    p.pitch = array->pitch;
    p.c = array->c;
    p.fs = tx->fs;
    p.t0 = tx->t0;
    p.fnumber = rx->fnumber;
    p.z0 = grid->z0;
    p.dz = grid->dz;
    p.x0 = grid->x0;
    p.dx = grid->dx;
    p.x_first = -0.5 * (double)(p.C - 1) * p.pitch;
    p.kappa = (float)(p.fs / p.c);
    for (int a = 0; a < p.A; ++a) {
        p.sin_a[a] = std::sin(tx->angles[a]);
        p.cos_a[a] = std::cos(tx->angles[a]);
    }
    hipStream_t s = (hipStream_t)stream;
    // several frames per thread amortise the geometry over a batch
    const bool multi = n_frames >= 8;
    if (p.A == 1) {
        if (multi) launch_das<4, 1>(p, rf, image, s);
        else launch_das<1, 1>(p, rf, image, s);
    } else if (p.A == 11) {
        launch_das<1, 11>(p, rf, image, s);
    } else {
        launch_das<1, 0>(p, rf, image, s);
    }
    return check_launch("das_beamform");
}
