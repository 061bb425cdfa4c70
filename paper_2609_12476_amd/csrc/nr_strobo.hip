// Stroboscopic-resampling baseline: nearest-neighbour reading of an
// oversampled segment on a uniform grid in the resampled time of
// Eq. (new_t), folded for an FFT at the requested bin spacing.  The grid
// times and nearest indices are computed in FP64 with the operations in a
// fixed order (no fused multiply-adds), so the integer decisions are those
// of the plain evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/nr_strobo.h"
#include "nr_params.hpp"

namespace {

thread_local std::string g_strobo_error;

nr_status fail(const std::string& m, nr_status st)
{
    g_strobo_error = m;
    return st;
}

// One thread per fold slot r of segment blockIdx.y: the grid points r,
// r + fold, ... < M.
template <bool CPLX>
__global__ __launch_bounds__(256) void fold_kernel(const float* __restrict__ x, int64_t n, double fs_o, double a,
                                                   double tscale, int identity, int64_t M, int64_t fold,
                                                   float2* __restrict__ out)
{
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= fold) return;
    x += (int64_t)blockIdx.y * n * (CPLX ? 2 : 1);
    out += (int64_t)blockIdx.y * fold;
    float re = 0.0f, im = 0.0f;
    for (int64_t m = r; m < M; m += fold) {
        const double tau = (double)m / fs_o;
        const double t = identity ? tau : -expm1(1.6 * log1p(-tau / a)) * tscale;
        const double q = rint(t * fs_o);
        if (q >= 0.0 && q < (double)n) {
            const int64_t s = (int64_t)q;
            if (CPLX) {
                re += x[2 * s];
                im += x[2 * s + 1];
            } else {
                re += x[s];
            }
        }
    }
    out[r] = make_float2(re, im);
}

// The grid of the segment: M and the constants of the inverse time map.
struct Grid {
    int64_t M;
    double a, tscale;
    int identity;
};

nr_status make_grid(double fs_o, int64_t n, double mc, double f0, Grid& g)
{
    if (!(std::isfinite(fs_o) && fs_o > 0.0) || n < 1 || !(std::isfinite(mc) && mc >= 0.0) ||
        !(std::isfinite(f0) && f0 > 0.0))
        return fail("fs_o, f0 must be positive, mc >= 0 and n_samples >= 1", NR_ERR_INVALID_ARG);
    const double b = mc > 0.0 ? nr::chirp_beta(mc, f0) : 0.0;
    const double t_last = (double)(n - 1) / fs_o;
    g.identity = b == 0.0;
    if (g.identity) {
        g.M = n;
        g.a = 0.0;
        g.tscale = 0.0;
        return NR_OK;
    }
    if (!(1.0 - (8.0 / 3.0) * b * t_last > 0.0)) return fail("the segment reaches coalescence", NR_ERR_INVALID_ARG);
    g.a = 3.0 / (5.0 * b);
    g.tscale = 3.0 / (8.0 * b);
    const double dtau_max = g.a * (-std::expm1(0.625 * std::log1p(-(8.0 / 3.0) * b * t_last)));
    g.M = (int64_t)std::floor(dtau_max * fs_o) + 1;
    return NR_OK;
}

}  // namespace

extern "C" {

nr_status nr_strobo_points(double fs_o, int64_t n_samples, double mc_msun, double f0, int64_t* m_out)
{
    if (!m_out) return fail("m_out is NULL", NR_ERR_INVALID_ARG);
    Grid g{};
    const nr_status st = make_grid(fs_o, n_samples, mc_msun, f0, g);
    if (st == NR_OK) *m_out = g.M;
    return st;
}

nr_status nr_strobo_fold(const void* x, int32_t x_complex, int64_t n_samples, int32_t n_seg, double fs_o,
                         double mc_msun, double f0, int64_t fold, void* out, void* stream)
{
    if (!x || !out) return fail("x and out must not be NULL", NR_ERR_INVALID_ARG);
    if (n_seg < 1 || n_seg > 65535) return fail("n_seg must be in [1, 65535]", NR_ERR_INVALID_ARG);
    if (fold < 1 || fold > (int64_t(1) << 34)) return fail("fold must be in [1, 2^34]", NR_ERR_INVALID_ARG);
    Grid g{};
    const nr_status st = make_grid(fs_o, n_samples, mc_msun, f0, g);
    if (st != NR_OK) return st;
    const dim3 blocks((unsigned)((fold + 255) / 256), (unsigned)n_seg);
    hipStream_t s = (hipStream_t)stream;
    if (x_complex)
        fold_kernel<true><<<blocks, 256, 0, s>>>((const float*)x, n_samples, fs_o, g.a, g.tscale, g.identity, g.M,
                                                 fold, (float2*)out);
    else
        fold_kernel<false><<<blocks, 256, 0, s>>>((const float*)x, n_samples, fs_o, g.a, g.tscale, g.identity, g.M,
                                                  fold, (float2*)out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(std::string("fold: ") + hipGetErrorString(e), NR_ERR_DEVICE);
    return NR_OK;
}

const char* nr_strobo_last_error(void) { return g_strobo_error.c_str(); }

}  // extern "C"
