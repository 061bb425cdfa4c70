// Weighted stack-slide along 0PN frequency tracks through stored per-segment
// power spectra: the semicoherent statistic of Sec. III.C,
// Eq. (semicoherent_statistic), with the Eq. (weights) weighting for white
// noise.  The track geometry (segment, beta template, bin and weight for each
// lag of each (chirp mass, start offset)) is computed once per plan in FP64;
// the statistic itself is a gather of one power value per (track, segment)
// and an FP64 multiply-add, so the execute kernel is bound by memory traffic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "../../include/nr_stackslide.h"
#include "nr_params.hpp"

namespace {

thread_local std::string g_ss_error;

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kTile = 32;

// One lag of one (chirp mass, start offset) track family.
struct SsEntry {
    int32_t k;       // bank template
    int32_t j;       // bin
    double w;        // unnormalised weight f^{4/3}
    double w2sum;    // running sum of w^2 through this lag
};

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Track tables: one thread per (chirp mass c, start offset s) walks the lags
// m = 0, 1, ... of the tracks t0 = (i0 - s/S) t_coh; lag m is the segment
// (m + s/S) t_coh after t0.  The arithmetic that decides integers (end of
// track, bin, template) is written operation by operation, without fused
// multiply-adds.
__global__ void tables_kernel(const double* __restrict__ beta_start, const double* __restrict__ bank, int n_beta,
                              int n_mc, int S, int n_seg, int n_bins, double t_coh, double f_lo, double df,
                              double f_start, double f_max, SsEntry* __restrict__ tab, int32_t* __restrict__ len)
{
#pragma clang fp contract(off)
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)n_mc * S) return;
    const int c = (int)(id / S), s = (int)(id % S);
    const double b0 = beta_start[c];
    SsEntry* row = tab + id * n_seg;
    double w2 = 0.0;
    int m = 0;
    for (; m < n_seg; ++m) {
        const double dt = ((double)m + (double)s / (double)S) * t_coh;
        const double u = 1.0 - (8.0 / 3.0) * b0 * dt;
        if (!(u > 0.0)) break;
        const double f = f_start * pow(u, -3.0 / 8.0);
        if (f > f_max) break;
        const double jf = floor((f - f_lo) / df + 0.5);
        if (jf < 0.0 || jf >= (double)n_bins) break;
        const double b = b0 / u;
        int lo = 0, hi = n_beta;  // first bank entry >= b
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (bank[mid] < b) lo = mid + 1; else hi = mid;
        }
        int k;
        if (lo == 0)
            k = 0;
        else if (lo == n_beta)
            k = n_beta - 1;
        else
            k = (fabs(bank[lo - 1] - b) <= fabs(bank[lo] - b)) ? lo - 1 : lo;
        const double w = pow(f, 4.0 / 3.0);
        w2 += w * w;
        row[m] = SsEntry{k, (int32_t)jf, w, w2};
    }
    len[id] = m;
}

// One wave per (chirp mass, start offset, 64 consecutive start segments i0):
// the lags' table entries are the same for every lane (scalar loads), and in
// layout 1 the lanes read 64 consecutive segments of one (template, bin).
// ACC: only the segments of [seg_lo, seg_hi) take part, the power buffer
// holds exactly those (segment i at position i - seg_lo, n_buf = seg_hi -
// seg_lo of them), and out and used are accumulated into (+=).  The weights
// are normalised over the whole track, so the partial sums of consecutive
// segment ranges add up to the statistic of the whole track.  Otherwise the
// buffer holds every segment and out and used are written.
template <int LAYOUT, bool ACC>
__global__ __launch_bounds__(kBlock) void gather_kernel(const float* __restrict__ P, const SsEntry* __restrict__ tab,
                                                        const int32_t* __restrict__ len, int64_t n_fam, int S,
                                                        int n_seg, int n_bins, int chunks, int seg_lo, int seg_hi,
                                                        double a, double b, float* __restrict__ out,
                                                        int32_t* __restrict__ used)
{
    const int64_t wid = uniform64(((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave);
    if (wid >= n_fam * chunks) return;  // whole waves
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t cs = wid / chunks;
    const int chunk = (int)(wid % chunks);
    const int i0 = chunk * kWave + lane;
    const int M = len[cs];
    const SsEntry* __restrict__ row = tab + cs * n_seg;
    // the whole array (ACC false) needs no range tests: every lag below lim is in it
    const int lo = ACC ? seg_lo : 0, hi = ACC ? seg_hi : n_seg;
    const int n_buf = hi - lo;
    const int lim = n_seg - i0;                       // lags this lane may take
    // lags of the wave's lanes that land in [lo, hi)
    const int m_lo = ACC ? max(0, lo - (chunk * kWave + kWave - 1)) : 0;
    const int m_hi = min(min(M, n_seg - chunk * kWave), hi - chunk * kWave);
    double acc = 0.0;
    int cnt = 0;
#pragma unroll 4
    for (int m = m_lo; m < m_hi; ++m) {
        const int k = row[m].k, j = row[m].j;
        const double w = row[m].w;
        const int i = i0 + m;
        if (m < lim && (!ACC || (i >= lo && i < hi))) {
            const int64_t idx = LAYOUT == 0 ? ((int64_t)k * n_buf + (i - lo)) * n_bins + j
                                            : ((int64_t)k * n_bins + j) * n_buf + (i - lo);
            acc += w * (a * (double)P[idx] - b);
            if (ACC) ++cnt;
        }
    }
    if (i0 < n_seg) {
        const int Me = min(M, lim);
        const double r = Me > 0 ? acc / sqrt(row[Me - 1].w2sum) : 0.0;
        const int c = (int)(cs / S), s = (int)(cs % S);
        const int64_t o = ((int64_t)c * n_seg + i0) * S + s;
        if (ACC) {
            out[o] += (float)r;
            if (used) used[o] += cnt;
        } else {
            out[o] = (float)r;
            if (used) used[o] = max(Me, 0);
        }
    }
}

// power[k][i][j] -> power[k][j][i] through 32 x 32 LDS tiles (grid: bins/32,
// segments/32, templates).
__global__ __launch_bounds__(kBlock) void transpose_kernel(const float* __restrict__ src, int n_seg, int n_bins,
                                                           float* __restrict__ dst)
{
    __shared__ float tile[kTile][kTile + 1];
    const int k = blockIdx.z;
    const int j0 = blockIdx.x * kTile, i0 = blockIdx.y * kTile;
    const float* s = src + (int64_t)k * n_seg * n_bins;
    float* d = dst + (int64_t)k * n_seg * n_bins;
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 32 x 8
    for (int r = ty; r < kTile; r += kBlock / kTile) {
        const int i = i0 + r, j = j0 + tx;
        if (i < n_seg && j < n_bins) tile[r][tx] = s[(int64_t)i * n_bins + j];
    }
    __syncthreads();
    for (int r = ty; r < kTile; r += kBlock / kTile) {
        const int j = j0 + r, i = i0 + tx;
        if (i < n_seg && j < n_bins) d[(int64_t)j * n_seg + i] = tile[tx][r];
    }
}

}  // namespace

struct nr_ss_s {
    std::string err;
    hipStream_t stream = nullptr;
    nr_ss_geometry g{};
    int32_t n_mc = 0, S = 0;
    SsEntry* tab = nullptr;
    int32_t* len = nullptr;
    ~nr_ss_s()
    {
        if (tab) (void)hipFree(tab);
        if (len) (void)hipFree(len);
    }
};

namespace {

nr_status fail_create(const std::string& m, nr_status st)
{
    g_ss_error = m;
    return st;
}

nr_status device_status(nr_ss_plan p, hipError_t e, const char* what)
{
    if (e == hipSuccess) return NR_OK;
    const std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (p) p->err = m; else g_ss_error = m;
    return e == hipErrorOutOfMemory ? NR_ERR_OUT_OF_MEMORY : NR_ERR_DEVICE;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

namespace {

nr_status gather(nr_ss_plan p, const float* power, int32_t seg_begin, int32_t seg_count, float* n_sigma,
                 int32_t* n_used, bool acc)
{
    const nr_ss_geometry& g = p->g;
    const int chunks = (g.n_seg + kWave - 1) / kWave;
    const int64_t fam = (int64_t)p->n_mc * p->S;
    const int64_t waves = fam * chunks;
    const unsigned blocks = (unsigned)((waves * kWave + kBlock - 1) / kBlock);
    const double a = g.norm / g.sigma, b = g.mu / g.sigma;
    const int lo = seg_begin, hi = seg_begin + seg_count;
#define NR_GATHER(LAY, ACC)                                                                                          \
    gather_kernel<LAY, ACC><<<blocks, kBlock, 0, p->stream>>>(power, p->tab, p->len, fam, p->S, g.n_seg, g.n_bins, \
                                                              chunks, lo, hi, a, b, n_sigma, n_used)
    if (g.layout == 0) {
        if (acc) NR_GATHER(0, true); else NR_GATHER(0, false);
    } else {
        if (acc) NR_GATHER(1, true); else NR_GATHER(1, false);
    }
#undef NR_GATHER
    return device_status(p, hipGetLastError(), "stack-slide");
}

}  // namespace

extern "C" {

nr_status nr_ss_create(nr_ss_plan* out, const nr_ss_geometry* g, const double* beta_bank, const double* mc,
                       int32_t n_mc, int32_t t0_steps, void* stream)
{
    if (!out) return fail_create("out is NULL", NR_ERR_INVALID_ARG);
    *out = nullptr;
    if (!g || !beta_bank || !mc) return fail_create("geometry, bank and chirp masses must not be NULL", NR_ERR_INVALID_ARG);
    if (g->n_seg < 1 || g->n_beta < 1 || g->n_bins < 1)
        return fail_create("n_seg, n_beta and n_bins must be >= 1", NR_ERR_INVALID_ARG);
    if (g->layout != 0 && g->layout != 1) return fail_create("layout must be 0 or 1", NR_ERR_INVALID_ARG);
    if (!finite_pos(g->t_coh) || !finite_pos(g->df) || !finite_pos(g->f_start) || !finite_pos(g->norm) ||
        !finite_pos(g->sigma) || !std::isfinite(g->f_lo) || !std::isfinite(g->mu) || !std::isfinite(g->f_max) ||
        !(g->f_max > g->f_start))
        return fail_create("t_coh, df, f_start, norm and sigma must be positive and finite, f_max > f_start",
                           NR_ERR_INVALID_ARG);
    if (n_mc < 1 || t0_steps < 1 || t0_steps > 64)
        return fail_create("n_mc must be >= 1 and t0_steps in [1, 64]", NR_ERR_INVALID_ARG);
    for (int32_t k = 0; k < g->n_beta; ++k)
        if (!finite_pos(beta_bank[k]) || (k > 0 && !(beta_bank[k] > beta_bank[k - 1])))
            return fail_create("beta_bank must be positive, finite and strictly ascending", NR_ERR_INVALID_ARG);
    for (int32_t c = 0; c < n_mc; ++c)
        if (!finite_pos(mc[c])) return fail_create("chirp masses must be positive and finite", NR_ERR_INVALID_ARG);
    const int64_t entries = (int64_t)n_mc * t0_steps * g->n_seg;
    if (entries > (int64_t(1) << 31) || (int64_t)g->n_beta * g->n_seg * g->n_bins > (int64_t(1) << 40))
        return fail_create("track tables or spectra too large", NR_ERR_INVALID_ARG);

    nr_ss_plan p = new (std::nothrow) nr_ss_s();
    if (!p) return fail_create("host allocation failed", NR_ERR_OUT_OF_MEMORY);
    p->stream = (hipStream_t)stream;
    p->g = *g;
    p->n_mc = n_mc;
    p->S = t0_steps;
    std::vector<double> b0((size_t)n_mc);
    for (int32_t c = 0; c < n_mc; ++c) b0[c] = nr::chirp_beta(mc[c], g->f_start);
    double *d_b0 = nullptr, *d_bank = nullptr;
    hipError_t e = hipMalloc((void**)&p->tab, (size_t)entries * sizeof(SsEntry));
    if (e == hipSuccess) e = hipMalloc((void**)&p->len, (size_t)n_mc * t0_steps * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&d_b0, (size_t)n_mc * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&d_bank, (size_t)g->n_beta * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(d_b0, b0.data(), b0.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_bank, beta_bank, (size_t)g->n_beta * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int64_t fam = (int64_t)n_mc * t0_steps;
        tables_kernel<<<(unsigned)((fam + 255) / 256), 256, 0, p->stream>>>(
            d_b0, d_bank, g->n_beta, n_mc, t0_steps, g->n_seg, g->n_bins, g->t_coh, g->f_lo, g->df, g->f_start,
            g->f_max, p->tab, p->len);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (d_b0) (void)hipFree(d_b0);
    if (d_bank) (void)hipFree(d_bank);
    if (e != hipSuccess) {
        const nr_status st = device_status(nullptr, e, "track tables");
        delete p;
        return st;
    }
    *out = p;
    return NR_OK;
}


nr_status nr_ss_execute(nr_ss_plan p, const float* power, float* n_sigma, int32_t* n_used)
{
    if (!p) return NR_ERR_INVALID_ARG;
    if (!power || !n_sigma) {
        p->err = "power and n_sigma must not be NULL";
        return NR_ERR_INVALID_ARG;
    }
    return gather(p, power, 0, p->g.n_seg, n_sigma, n_used, false);
}

nr_status nr_ss_execute_range(nr_ss_plan p, const float* power, int32_t seg_begin, int32_t seg_count,
                              float* n_sigma, int32_t* n_used)
{
    if (!p) return NR_ERR_INVALID_ARG;
    if (!power || !n_sigma) {
        p->err = "power and n_sigma must not be NULL";
        return NR_ERR_INVALID_ARG;
    }
    if (seg_begin < 0 || seg_count < 1 || seg_begin > p->g.n_seg - seg_count) {
        p->err = "segment range outside [0, n_seg)";
        return NR_ERR_INVALID_ARG;
    }
    return gather(p, power, seg_begin, seg_count, n_sigma, n_used, true);
}

nr_status nr_ss_tables(nr_ss_plan p, int32_t* k, int32_t* j, double* w2sum, int32_t* len)
{
    if (!p) return NR_ERR_INVALID_ARG;
    const int64_t fam = (int64_t)p->n_mc * p->S;
    const int64_t entries = fam * p->g.n_seg;
    std::vector<SsEntry> t((size_t)entries);
    std::vector<int32_t> l((size_t)fam);
    nr_status st = device_status(p, hipMemcpyAsync(t.data(), p->tab, t.size() * sizeof(SsEntry),
                                                   hipMemcpyDeviceToHost, p->stream), "tables");
    if (st == NR_OK)
        st = device_status(p, hipMemcpyAsync(l.data(), p->len, l.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                                             p->stream), "tables");
    if (st == NR_OK) st = device_status(p, hipStreamSynchronize(p->stream), "tables");
    if (st != NR_OK) return st;
    for (int64_t f = 0; f < fam; ++f) {
        if (len) len[f] = l[f];
        for (int m = 0; m < p->g.n_seg; ++m) {
            const int64_t q = f * p->g.n_seg + m;
            const bool on = m < l[f];
            if (k) k[q] = on ? t[q].k : -1;
            if (j) j[q] = on ? t[q].j : -1;
            if (w2sum) w2sum[q] = on ? t[q].w2sum : 0.0;
        }
    }
    return NR_OK;
}

nr_status nr_ss_transpose(const float* power_kij, int32_t n_beta, int32_t n_seg, int32_t n_bins, float* power_kji,
                          void* stream)
{
    if (!power_kij || !power_kji || n_beta < 1 || n_seg < 1 || n_bins < 1 || n_beta > 65535)
        return fail_create("transpose: NULL array or size out of range", NR_ERR_INVALID_ARG);
    if (power_kij == power_kji) return fail_create("transpose: arrays must not alias", NR_ERR_INVALID_ARG);
    dim3 grid((unsigned)((n_bins + kTile - 1) / kTile), (unsigned)((n_seg + kTile - 1) / kTile), (unsigned)n_beta);
    transpose_kernel<<<grid, kBlock, 0, (hipStream_t)stream>>>(power_kij, n_seg, n_bins, power_kji);
    return device_status(nullptr, hipGetLastError(), "transpose");
}

const char* nr_ss_last_error(nr_ss_plan p)
{
    return p ? p->err.c_str() : g_ss_error.c_str();
}

void nr_ss_destroy(nr_ss_plan p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    delete p;
}

}  // extern "C"
