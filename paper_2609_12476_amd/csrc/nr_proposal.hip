// gfx950 kernels of the learned proposal's ranking and refinement steps
// (see include/nr_proposal.h): the largest standardised segment sum of each
// group of templates, and the top-k regions of each row of scores.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/nr_proposal.h"

namespace {

thread_local std::string g_prop_error;

constexpr int kWave = 64;
constexpr int kMaxGroup = 64;
constexpr int kMaxK = 4096;
constexpr int kTopkThreads = 1024;
constexpr int kTopkMaxN = 16384;

nr_status fail(const std::string& m)
{
    g_prop_error = m;
    return NR_ERR_INVALID_ARG;
}

nr_status launched(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return NR_OK;
    g_prop_error = std::string(what) + ": " + hipGetErrorString(e);
    return NR_ERR_DEVICE;
}

// (z, index) pair that wins a comparison: the larger z, the lower index on
// equal z; NaN never wins (index -1 marks "no number yet").
__device__ __forceinline__ bool better(double z, int i, double bz, int bi)
{
    return bi < 0 ? !isnan(z) : (z > bz || (z == bz && i < bi));
}

// One wave per group: lanes stride over the group's (template, bin) pairs in
// index order, keep their best, and combine by a butterfly of lane exchanges.
__global__ __launch_bounds__(256) void max_z_kernel(const float* __restrict__ stat,
                                                    const int32_t* __restrict__ n_used, int64_t n_groups,
                                                    int group, int K, double norm, float* __restrict__ zmax,
                                                    int32_t* __restrict__ arg)
{
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (g >= n_groups) return;  // whole waves
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t t0 = g * group;
    const int cnt = group * K;
    double bz = 0.0;
    int bi = -1;
    for (int e = lane; e < cnt; e += kWave) {
        const int t = e / K, k = e - t * K;
        const int32_t N = n_used[t0 + t];
        double z = 0.0;
        if (N > 0) {
            const double Nd = (double)N;
            z = ((double)stat[(t0 + t) * K + k] * norm - Nd) / sqrt(Nd);
        }
        if (better(z, e, bz, bi)) {
            bz = z;
            bi = e;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double oz = __shfl_xor(bz, o);
        const int oi = __shfl_xor(bi, o);
        if (oi >= 0 && better(oz, oi, bz, bi)) {
            bz = oz;
            bi = oi;
        }
    }
    if (lane == 0) {
        zmax[g] = bi < 0 ? NAN : (float)bz;
        if (arg) arg[g] = bi;
    }
}

// Sort key of a score: ascending keys give descending scores, equal scores
// ascending items; -0 is +0 and NaN sorts after every number.
__device__ __forceinline__ uint64_t rank_key(float s, uint32_t item)
{
    uint32_t hi;
    if (isnan(s)) {
        hi = 0xFFFFFFFFu;
    } else {
        uint32_t u = __float_as_uint(s == 0.0f ? 0.0f : s);
        u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // increasing with s
        hi = ~u;                                          // decreasing with s; below 2^32 - 1
    }
    return ((uint64_t)hi << 32) | item;
}

// One workgroup per row: bitonic sort of the row's keys (padded to a power
// of two with keys above every item) in LDS, then the first k items.
__global__ __launch_bounds__(kTopkThreads) void topk_kernel(const float* __restrict__ scores, int n, int P, int k,
                                                            int32_t* __restrict__ idx)
{
    extern __shared__ uint64_t keys[];
    const int64_t r = blockIdx.x;
    const float* row = scores + r * n;
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        keys[i] = i < n ? rank_key(row[i], (uint32_t)i) : ~(uint64_t)0;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = keys[lo], b = keys[hi];
                if ((a > b) == up) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < k; j += blockDim.x) idx[r * k + j] = (int32_t)(uint32_t)keys[j];
}

}  // namespace

extern "C" {

nr_status nr_prop_max_z(const float* stat, const int32_t* n_used, int64_t n_groups, int32_t group, int32_t K,
                        double norm, float* zmax, int32_t* arg, void* stream)
{
    if (n_groups < 0 || group < 1 || group > kMaxGroup || K < 1 || K > kMaxK || !(norm > 0.0) ||
        !std::isfinite(norm))
        return fail("nr_prop_max_z: need n_groups >= 0, 1 <= group <= 64, 1 <= K <= 4096, norm > 0");
    if (n_groups == 0) return NR_OK;
    if (!stat || !n_used || !zmax) return fail("nr_prop_max_z: stat, n_used and zmax must not be NULL");
    if (n_groups > (int64_t)INT_MAX * 4) return fail("nr_prop_max_z: too many groups");
    const unsigned blocks = (unsigned)((n_groups + 3) / 4);
    max_z_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(stat, n_used, n_groups, group, K, norm, zmax, arg);
    return launched("nr_prop_max_z");
}

nr_status nr_prop_topk(const float* scores, int64_t rows, int32_t n, int32_t k, int32_t* idx, void* stream)
{
    if (rows < 0 || n < 1 || n > kTopkMaxN || k < 1 || k > n)
        return fail("nr_prop_topk: need rows >= 0, 1 <= n <= 16384, 1 <= k <= n");
    if (rows == 0) return NR_OK;
    if (!scores || !idx) return fail("nr_prop_topk: scores and idx must not be NULL");
    if (rows > INT_MAX) return fail("nr_prop_topk: too many rows");
    int P = 2;
    while (P < n) P <<= 1;
    const size_t lds = (size_t)P * sizeof(uint64_t);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(topk_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            g_prop_error = std::string("nr_prop_topk: LDS limit: ") + hipGetErrorString(e);
            return NR_ERR_DEVICE;
        }
    }
    topk_kernel<<<(unsigned)rows, kTopkThreads, lds, (hipStream_t)stream>>>(scores, n, P, k, idx);
    return launched("nr_prop_topk");
}

const char* nr_prop_last_error(void) { return g_prop_error.c_str(); }

}  // extern "C"
