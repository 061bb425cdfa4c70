// gfx950 kernels of the learned proposal's network (see include/nr_mlp.h):
// bfloat16 weight copies, fused three-layer forward, backward through the
// activations, deterministic weight gradients, the loss, Adam, and the
// region feature builder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>

#include "../../include/nr_mlp.h"

namespace {

constexpr int IN = NR_MLP_IN, HID = NR_MLP_HIDDEN, NP = NR_MLP_PARAMS;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + HID * IN, OFF_W2 = OFF_B1 + HID,
              OFF_B2 = OFF_W2 + HID * HID, OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
static_assert(OFF_B3 + 1 == NP, "parameter layout");
constexpr int RB = 32;     // rows per workgroup in the row-parallel kernels
constexpr int BLK = 256;   // one thread per hidden unit

thread_local std::string g_mlp_error;

// ---------------------------------------------------------------- bf16 --

typedef uint16_t bf16_t;

__device__ __forceinline__ bf16_t to_bf16(float f)
{
    // round to nearest, ties to even
    const uint32_t u = __float_as_uint(f);
    return (bf16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float from_bf16(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Weight copies used by the products: W1t[k][j] = W1[j][k], W2t[k][j] =
// W2[j][k] (column access by unit j is contiguous across threads), W2 as is
// (for the backward product), w3.
__global__ void refresh_bf16_kernel(const float* __restrict__ p, bf16_t* __restrict__ w1t,
                                    bf16_t* __restrict__ w2, bf16_t* __restrict__ w2t,
                                    bf16_t* __restrict__ w3)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < HID * IN) {
        const int j = i / IN, k = i % IN;
        w1t[k * HID + j] = to_bf16(p[OFF_W1 + i]);
    }
    if (i < HID * HID) {
        const int j = i / HID, k = i % HID;
        const bf16_t h = to_bf16(p[OFF_W2 + i]);
        w2[i] = h;
        w2t[k * HID + j] = h;
    }
    if (i < HID) w3[i] = to_bf16(p[OFF_W3 + i]);
}

// ------------------------------------------------------------- forward --

// The two hidden layers are dense products [RB rows x KW] x [KW x HID] on
// the matrix cores: v_mfma_f32_32x32x2f32 takes FP32 activations and the
// bfloat16 weights widened exactly to FP32, so the products keep the FP32
// activation precision.  Wave wv of the workgroup owns output columns
// 64 wv .. 64 wv + 63 as two 32 x 32 tiles.  Operand layout of the
// instruction (lane l, m = l % 32, h = l / 32): A[m][k = h], B[k = h][n = m];
// accumulator e of lane l is C[8 (e / 4) + 4 h + e % 4][m].
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int XS = IN + 1, HS = HID + 1;   // LDS row strides (odd: no bank conflicts)

__device__ __forceinline__ int tile_row(int e, int h) { return 8 * (e >> 2) + 4 * h + (e & 3); }

template <int KW, int STRIDE>
__device__ __forceinline__ void rows_times_weights(const float* __restrict__ src, const bf16_t* __restrict__ wt,
                                                   int n0, floatx16& c0, floatx16& c1)
{
    const int l = threadIdx.x & 63;
    const int m = l & 31, h = l >> 5;
    // unrolled so that the weight loads of several steps are in flight together
#pragma unroll 16
    for (int k = 0; k < KW; k += 2) {
        const float a = src[m * STRIDE + k + h];
        const float b0 = from_bf16(wt[(k + h) * HID + n0 + m]);
        const float b1 = from_bf16(wt[(k + h) * HID + n0 + 32 + m]);
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, c1, 0, 0, 0);
    }
}

// One workgroup per RB = 32 rows (four waves).
__global__ __launch_bounds__(BLK) void forward_kernel(const float* __restrict__ x, int64_t B,
                                                      const float* __restrict__ p,
                                                      const bf16_t* __restrict__ w1t,
                                                      const bf16_t* __restrict__ w2t,
                                                      const bf16_t* __restrict__ w3,
                                                      float* __restrict__ h1_out,
                                                      float* __restrict__ h2_out,
                                                      float* __restrict__ z_out)
{
    static_assert(RB == 32 && BLK == 256 && HID == 256, "four waves of two 32 x 32 tiles");
    __shared__ float xs[RB * XS];
    __shared__ float hs[RB * HS];
    __shared__ float red[4][RB];
    const int t = threadIdx.x;
    const int l = t & 63, wv = t >> 6;
    const int m = l & 31, h = l >> 5;
    const int n0 = 64 * wv;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int nr = (int)((B - r0) < RB ? (B - r0) : RB);
    for (int i = t; i < RB * IN; i += BLK) {
        const int r = i / IN, k = i % IN;
        xs[r * XS + k] = r < nr ? x[(r0 + r) * IN + k] : 0.0f;
    }
    __syncthreads();
    floatx16 c0, c1;
    {
        const float b0 = p[OFF_B1 + n0 + m], b1 = p[OFF_B1 + n0 + 32 + m];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            c0[e] = b0;
            c1[e] = b1;
        }
    }
    rows_times_weights<IN, XS>(xs, w1t, n0, c0, c1);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int r = tile_row(e, h);
        const float v0 = fmaxf(c0[e], 0.0f), v1 = fmaxf(c1[e], 0.0f);
        hs[r * HS + n0 + m] = v0;
        hs[r * HS + n0 + 32 + m] = v1;
        if (h1_out && r < nr) {
            h1_out[(r0 + r) * HID + n0 + m] = v0;
            h1_out[(r0 + r) * HID + n0 + 32 + m] = v1;
        }
    }
    __syncthreads();
    {
        const float b0 = p[OFF_B2 + n0 + m], b1 = p[OFF_B2 + n0 + 32 + m];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            c0[e] = b0;
            c1[e] = b1;
        }
    }
    rows_times_weights<HID, HS>(hs, w2t, n0, c0, c1);
    const float w0 = from_bf16(w3[n0 + m]), w1 = from_bf16(w3[n0 + 32 + m]);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int r = tile_row(e, h);
        const float v0 = fmaxf(c0[e], 0.0f), v1 = fmaxf(c1[e], 0.0f);
        if (h2_out && r < nr) {
            h2_out[(r0 + r) * HID + n0 + m] = v0;
            h2_out[(r0 + r) * HID + n0 + 32 + m] = v1;
        }
        // sum over the wave's 64 columns of row r, in a fixed butterfly order
        float v = v0 * w0 + v1 * w1;
        for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (m == 0) red[wv][r] = v;
    }
    __syncthreads();
    if (t < nr) z_out[r0 + t] = ((red[0][t] + red[1][t]) + (red[2][t] + red[3][t])) + p[OFF_B3];
}

// ------------------------------------------------------------ backward --

// Per RB rows: dz = (sigmoid(z) - y) / B; da2 = dz w3 [h2 > 0];
// da1 = (da2 W2) [h1 > 0].
__global__ __launch_bounds__(BLK) void backward_act_kernel(
    const float* __restrict__ z, const float* __restrict__ y, int64_t B,
    const float* __restrict__ h1, const float* __restrict__ h2, const bf16_t* __restrict__ w2,
    const bf16_t* __restrict__ w3, float* __restrict__ dz_out, float* __restrict__ da2_out,
    float* __restrict__ da1_out)
{
    __shared__ float d2[RB * HS];
    __shared__ float dzs[RB];
    const int j = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    const int nr = (int)((B - r0) < RB ? (B - r0) : RB);
    if (j < RB) {
        float d = 0.0f;
        if (j < nr) {
            const float zz = z[r0 + j];
            d = (1.0f / (1.0f + expf(-zz)) - y[r0 + j]) / (float)B;
            dz_out[r0 + j] = d;
        }
        dzs[j] = d;
    }
    __syncthreads();
    const float wj = from_bf16(w3[j]);
#pragma unroll 8
    for (int r = 0; r < RB; ++r) {
        float d = 0.0f;
        if (r < nr && h2[(r0 + r) * HID + j] > 0.0f) d = dzs[r] * wj;
        d2[r * HS + j] = d;
        if (r < nr) da2_out[(r0 + r) * HID + j] = d;
    }
    __syncthreads();
    // da2 [RB x HID] times W2 [HID (row j) x HID (column k)] on the matrix cores
    const int l = j & 63, wv = j >> 6;
    const int m = l & 31, h = l >> 5;
    const int n0 = 64 * wv;
    floatx16 c0, c1;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        c0[e] = 0.0f;
        c1[e] = 0.0f;
    }
    rows_times_weights<HID, HS>(d2, w2, n0, c0, c1);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int r = tile_row(e, h);
        if (r < nr) {
            const int64_t o = (r0 + r) * HID + n0 + m;
            da1_out[o] = h1[o] > 0.0f ? c0[e] : 0.0f;
            da1_out[o + 32] = h1[o + 32] > 0.0f ? c1[e] : 0.0f;
        }
    }
}

// Weight gradients as dense products on the matrix cores:
//   dW1[j][k] = sum_r da1[r][j] x[r][k],   dW2[j][k] = sum_r da2[r][j] h1[r][k],
// i.e. C = A B with A[j][r] = da[r][j] and B[r][k] = x[r][k] (or h1): the
// batch row r is the contraction index.  The batch is cut into S chunks of
// RC rows; wave (strip, chunk) accumulates a 32 x 64 strip of one matrix over
// its chunk with v_mfma_f32_32x32x2f32 (FP32 operands, so the gradient keeps
// FP32 precision) and stores it in the chunk's partial gradient.  Lane
// (m, h) of a step over rows r, r + 1 supplies A[m][h] = da[r + h][j0 + m]
// and B[h][n = m] = src[r + h][k0 + m] (each a pair of coalesced 32-float
// row pieces); accumulator e of the lane is C[8 (e / 4) + 4 h + e % 4][m].
// The bias and output-vector gradients (db1, db2, dw3, db3) are VALU sums
// over the chunk by the remaining waves, one entry per lane.  A second pass
// adds the S partials of every parameter in chunk order in FP64, so the
// gradient is bitwise reproducible.
constexpr int kW1Strips = HID / 32;                    // 32 x 64 strips of dW1 (64 columns)
constexpr int kW2Strips = (HID / 32) * (HID / 64);     // of dW2
constexpr int kVecStrips = 3 * (HID / 64) + 1;         // db1, db2, dw3 by 64 entries; db3
constexpr int kGradStrips = kW1Strips + kW2Strips + kVecStrips;
constexpr int kMaxChunks = 64;

__host__ __device__ inline int grad_chunk_rows(int64_t B)
{
    // at least 32 rows per chunk, at most kMaxChunks chunks; even (MFMA steps of two rows)
    int64_t rc = (B + kMaxChunks - 1) / kMaxChunks;
    if (rc < 32) rc = 32;
    return (int)((rc + 1) & ~int64_t(1));
}

__global__ __launch_bounds__(BLK) void weight_grad_partial_kernel(
    const float* __restrict__ x, const float* __restrict__ h1, const float* __restrict__ h2,
    const float* __restrict__ dz, const float* __restrict__ da1, const float* __restrict__ da2, int64_t B,
    int rc, int n_chunks, float* __restrict__ part)
{
    const int wv = (int)(blockIdx.x * (BLK / 64) + (threadIdx.x >> 6));
    if (wv >= kGradStrips * n_chunks) return;  // whole waves
    const int strip = wv % kGradStrips, chunk = wv / kGradStrips;
    const int l = threadIdx.x & 63;
    const int m = l & 31, h = l >> 5;
    const int64_t r0 = (int64_t)chunk * rc;
    const int64_t r1 = (r0 + rc < B) ? r0 + rc : B;
    float* out = part + (int64_t)chunk * NP;
    if (strip < kW1Strips + kW2Strips) {
        const float* A;
        const float* S;
        int ld, j0, k0, off, ldw;
        if (strip < kW1Strips) {
            A = da1; S = x; ld = IN; j0 = 32 * strip; k0 = 0; off = OFF_W1; ldw = IN;
        } else {
            const int q = strip - kW1Strips;
            A = da2; S = h1; ld = HID; j0 = 32 * (q / (HID / 64)); k0 = 64 * (q % (HID / 64)); off = OFF_W2;
            ldw = HID;
        }
        floatx16 c0, c1;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            c0[e] = 0.0f;
            c1[e] = 0.0f;
        }
#pragma unroll 8
        for (int64_t r = r0; r < r1; r += 2) {
            const int64_t rr = r + h;
            const bool in = rr < r1;
            const float a = in ? A[rr * HID + j0 + m] : 0.0f;
            const float b0 = in ? S[rr * ld + k0 + m] : 0.0f;
            const float b1 = in ? S[rr * ld + k0 + 32 + m] : 0.0f;
            c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, c1, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int j = j0 + tile_row(e, h);
            out[off + j * ldw + k0 + m] = c0[e];
            out[off + j * ldw + k0 + 32 + m] = c1[e];
        }
        return;
    }
    // vector gradients: one entry per lane
    const int v = strip - kW1Strips - kW2Strips;
    const int which = v / (HID / 64);          // 0 db1, 1 db2, 2 dw3, 3 db3
    const int j = (v % (HID / 64)) * 64 + l;
    float s = 0.0f;
    if (which == 0) {
        for (int64_t r = r0; r < r1; ++r) s += da1[r * HID + j];
        out[OFF_B1 + j] = s;
    } else if (which == 1) {
        for (int64_t r = r0; r < r1; ++r) s += da2[r * HID + j];
        out[OFF_B2 + j] = s;
    } else if (which == 2) {
        for (int64_t r = r0; r < r1; ++r) s = fmaf(dz[r], h2[r * HID + j], s);
        out[OFF_W3 + j] = s;
    } else if (l == 0) {
        for (int64_t r = r0; r < r1; ++r) s += dz[r];
        out[OFF_B3] = s;
    }
}

// Mean of softplus(z) - y z over the batch, one workgroup, fixed order.
__global__ __launch_bounds__(BLK) void loss_kernel(const float* __restrict__ z,
                                                   const float* __restrict__ y, int64_t B,
                                                   float* __restrict__ loss)
{
    __shared__ double part[BLK];
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < B; r += BLK) {
        const double zz = z[r];
        const double sp = zz > 0.0 ? zz + log1p(exp(-zz)) : log1p(exp(zz));
        s += sp - (double)y[r] * zz;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(part[0] / (double)B);
}

// The bfloat16 copies of parameter i (new value q) where the products read
// them (see refresh_bf16_kernel); biases have none.
__device__ __forceinline__ void store_bf16(int i, float q, bf16_t* __restrict__ w1t, bf16_t* __restrict__ w2,
                                           bf16_t* __restrict__ w2t, bf16_t* __restrict__ w3)
{
    if (i < OFF_B1) {
        w1t[(i % IN) * HID + i / IN] = to_bf16(q);
    } else if (i >= OFF_W2 && i < OFF_B2) {
        const int q2 = i - OFF_W2;
        const bf16_t h = to_bf16(q);
        w2[q2] = h;
        w2t[(q2 % HID) * HID + q2 / HID] = h;
    } else if (i >= OFF_W3 && i < OFF_B3) {
        w3[i - OFF_W3] = to_bf16(q);
    }
}

// One thread per parameter.  FROM_PARTS: the gradient is the sum over the
// chunks, in chunk order, of the partial gradients (FP64; else it is read
// from grad_in).  It is stored to grad_out when given.  ADAM: one Adam update
// (beta1 0.9, beta2 0.999, eps 1e-8; c1, c2 the bias corrections) of the
// masters and moments, and the bfloat16 copies of the new masters.
template <bool FROM_PARTS, bool ADAM>
__global__ void update_kernel(const float* __restrict__ part, int n_chunks, const float* __restrict__ grad_in,
                              float* __restrict__ grad_out, float* __restrict__ p, float* __restrict__ m,
                              float* __restrict__ v, float lr, float c1, float c2, bf16_t* __restrict__ w1t,
                              bf16_t* __restrict__ w2, bf16_t* __restrict__ w2t, bf16_t* __restrict__ w3)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    float gi;
    if (FROM_PARTS) {
        double s = 0.0;
#pragma unroll 8
        for (int c = 0; c < n_chunks; ++c) s += (double)part[(int64_t)c * NP + i];
        gi = (float)s;
    } else {
        gi = grad_in[i];
    }
    if (grad_out) grad_out[i] = gi;
    if (ADAM) {
        const float mi = 0.9f * m[i] + 0.1f * gi;
        const float vi = 0.999f * v[i] + 0.001f * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float q = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
        p[i] = q;
        store_bf16(i, q, w1t, w2, w2t, w3);
    }
}

// ------------------------------------------------------------- features --

// One workgroup per (mc, sb) region; 64 threads build its 8 x 8 patch.
__global__ void region_features_kernel(const float* __restrict__ stat,
                                       const int32_t* __restrict__ n_used, int n_mc, int n_sub,
                                       int K, double norm, float* __restrict__ out)
{
    const int region = blockIdx.x;
    const int mc = region / n_sub, sb = region % n_sub;
    __shared__ int kstar;
    if (threadIdx.x == 0) {
        const float* s = stat + (int64_t)region * K;
        int best = 0;
        float bv = s[0];
        for (int k = 1; k < K; ++k)
            if (s[k] > bv) {
                bv = s[k];
                best = k;
            }
        kstar = best;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= 64) return;
    const int i = t >> 3, c = t & 7;
    int m2 = mc - 3 + i;
    m2 = m2 < 0 ? 0 : (m2 >= n_mc ? n_mc - 1 : m2);
    int k = kstar - 3 + c;
    k = k < 0 ? 0 : (k >= K ? K - 1 : k);
    const int tm = m2 * n_sub + sb;
    const double N = (double)n_used[tm];
    float z = 0.0f;
    if (N > 0.0) z = (float)(((double)stat[(int64_t)tm * K + k] * norm - N) / sqrt(N));
    out[(int64_t)region * 64 + t] = z;
}

}  // namespace

// ---------------------------------------------------------------- state --

struct nr_mlp_s {
    std::string err;
    hipStream_t stream = nullptr;
    int64_t max_batch = 0;
    int64_t step = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bf16_t *w1t = nullptr, *w2 = nullptr, *w2t = nullptr, *w3 = nullptr;
    float *h1 = nullptr, *h2 = nullptr, *z = nullptr, *dz = nullptr, *da1 = nullptr, *da2 = nullptr;
    float* loss = nullptr;
    float* gpart = nullptr;   // per-chunk partial gradients [gchunks][NP]
    int gchunks = 0;
    ~nr_mlp_s()
    {
        for (void* q : {(void*)p, (void*)m, (void*)v, (void*)grad, (void*)w1t, (void*)w2, (void*)w2t,
                        (void*)w3, (void*)h1, (void*)h2, (void*)z, (void*)dz, (void*)da1, (void*)da2,
                        (void*)loss, (void*)gpart})
            if (q) (void)hipFree(q);
    }
};

namespace {

bool set_err(nr_mlp m, const std::string& s)
{
    if (m)
        m->err = s;
    else
        g_mlp_error = s;
    return false;
}

nr_status hip_status(nr_mlp m, hipError_t e, const char* what)
{
    if (e == hipSuccess) return NR_OK;
    set_err(m, std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? NR_ERR_OUT_OF_MEMORY : NR_ERR_DEVICE;
}

template <typename T>
hipError_t dalloc(T** ptr, size_t count)
{
    return hipMalloc((void**)ptr, count * sizeof(T));
}

nr_status refresh(nr_mlp m)
{
    refresh_bf16_kernel<<<(HID * HID + 255) / 256, 256, 0, m->stream>>>(m->p, m->w1t, m->w2, m->w2t, m->w3);
    return hip_status(m, hipGetLastError(), "weight copies");
}

nr_status check_batch(nr_mlp m, int64_t B)
{
    if (B < 1 || B > m->max_batch) {
        set_err(m, "batch size " + std::to_string(B) + " outside [1, " + std::to_string(m->max_batch) + "]");
        return NR_ERR_INVALID_ARG;
    }
    return NR_OK;
}

nr_status run_forward(nr_mlp m, const float* x, int64_t B, bool keep, float* logits)
{
    const unsigned blocks = (unsigned)((B + RB - 1) / RB);
    forward_kernel<<<blocks, BLK, 0, m->stream>>>(x, B, m->p, m->w1t, m->w2t, m->w3, keep ? m->h1 : nullptr,
                                                  keep ? m->h2 : nullptr, logits);
    return hip_status(m, hipGetLastError(), "forward");
}

// Bias corrections of the next Adam step (advances the step count).
void adam_corrections(nr_mlp m, float* c1, float* c2)
{
    m->step += 1;
    *c1 = (float)(1.0 - std::pow(0.9, (double)m->step));
    *c2 = (float)(1.0 - std::pow(0.999, (double)m->step));
}

// Gradient of the batch into grad (or NULL); lr > 0: followed by one Adam
// update in the same pass over the parameters.
nr_status run_gradient(nr_mlp m, const float* x, const float* y, int64_t B, float* grad, float* loss, float lr)
{
    nr_status st = run_forward(m, x, B, true, m->z);
    if (st != NR_OK) return st;
    const unsigned blocks = (unsigned)((B + RB - 1) / RB);
    backward_act_kernel<<<blocks, BLK, 0, m->stream>>>(m->z, y, B, m->h1, m->h2, m->w2, m->w3, m->dz, m->da2,
                                                       m->da1);
    if ((st = hip_status(m, hipGetLastError(), "backward")) != NR_OK) return st;
    const int rc = grad_chunk_rows(B);
    const int n_chunks = (int)((B + rc - 1) / rc);
    if (n_chunks > m->gchunks) {
        set_err(m, "internal: gradient chunks exceed the workspace");
        return NR_ERR_DEVICE;
    }
    const unsigned gblocks = (unsigned)((kGradStrips * n_chunks + BLK / 64 - 1) / (BLK / 64));
    weight_grad_partial_kernel<<<gblocks, BLK, 0, m->stream>>>(x, m->h1, m->h2, m->dz, m->da1, m->da2, B, rc,
                                                               n_chunks, m->gpart);
    if ((st = hip_status(m, hipGetLastError(), "weight gradients")) != NR_OK) return st;
    if (loss) {
        loss_kernel<<<1, BLK, 0, m->stream>>>(m->z, y, B, loss);
        if ((st = hip_status(m, hipGetLastError(), "loss")) != NR_OK) return st;
    }
    const unsigned ublocks = (NP + 255) / 256;
    if (lr > 0.0f) {
        float c1, c2;
        adam_corrections(m, &c1, &c2);
        update_kernel<true, true><<<ublocks, 256, 0, m->stream>>>(m->gpart, n_chunks, nullptr, grad, m->p, m->m,
                                                                  m->v, lr, c1, c2, m->w1t, m->w2, m->w2t, m->w3);
    } else {
        update_kernel<true, false><<<ublocks, 256, 0, m->stream>>>(m->gpart, n_chunks, nullptr, grad, nullptr,
                                                                   nullptr, nullptr, 0.0f, 1.0f, 1.0f, nullptr,
                                                                   nullptr, nullptr, nullptr);
    }
    return hip_status(m, hipGetLastError(), "gradient sum / Adam");
}

nr_status run_adam(nr_mlp m, const float* grad, float lr)
{
    float c1, c2;
    adam_corrections(m, &c1, &c2);
    update_kernel<false, true><<<(NP + 255) / 256, 256, 0, m->stream>>>(nullptr, 0, grad, nullptr, m->p, m->m, m->v,
                                                                        lr, c1, c2, m->w1t, m->w2, m->w2t, m->w3);
    return hip_status(m, hipGetLastError(), "adam");
}

}  // namespace

extern "C" {

nr_status nr_mlp_create(nr_mlp* out, int64_t max_batch, void* stream)
{
    if (!out) {
        g_mlp_error = "out is NULL";
        return NR_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (max_batch < 1 || max_batch > (int64_t(1) << 26)) {
        g_mlp_error = "max_batch must be in [1, 2^26]";
        return NR_ERR_INVALID_ARG;
    }
    nr_mlp m = new (std::nothrow) nr_mlp_s();
    if (!m) {
        g_mlp_error = "host allocation failed";
        return NR_ERR_OUT_OF_MEMORY;
    }
    m->stream = (hipStream_t)stream;
    m->max_batch = max_batch;
    hipError_t e = hipSuccess;
    const size_t act = (size_t)max_batch * HID;
    if (e == hipSuccess) e = dalloc(&m->p, NP);
    if (e == hipSuccess) e = dalloc(&m->m, NP);
    if (e == hipSuccess) e = dalloc(&m->v, NP);
    if (e == hipSuccess) e = dalloc(&m->grad, NP);
    if (e == hipSuccess) e = dalloc(&m->w1t, (size_t)HID * IN);
    if (e == hipSuccess) e = dalloc(&m->w2, (size_t)HID * HID);
    if (e == hipSuccess) e = dalloc(&m->w2t, (size_t)HID * HID);
    if (e == hipSuccess) e = dalloc(&m->w3, (size_t)HID);
    if (e == hipSuccess) e = dalloc(&m->h1, act);
    if (e == hipSuccess) e = dalloc(&m->h2, act);
    if (e == hipSuccess) e = dalloc(&m->da1, act);
    if (e == hipSuccess) e = dalloc(&m->da2, act);
    if (e == hipSuccess) e = dalloc(&m->z, (size_t)max_batch);
    if (e == hipSuccess) e = dalloc(&m->dz, (size_t)max_batch);
    if (e == hipSuccess) e = dalloc(&m->loss, 1);
    // chunks of any batch B <= max_batch: at most min(kMaxChunks, ceil(B / 32))
    m->gchunks = (int)std::min<int64_t>(kMaxChunks, (max_batch + 31) / 32);
    if (e == hipSuccess) e = dalloc(&m->gpart, (size_t)m->gchunks * NP);
    if (e == hipSuccess) e = hipMemsetAsync(m->p, 0, NP * sizeof(float), m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, NP * sizeof(float), m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, NP * sizeof(float), m->stream);
    if (e != hipSuccess) {
        g_mlp_error = std::string("device allocation failed: ") + hipGetErrorString(e);
        delete m;
        return NR_ERR_OUT_OF_MEMORY;
    }
    if (refresh(m) != NR_OK) {
        g_mlp_error = m->err;
        delete m;
        return NR_ERR_DEVICE;
    }
    *out = m;
    return NR_OK;
}

nr_status nr_mlp_set_params(nr_mlp m, const float* host_params)
{
    if (!m || !host_params) return NR_ERR_INVALID_ARG;
    nr_status st = hip_status(m, hipMemcpyAsync(m->p, host_params, NP * sizeof(float), hipMemcpyHostToDevice, m->stream),
                              "parameter upload");
    if (st == NR_OK) st = hip_status(m, hipMemsetAsync(m->m, 0, NP * sizeof(float), m->stream), "moments");
    if (st == NR_OK) st = hip_status(m, hipMemsetAsync(m->v, 0, NP * sizeof(float), m->stream), "moments");
    if (st == NR_OK) st = refresh(m);
    if (st == NR_OK) st = hip_status(m, hipStreamSynchronize(m->stream), "parameter upload");
    m->step = 0;
    return st;
}

nr_status nr_mlp_get_params(nr_mlp m, float* host_params)
{
    if (!m || !host_params) return NR_ERR_INVALID_ARG;
    nr_status st = hip_status(m, hipMemcpyAsync(host_params, m->p, NP * sizeof(float), hipMemcpyDeviceToHost, m->stream),
                              "parameter download");
    if (st == NR_OK) st = hip_status(m, hipStreamSynchronize(m->stream), "parameter download");
    return st;
}

nr_status nr_mlp_get_state(nr_mlp m, float* host_state, int64_t* step)
{
    if (!m || !host_state || !step) return NR_ERR_INVALID_ARG;
    const size_t b = NP * sizeof(float);
    nr_status st = hip_status(m, hipMemcpyAsync(host_state, m->p, b, hipMemcpyDeviceToHost, m->stream), "state");
    if (st == NR_OK) st = hip_status(m, hipMemcpyAsync(host_state + NP, m->m, b, hipMemcpyDeviceToHost, m->stream), "state");
    if (st == NR_OK)
        st = hip_status(m, hipMemcpyAsync(host_state + 2 * NP, m->v, b, hipMemcpyDeviceToHost, m->stream), "state");
    if (st == NR_OK) st = hip_status(m, hipStreamSynchronize(m->stream), "state");
    if (st == NR_OK) *step = m->step;
    return st;
}

nr_status nr_mlp_set_state(nr_mlp m, const float* host_state, int64_t step)
{
    if (!m || !host_state || step < 0) return NR_ERR_INVALID_ARG;
    const size_t b = NP * sizeof(float);
    nr_status st = hip_status(m, hipMemcpyAsync(m->p, host_state, b, hipMemcpyHostToDevice, m->stream), "state");
    if (st == NR_OK) st = hip_status(m, hipMemcpyAsync(m->m, host_state + NP, b, hipMemcpyHostToDevice, m->stream), "state");
    if (st == NR_OK)
        st = hip_status(m, hipMemcpyAsync(m->v, host_state + 2 * NP, b, hipMemcpyHostToDevice, m->stream), "state");
    if (st == NR_OK) st = refresh(m);
    if (st == NR_OK) st = hip_status(m, hipStreamSynchronize(m->stream), "state");
    if (st == NR_OK) m->step = step;
    return st;
}

nr_status nr_mlp_forward(nr_mlp m, const float* x, int64_t B, float* logits)
{
    if (!m || !x || !logits) return NR_ERR_INVALID_ARG;
    if (B < 1) {
        set_err(m, "batch size must be >= 1");
        return NR_ERR_INVALID_ARG;
    }
    // inference keeps no activations, so any batch size streams through
    return run_forward(m, x, B, false, logits);
}

nr_status nr_mlp_gradient(nr_mlp m, const float* x, const float* y, int64_t B, float* grad, float* loss)
{
    if (!m || !x || !y) return NR_ERR_INVALID_ARG;
    nr_status st = check_batch(m, B);
    if (st != NR_OK) return st;
    st = run_gradient(m, x, y, B, m->grad, loss, 0.0f);
    if (st == NR_OK && grad)
        st = hip_status(m, hipMemcpyAsync(grad, m->grad, NP * sizeof(float), hipMemcpyDeviceToDevice, m->stream),
                        "gradient copy");
    return st;
}

nr_status nr_mlp_adam_step(nr_mlp m, const float* grad, float lr)
{
    if (!m || !grad || !(lr > 0.0f)) return NR_ERR_INVALID_ARG;
    return run_adam(m, grad, lr);
}

nr_status nr_mlp_train_step(nr_mlp m, const float* x, const float* y, int64_t B, float lr, float* loss)
{
    if (!m || !x || !y || !(lr > 0.0f)) return NR_ERR_INVALID_ARG;
    nr_status st = check_batch(m, B);
    if (st != NR_OK) return st;
    return run_gradient(m, x, y, B, nullptr, loss, lr);
}

nr_status nr_mlp_region_features(const float* stat, const int32_t* n_used, int32_t n_mc, int32_t n_sub,
                                 int32_t K, double norm, float* features, void* stream)
{
    if (!stat || !n_used || !features || n_mc < 1 || n_sub < 1 || K < 1 || K > 4096 || !(norm > 0.0)) {
        g_mlp_error = "invalid region feature arguments";
        return NR_ERR_INVALID_ARG;
    }
    region_features_kernel<<<(unsigned)((int64_t)n_mc * n_sub), 64, 0, (hipStream_t)stream>>>(
        stat, n_used, n_mc, n_sub, K, norm, features);
    return hip_status(nullptr, hipGetLastError(), "region features");
}

const char* nr_mlp_last_error(nr_mlp m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

void nr_mlp_destroy(nr_mlp m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
}

}  // extern "C"
