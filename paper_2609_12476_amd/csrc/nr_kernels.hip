// gfx950 kernels of the semicoherent NUFFT resampling path.
//
//   strain_lane_major : per segment, copy the samples into the lane-major
//                       order the spreader walks (see InstDev).
//   tau               : (staged method) per sample, the resampled time offset
//                       dtau_j = tau(t_j) - tau(t_s) of Eq. (new_t) in FP64
//                       and its reduction modulo one grid period and one
//                       heterodyne cycle, written as a point stream.
//   spread            : "exponential of semicircle" kernel spreading onto a
//                       periodic grid held in LDS (one grid per wave), with
//                       per-cell Chebyshev moments; the fused method computes
//                       the point stream inline instead of loading it.
//   epilogue_*        : mixed-radix Stockham FFT in LDS, deconvolution by the
//                       kernel's Fourier transform, |X|^2, and either the
//                       per-instance outputs or the per-template segment sum.
//
// Type-I NUFFT construction (Sec. III.B and App. A: interpolation with a
// kernel onto a uniform grid followed by an FFT): with the band centre f_c
// and grid period df, c_j = x_j exp(-2 pi i f_c dtau_j) is spread at grid
// position n * frac(df dtau_j); the DFT of the grid at mode m, divided by the
// kernel's Fourier transform at 2 pi m / n, approximates
// sum_j c_j exp(-2 pi i m df dtau_j) = X(f_c + m df).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "nr_internal.hpp"

namespace nr {

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
struct PointOf;
template <>
struct PointOf<float> {
    using type = uint2;  // (grid position, heterodyne phase) as 32-bit fractions of a period
};
template <>
struct PointOf<double> {
    using type = double2;  // the same two fractions in FP64
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }


// ------------------------------------------------------------------ tau --

constexpr int kHornerFast = 16;   // tau series degrees evaluated from registers

// Resampling constants of the wave's instance, loaded once per wave
// (uniform, so they live in scalar registers).
struct TauConsts {
    double a, c, df, fc, hn;
    int ndeg, L;
    const double* b;               // Horner coefficients (global; zero padded)
    double bc[kHornerFast];
};

__device__ __forceinline__ void load_tau(TauConsts& t, const InstDev& d,
                                         const double* __restrict__ coef, double hn)
{
    t.a = d.a;
    t.c = d.c;
    t.df = d.df;
    t.fc = d.fc;
    t.hn = hn;
    t.ndeg = d.ndeg;
    t.L = d.L;
    t.b = coef + d.coef_off;
#pragma unroll
    for (int k = 0; k < kHornerFast; ++k) t.bc[k] = t.b[k];  // the array carries kHornerFast zeros of padding
}

template <int N>
__device__ __forceinline__ double horner(const double* b, double x)
{
    double acc = b[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) acc = fma(acc, x, b[k]);
    return acc * x;
}

// dtau_j = tau(t_s + j/fs) - tau(t_s) of Eq. (new_t).  With
// y = (8/3) beta j / (u_s fs), dtau = a (1 - (1 - y)^{5/8}); the binomial
// series in y is a polynomial in j whose coefficients the plan stores per
// instance (Horner in FP64); instances whose series converges too slowly use
// a * (-expm1((5/8) log1p(-y))).  Both forms avoid the cancellation of the
// direct difference of two values of size 3/(5 beta).
// FALLBACK: also the log1p/expm1 form (the tau kernel); the fused
// spreaders only ever see series instances and leave it out, which keeps
// their register count low.
template <bool FALLBACK = true>
__device__ __forceinline__ double dtau_of(const TauConsts& t, int j)
{
    const double jd = (double)j;
    switch (t.ndeg) {
    case 0: return jd * t.c;
#define NR_H(N) \
    case N: return horner<N>(t.bc, jd);
        NR_H(1) NR_H(2) NR_H(3) NR_H(4) NR_H(5) NR_H(6) NR_H(7) NR_H(8) NR_H(9) NR_H(10) NR_H(11)
        NR_H(12) NR_H(13) NR_H(14) NR_H(15) NR_H(16)
#undef NR_H
    default:
        break;
    }
    if (!FALLBACK || t.ndeg > 0) {
        double acc = t.b[t.ndeg - 1];
        for (int k = t.ndeg - 2; k >= 0; --k) acc = fma(acc, jd, t.b[k]);
        return acc * jd;
    }
    return t.a * (-expm1(0.625 * log1p(-t.c * jd)));
}

// dtau of the four samples j0 .. j0+3 of a quad (series form only): one
// dispatch on the degree for all four.
// top: b[N - 1] held in a vector register for the whole loop (a VALU
// operation may read only one scalar operand, so starting each Horner
// chain from it saves a move per sample).
template <int N>
__device__ __forceinline__ void horner4(const double* b, double top, double jd0, double* out)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double x = jd0 + (double)e;
        double acc = top;
#pragma unroll
        for (int k = N - 2; k >= 0; --k) acc = fma(acc, x, b[k]);
        out[e] = acc * x;
    }
}

__device__ __forceinline__ void dtau4(const TauConsts& t, double top, double jd0, double* out)
{
    switch (t.ndeg) {
    case 0:
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = (jd0 + (double)e) * t.c;
        return;
#define NR_H4(N) \
    case N: horner4<N>(t.bc, top, jd0, out); return;
        NR_H4(1) NR_H4(2) NR_H4(3) NR_H4(4) NR_H4(5) NR_H4(6) NR_H4(7) NR_H4(8) NR_H4(9) NR_H4(10)
        NR_H4(11) NR_H4(12) NR_H4(13) NR_H4(14) NR_H4(15) NR_H4(16)
#undef NR_H4
    default:
        break;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double jd = jd0 + (double)e;
        double acc = t.b[t.ndeg - 1];
        for (int k = t.ndeg - 2; k >= 0; --k) acc = fma(acc, jd, t.b[k]);
        out[e] = acc * jd;
    }
}

// The two reductions modulo one period, in FP64:
//   pos   = frac(df dtau - w/(2n))  (grid position of the support's start, in periods)
//   phase = frac(fc dtau)           (heterodyne phase, in cycles)
struct Reduced {
    double pos, phase;
};

template <bool FALLBACK = true>
__device__ __forceinline__ Reduced reduce_point(const TauConsts& t, int j)
{
    const double dt = dtau_of<FALLBACK>(t, j);
    Reduced r;
    r.pos = __builtin_amdgcn_fract(fma(t.df, dt, -t.hn));
    r.phase = __builtin_amdgcn_fract(t.fc * dt);
    return r;
}

// 32-bit fixed-point fraction of a value in [0, 1) (truncating).
__device__ __forceinline__ uint32_t to_u32(double f) { return (uint32_t)ldexp(f, 32); }

template <typename T>
__device__ __forceinline__ typename PointOf<T>::type pack_point(Reduced r);
template <>
__device__ __forceinline__ uint2 pack_point<float>(Reduced r)
{
    return make_uint2(to_u32(r.pos), to_u32(r.phase));
}
template <>
__device__ __forceinline__ double2 pack_point<double>(Reduced r)
{
    return make_double2(r.pos, r.phase);
}

template <typename T>
__device__ __forceinline__ Reduced unpack_point(typename PointOf<T>::type p);
template <>
__device__ __forceinline__ Reduced unpack_point<float>(uint2 p)
{
    return Reduced{ldexp((double)p.x, -32), ldexp((double)p.y, -32)};
}
template <>
__device__ __forceinline__ Reduced unpack_point<double>(double2 p)
{
    return Reduced{p.x, p.y};
}

__device__ __forceinline__ double half_width_periods(int w, int n) { return 0.5 * (double)w / (double)n; }

// Logical workgroup of this hardware workgroup in a single-class spread
// launch: the plan may hand each XCD a segment-local share of the work.
__device__ __forceinline__ int64_t logical_block(const SpreadArgs& a)
{
    return a.block_order ? (int64_t)a.block_order[blockIdx.x] : (int64_t)blockIdx.x;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void tau_kernel(SpreadArgs a)
{
    using P = typename PointOf<T>::type;
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int parts = a.parts;
    int64_t item;
    int part;
    if (parts <= 4) {
        item = (int64_t)blockIdx.x * (4 / parts) + wave / parts;
        part = wave % parts;
    } else {
        item = (int64_t)blockIdx.x / (parts / 4);
        part = (int)((int64_t)blockIdx.x % (parts / 4)) * 4 + wave;
    }
    if (item >= a.count) return;
    const InstDev d = a.inst[a.first + item];
    TauConsts tc;
    load_tau(tc, d, a.coef, half_width_periods(a.w, a.n));
    const int C = d.C;
    const int v = part * kWave + lane;
    P* out = reinterpret_cast<P*>(a.points) + (d.pt_off - a.pt_base) + (int64_t)part * C * kWave + lane;
    for (int s = 0; s < C; ++s) {
        const int j = v * C + s;
        P pt;
        if (j < d.L) {
            pt = pack_point<T>(reduce_point(tc, j));
        } else {
            pt.x = 0;
            pt.y = 0;
        }
        out[(int64_t)s * kWave] = pt;
    }
}

// ------------------------------------------------------------------ FFT --

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return cpx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b)
{
    return cpx<T>{a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b)
{
    return cpx<T>{a.x - b.x, a.y - b.y};
}
// -i z
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a)
{
    return cpx<T>{a.y, -a.x};
}

// In-register DFT of length R (forward sign): y_q = sum_r v_r exp(-2 pi i r q / R).
template <typename T>
__device__ __forceinline__ void dft_small(cpx<T>* v, int R)
{
    if (R == 2) {
        const cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 3) {
        const T s3 = T(0.86602540378443864676);
        const cpx<T> t = cadd(v[1], v[2]);
        const cpx<T> d = csub(v[1], v[2]);
        const cpx<T> m = cpx<T>{v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
        const cpx<T> r = cpx<T>{s3 * d.y, -s3 * d.x};  // -i s3 d
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    } else if (R == 4) {
        const cpx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        const cpx<T> c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, mul_mi(d));
        v[3] = csub(b, mul_mi(d));
    } else {  // R == 5
        const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
        const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
        const cpx<T> t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
        const cpx<T> t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
        const cpx<T> a1 = cpx<T>{v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
        const cpx<T> a2 = cpx<T>{v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
        const cpx<T> b1 = cpx<T>{s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
        const cpx<T> b2 = cpx<T>{s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, mul_mi(b1));
        v[4] = csub(a1, mul_mi(b1));
        v[2] = cadd(a2, mul_mi(b2));
        v[3] = csub(a2, mul_mi(b2));
    }
}

// Lanes cooperating on one transform: 16 for grids up to 128 points (sixteen
// transforms per workgroup), one wave up to 512, the whole workgroup above
// (which keeps the LDS of the largest grids within one workgroup).
__host__ __device__ __forceinline__ int team_size_for(int n) { return n <= 128 ? 16 : (n <= 512 ? kWave : kBlock); }

// Synchronise the lanes of a team: teams inside one wave only need their LDS
// writes completed (the wave runs in lockstep); larger teams use the
// workgroup barrier.  Uniform across the workgroup.
__device__ __forceinline__ void team_sync(int ts)
{
    if (ts > kWave) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// Stockham autosort FFT of the team's n points (ping-pong between buf[0..n)
// and buf[n..2n)).  Pass with radix R and span Ns (product of the earlier
// radices): butterfly j (0 <= j < n/R) takes inputs j + r n/R, applies the
// twiddles exp(-2 pi i r k / (Ns R)) with k = j mod Ns, and writes output q
// to (j / Ns) Ns R + k + q Ns.  tw is the LDS copy of exp(-2 pi i t / n).
// Every lane of the workgroup runs every pass.  Returns the buffer holding
// the result.
// One pass of radix R (a compile-time constant, so the R values of a
// butterfly stay in registers).
template <typename T, int R>
__device__ __forceinline__ void fft_pass(const cpx<T>* src, cpx<T>* dst, const cpx<T>* tw, int n, int Ns, int tid,
                                         int ts)
{
    const int nb = n / R;
    const int twstep = n / (Ns * R);
    for (int j = tid; j < nb; j += ts) {
        const int k = j % Ns;
        cpx<T> v[R];
        v[0] = src[j];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(src[j + r * nb], tw[r * k * twstep]);
        dft_small(v, R);
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[base + q * Ns] = v[q];
    }
}

template <typename T>
__device__ cpx<T>* fft_team(cpx<T>* buf, const cpx<T>* tw, const FftPlanDev& fp, int tid, int ts)
{
    const int n = fp.n;
    cpx<T>* src = buf;
    cpx<T>* dst = buf + n;
    int Ns = 1;
    const int nr = fp.nr;
    for (int p = 0; p < nr; ++p) {
        const int R = fp.radix[p];
        switch (R) {
        case 2: fft_pass<T, 2>(src, dst, tw, n, Ns, tid, ts); break;
        case 3: fft_pass<T, 3>(src, dst, tw, n, Ns, tid, ts); break;
        case 4: fft_pass<T, 4>(src, dst, tw, n, Ns, tid, ts); break;
        default: fft_pass<T, 5>(src, dst, tw, n, Ns, tid, ts); break;
        }
        team_sync(ts);
        cpx<T>* t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
    return src;
}

// --------------------------------------------------------------- spread --

// exp(2 pi i k / N) for k < N, the coarse part of the FP64 heterodyne phasor
// (FP32 classes take the phase's cosine and sine from the hardware).
template <typename T>
struct PhaseTable;
template <>
struct PhaseTable<double> {
    static constexpr int bits = 8;    // 256 entries; fine angle |theta| <= pi/256
};

// Decoded point: first grid cell g of its support (in [1, n]), the
// Chebyshev variable u = 2 (g - (x - w/2)) - 1 in (-1, 1], and the
// heterodyned strength (cr, ci) = x_j exp(-2 pi i phase).
template <typename T>
struct Decoded {
    int g;
    T u, cr, ci;
};

// Units of the phase argument of heterodyne_scaled: 2^-kPhaseShift cycles
// (FP64: table steps; FP32: cycles).
template <typename T>
constexpr int phase_shift()
{
    if constexpr (sizeof(T) == 4) return 0;
    else return PhaseTable<T>::bits;
}
template <typename T>
constexpr int kPhaseShift = phase_shift<T>();

// Entries of the phase table a spreader workgroup keeps in LDS.
template <typename T>
constexpr int phase_table_entries()
{
    if constexpr (sizeof(T) == 4) return 0;
    else return 1 << PhaseTable<T>::bits;
}

// Heterodyned sample value c = x exp(-2 pi i phase), sc = phase 2^kPhaseShift.
// FP32: the phase is reduced to [-1/2, 1/2] cycle in FP64 and its cosine and
// sine come from the hardware's transcendental unit (arguments in cycles;
// largest error 1.3e-7 over that range, measured on the device), which works
// beside the vector ALU.  FP64: N = 2^B table entries, sc = k + theta N /
// (2 pi), |theta| <= pi / N, the entry times a series in theta; this needs
// |sc| < 2^31, the range of the 32-bit conversion of k that picks the entry:
// the plan gives instances whose phase spans 2^30 table steps or more to the
// staged method, whose points carry the phase already reduced modulo one
// cycle.
template <typename T, bool CPLX>
__device__ __forceinline__ void heterodyne_scaled(double sc, T xr, T xi, const cpx<T>* tab, T& cr, T& ci)
{
    T cs, sn;   // exp(i 2 pi phase) = cs + i sn
    if constexpr (sizeof(T) == 4) {
        const float f = (float)(sc - rint(sc));
        cs = __builtin_amdgcn_cosf(f);
        sn = __builtin_amdgcn_sinf(f);
    } else {
        constexpr int B = PhaseTable<T>::bits;
        const double k = rint(sc);
        const T th = (T)((sc - k) * (6.283185307179586476925 / (double)(1 << B)));
        const cpx<T> e = tab[(int)k & ((1 << B) - 1)];
        const T t2 = th * th;
        const T c = fma(t2, fma(t2, fma(t2, T(-1.0 / 720.0), T(1.0 / 24.0)), T(-0.5)), T(1));
        const T s = fma(th * t2, fma(t2, fma(t2, T(-1.0 / 5040.0), T(1.0 / 120.0)), T(-1.0 / 6.0)), th);
        cs = e.x * c - e.y * s;
        sn = e.y * c + e.x * s;
    }
    // strength = x * conj(exp(i 2 pi phase))
    if (CPLX) {
        cr = xr * cs + xi * sn;
        ci = xi * cs - xr * sn;
    } else {
        cr = xr * cs;
        ci = -xr * sn;
    }
}

// The same from the phase in cycles.
template <typename T, bool CPLX>
__device__ __forceinline__ void heterodyne(double phase, T xr, T xi, const cpx<T>* tab, T& cr, T& ci)
{
    heterodyne_scaled<T, CPLX>(phase * (double)(1 << kPhaseShift<T>), xr, xi, tab, cr, ci);
}

// Fused path: cell and position straight from dtau.  S = x n with
// x = df dtau - w/(2n); g = floor(S) + 1 is the unwrapped cell of the
// support's first tap (the flush reduces it mod n) and frac(S) =
// frac(frac(x) n) its position in that cell.
template <typename T, bool CPLX>
__device__ __forceinline__ Decoded<T> decode_dt(double dt, double dfn, double hnn, double fcs, T xr, T xi,
                                                const cpx<T>* tab)
{
    Decoded<T> o;
    const double S = fma(dfn, dt, -hnn);
    const double fl = floor(S);
    o.g = (int)fl + 1;
    o.u = (T)fma(-2.0, S - fl, 1.0);
    heterodyne_scaled<T, CPLX>(fcs * dt, xr, xi, tab, o.cr, o.ci);
    return o;
}

template <typename T, bool CPLX>
__device__ __forceinline__ Decoded<T> decode(Reduced r, T xr, T xi, int n, const cpx<T>* tab)
{
    Decoded<T> o;
    const double S = r.pos * (double)n;           // (x - w/2) mod n, in cells
    const double fl = floor(S);
    // in [1, n + 1]; n + 1 (S rounded up to n) is cell 1 again, which the
    // flush's single modulo step maps correctly
    o.g = (int)fl + 1;
    o.u = (T)fma(-2.0, S - fl, 1.0);
    heterodyne<T, CPLX>(r.phase, xr, xi, tab, o.cr, o.ci);
    return o;
}

template <typename T, int D>
struct Moments {
    T re[D + 1];
    T im[D + 1];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int p = 0; p <= D; ++p) re[p] = im[p] = T(0);
    }
    // Add c * T_p(u) for p = 0..D (Chebyshev recurrence).
    __device__ __forceinline__ void add(T u, T cr, T ci)
    {
        re[0] += cr;
        im[0] += ci;
        if (D >= 1) {
            re[1] = fma(cr, u, re[1]);
            im[1] = fma(ci, u, im[1]);
        }
        T t0 = T(1), t1 = u;
        const T u2 = u + u;
#pragma unroll
        for (int p = 2; p <= D; ++p) {
            const T t2 = fma(u2, t1, -t0);
            re[p] = fma(cr, t2, re[p]);
            im[p] = fma(ci, t2, im[p]);
            t0 = t1;
            t1 = t2;
        }
    }
};

__device__ __forceinline__ void lds_add(float* p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Turn the moments of every point whose support starts at cell g into the
// w tap sums and add them to the wave's LDS grid:
//   tap t = sum_p A[t][p] M_p, added at cell (g + t) mod n.
template <typename T, int D>
__device__ __forceinline__ void flush(const Moments<T, D>& M, int g, const T* __restrict__ A,
                                      cpx<T>* grid, int n, int w)
{
    // g may be any integer (an unwrapped cell index): reduce it mod n once
    g %= n;
    if (g < 0) g += n;
    for (int t = 0; t < w; ++t) {
        const T* At = A + t * (D + 1);
        T vr = T(0), vi = T(0);
#pragma unroll
        for (int p = 0; p <= D; ++p) {
            vr = fma(At[p], M.re[p], vr);
            vi = fma(At[p], M.im[p], vi);
        }
        int cell = g + t;
        if (cell >= n) cell -= n;
        lds_add(&grid[cell].x, vr);
        lds_add(&grid[cell].y, vi);
    }
}

// Whole-wave lane shifts (DPP): lane i receives lane i - 1's value; shr
// gives lane 0 zero, ror gives it lane 63's.
__device__ __forceinline__ int dpp_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_ror1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x13C, 0xF, 0xF, false); }
// lane i receives lane i + 1's value (lane 63 receives zero)
__device__ __forceinline__ int dpp_shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false); }
template <bool ROT>
__device__ __forceinline__ float wave_shift(float v)
{
    const int b = __float_as_int(v);
    return __int_as_float(ROT ? dpp_ror1(b) : dpp_shr1(b));
}
template <bool ROT>
__device__ __forceinline__ double wave_shift(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    const int l2 = ROT ? dpp_ror1(lo) : dpp_shr1(lo);
    const int h2 = ROT ? dpp_ror1(hi) : dpp_shr1(hi);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)h2 << 32) | (unsigned)l2));
}

// Flush of one cell-run round.  Lane v holds the moments of the points
// whose support starts at cell g = U_r + v + 1 (consecutive cells over the
// wave's lanes; a lane without a cell holds zero moments), so tap t of lane
// v lands on cell g + t, which is also where tap t - 1 of lane v + 1 lands.  The taps are summed across lanes in registers
// first: folding taps t = w - 1 .. 0 into h = shift(h) + tap_t leaves lane
// v with the sum of tap_s of lane v - s over s, everything that this round
// adds to its cell g; the same chain with rotation, fed only by the lanes
// whose supports pass the round's last cell (v >= 65 - w), leaves lanes
// v < w - 1 with what lands on cell g + 64.  Each lane then makes one LDS
// addition per component (two for the lanes carrying that spill) instead of
// w.  Every lane takes part (empty runs have zero moments), and the order of
// the additions is fixed, so the result does not depend on scheduling.
template <typename T, int D>
__device__ __forceinline__ void flush_round(const Moments<T, D>& M, int g, int lane, const T* __restrict__ A,
                                            cpx<T>* grid, int n, int w)
{
    const bool spill = lane >= kWave + 1 - w;
    T hr = T(0), hi = T(0), sr = T(0), si = T(0);
    for (int t = w - 1; t >= 0; --t) {
        const T* At = A + t * (D + 1);
        T vr = T(0), vi = T(0);
#pragma unroll
        for (int p = 0; p <= D; ++p) {
            vr = fma(At[p], M.re[p], vr);
            vi = fma(At[p], M.im[p], vi);
        }
        hr = wave_shift<false>(hr) + vr;
        hi = wave_shift<false>(hi) + vi;
        sr = wave_shift<true>(sr) + (spill ? vr : T(0));
        si = wave_shift<true>(si) + (spill ? vi : T(0));
    }
    int c = g % n;
    if (c < 0) c += n;
    lds_add(&grid[c].x, hr);
    lds_add(&grid[c].y, hi);
    if (lane < w - 1) {
        const int c2 = (c + kWave) % n;
        lds_add(&grid[c2].x, sr);
        lds_add(&grid[c2].y, si);
    }
}

// Flush the difference of two cumulative moment snapshots.
template <typename T, int D>
__device__ __forceinline__ void flush_diff(const Moments<T, D>& E, const Moments<T, D>& P, int g,
                                           const T* __restrict__ A, cpx<T>* grid, int n, int w)
{
    Moments<T, D> V;
#pragma unroll
    for (int p = 0; p <= D; ++p) {
        V.re[p] = E.re[p] - P.re[p];
        V.im[p] = E.im[p] - P.im[p];
    }
    flush<T, D>(V, g, A, grid, n, w);
}

// Grid stride of a spreader workgroup's per-wave grids: a second grid per
// wave when the fused epilogue runs an instance's FFT within one wave.
__device__ __forceinline__ int grid_stride(const SpreadArgs& a, int wpi) { return (a.epi_fused && wpi == 1) ? 2 * a.n : a.n; }

// After spreading, the instance's grids (one per wave of the instance, at
// lds + (first_wave + q) gstride) become either its partial grid in global
// memory (call mode 0, or a class without the fused epilogue: a separate
// epilogue kernel follows) or, fused, are summed into the first wave's grid,
// transformed in LDS by the instance's waves (the grid after it is the
// Stockham ping-pong half: the next wave's grid, or the wave's own second
// grid), deconvolved and written as power rows (mode 1) or spectra / power
// (mode 2), with the arithmetic of the separate epilogue.
// Every wave of the workgroup takes part (the transforms synchronise);
// waves past the last instance transform their zero grids and write nothing.
template <typename T>
__device__ __forceinline__ void finish_instance(const SpreadArgs& a, const EpilogueOut& o, int64_t item, int slot,
                                                cpx<T>* lds, int wave, int lane, int wpi)
{
    const int n = a.n;
    const int gs = grid_stride(a, wpi);
    const int first_wave = (wave / wpi) * wpi;
    const bool live = item < a.count;
    if (!a.epi_fused || o.mode == 0) {
        if (!live) return;
        // Sum the grids of the instance's waves in this workgroup in wave
        // order and store them as the workgroup's partial grid (slot).
        cpx<T>* out = reinterpret_cast<cpx<T>*>(a.grid) + (item * grid_slots(a.parts) + slot) * n;
        for (int c = (wave % wpi) * kWave + lane; c < n; c += kWave * wpi) {
            T r = T(0), i = T(0);
            for (int q = 0; q < wpi; ++q) {
                const cpx<T> gv = lds[(first_wave + q) * gs + c];
                r += gv.x;
                i += gv.y;
            }
            out[c] = cpx<T>{r, i};
        }
        return;
    }
    cpx<T>* buf = lds + first_wave * gs;
    const int ts = wpi * kWave, tid = (wave % wpi) * kWave + lane;
    if (wpi > 1) {
        for (int c = tid; c < n; c += ts) {
            T r = T(0), i = T(0);
            for (int q = 0; q < wpi; ++q) {
                const cpx<T> gv = lds[(first_wave + q) * gs + c];
                r += gv.x;
                i += gv.y;
            }
            buf[c] = cpx<T>{r, i};
        }
    }
    __syncthreads();
    const cpx<T>* res = fft_team<T>(buf, reinterpret_cast<const cpx<T>*>(a.twiddle), a.fft, tid, ts);
    if (!live) return;
    const InstDev d = a.inst[a.first + item];
    const T* __restrict__ dec = reinterpret_cast<const T*>(a.dec);
    for (int k = tid; k < d.K; k += ts) {
        int l = k - d.m0;
        if (l < 0) l += n;
        const T f = dec[l];
        const cpx<T> X = cpx<T>{res[l].x * f, res[l].y * f};
        if (o.out_fp64) {
            const double pw = (double)X.x * (double)X.x + (double)X.y * (double)X.y;
            if (o.mode == 1) {
                reinterpret_cast<double*>(o.rows)[a.row_base + (int64_t)d.entry * a.kmax + k] = pw;
            } else {
                if (o.spectra) reinterpret_cast<cpx<double>*>(o.spectra)[d.bin_off + k] = cpx<double>{(double)X.x, (double)X.y};
                if (o.power) reinterpret_cast<double*>(o.power)[d.bin_off + k] = pw;
            }
        } else {
            const float pw = (float)X.x * (float)X.x + (float)X.y * (float)X.y;
            if (o.mode == 1) {
                reinterpret_cast<float*>(o.rows)[a.row_base + (int64_t)d.entry * a.kmax + k] = pw;
            } else {
                if (o.spectra) reinterpret_cast<cpx<float>*>(o.spectra)[d.bin_off + k] = cpx<float>{(float)X.x, (float)X.y};
                if (o.power) reinterpret_cast<float*>(o.power)[d.bin_off + k] = pw;
            }
        }
    }
}

// One wave per (instance, part).  Each lane walks its run of samples in
// order; because tau is monotone in t the support's first cell g only
// moves forward (and wraps once per period), so a lane keeps the Chebyshev
// moments of the points sharing one g and turns them into kernel taps only
// when g changes.  A change parks the finished cell; parked cells are
// flushed by the whole wave every flush_period steps (or at once if a lane
// changes cell twice within a period).
//   SNAP = false: the moments restart at zero for every cell and the
//                 finished ones are parked (copied) aside.
//   SNAP = true:  the moments are cumulative over the lane's run; a change
//                 only copies them into a snapshot, and a flush turns the
//                 difference of two snapshots into taps.
// Each wave owns its grid copy, so the LDS additions of one grid come from
// one wave in program order and the result does not depend on scheduling.
template <typename T, int D, bool FUSED, bool CPLX, bool SNAP>
__device__ __forceinline__ void spread_block(const SpreadArgs& a, const EpilogueOut& o, int64_t lblock)
{
    using P = typename PointOf<T>::type;
    constexpr int NT = phase_table_entries<T>();   // FP32: no table (hardware sine and cosine)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* tab = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* lds = tab + NT;

    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int parts = a.parts;
    const int n = a.n, w = a.w;
    // waves of one instance inside this workgroup
    const int wpi = parts < 4 ? parts : 4;
    cpx<T>* grid = lds + wave * grid_stride(a, wpi);
    const cpx<T>* gtab = reinterpret_cast<const cpx<T>*>(a.phase_table);
    for (int k = threadIdx.x; k < NT; k += kBlock) tab[k] = gtab[k];
    for (int c = lane; c < n; c += kWave) grid[c] = cpx<T>{T(0), T(0)};
    __syncthreads();

    // which instance, which part
    int64_t item;
    int part, slot = 0;
    if (parts <= 4) {
        item = lblock * (4 / parts) + wave / parts;
        part = wave % parts;
    } else {
        item = lblock / (parts / 4);
        slot = (int)(lblock % (parts / 4));
        part = slot * 4 + wave;
    }
    const T* __restrict__ A = reinterpret_cast<const T*>(a.taps);

    if (item < a.count) {
        const InstDev d = a.inst[a.first + item];
        TauConsts tc;
        load_tau(tc, d, a.coef, half_width_periods(w, n));
        const int C = d.C;
        const int L = d.L;
        const int v = part * kWave + lane;
        const int64_t row0 = (int64_t)part * C * kWave + lane;
        const P* __restrict__ pts =
            FUSED ? nullptr
                  : reinterpret_cast<const P*>(a.points) + (d.pt_off - a.pt_base) + row0;
        const int64_t xs0 = d.strain_off + row0;
        const int fmask = a.flush_period - 1;
        // fused: grid position in cells and phase in table steps per unit dtau
        const double dfn = tc.df * (double)n, hnn = tc.hn * (double)n;
        const double fcs = tc.fc * (double)(1 << kPhaseShift<T>);

        // SNAP: M cumulative, E = snapshot at the end of the parked cell,
        //       S = snapshot at its start.
        // otherwise: M for the current cell, E = the parked cell's moments.
        Moments<T, D> M, E, S;
        M.zero();
        E.zero();
        if (SNAP) S.zero();
        // cells are unwrapped integers on the fused path (any sign)
        constexpr int kNone = INT_MIN;
        int g_cur = kNone, g_pend = kNone;
        for (int s = 0; s < C; ++s) {
            const int j = v * C + s;
            if (j < L) {
                T xr, xi;
                if (CPLX) {
                    const cpx<T> xv = reinterpret_cast<const cpx<T>*>(a.strain_lm)[xs0 + (int64_t)s * kWave];
                    xr = xv.x;
                    xi = xv.y;
                } else {
                    xr = reinterpret_cast<const T*>(a.strain_lm)[xs0 + (int64_t)s * kWave];
                    xi = T(0);
                }
                const Decoded<T> q = FUSED ? decode_dt<T, CPLX>(dtau_of<false>(tc, j), dfn, hnn, fcs, xr, xi, tab)
                                           : decode<T, CPLX>(unpack_point<T>(pts[(int64_t)s * kWave]), xr, xi, n, tab);
                if (q.g != g_cur) {
                    if (g_cur != kNone) {
                        if (SNAP) {
                            if (g_pend != kNone) {
                                flush_diff<T, D>(E, S, g_pend, A, grid, n, w);
                                S = E;
                            }
                        } else {
                            if (g_pend != kNone) flush<T, D>(E, g_pend, A, grid, n, w);
                        }
                        E = M;
                        g_pend = g_cur;
                    }
                    if (!SNAP) M.zero();
                    g_cur = q.g;
                }
                M.add(q.u, q.cr, q.ci);
            }
            if ((s & fmask) == fmask) {
                if (g_pend != kNone) {
                    if (SNAP) {
                        flush_diff<T, D>(E, S, g_pend, A, grid, n, w);
                        S = E;
                    } else {
                        flush<T, D>(E, g_pend, A, grid, n, w);
                    }
                    g_pend = kNone;
                }
            }
        }
        if (SNAP) {
            if (g_pend != kNone) {
                flush_diff<T, D>(E, S, g_pend, A, grid, n, w);
                S = E;
            }
            if (g_cur != kNone) flush_diff<T, D>(M, S, g_cur, A, grid, n, w);
        } else {
            if (g_pend != kNone) flush<T, D>(E, g_pend, A, grid, n, w);
            if (g_cur != kNone) flush<T, D>(M, g_cur, A, grid, n, w);
        }
    }
    __syncthreads();
    finish_instance<T>(a, o, item, slot, lds, wave, lane, wpi);
}

template <typename T, int D, bool FUSED, bool CPLX, bool SNAP>
__global__ __launch_bounds__(kBlock) void spread_kernel(SpreadArgs a, EpilogueOut o)
{
    spread_block<T, D, FUSED, CPLX, SNAP>(a, o, logical_block(a));
}

// ------------------------------------------------- cell-run schedule --
//
// S_j = n (df dtau_j) - w/2 is sample j's grid coordinate in cells, not
// reduced modulo the grid; it grows with j, so the unwrapped cell index
// U_j = floor(S_j) never decreases and the samples sharing one value of U
// form a contiguous run.  A wave takes 63 consecutive cells per round: lane
// v finds the first sample of the run of cell U_0 + 63 r + v by a bracketed
// binary search, the lane before it ends there (lane 63's search only ends
// lane 62's run), every lane accumulates its run's moments without a cell
// change (its Chebyshev
// variable is 1 - 2 (S_j - U), from the same S_j that placed the sample in
// the run), and all lanes flush together.  The strain is read as aligned
// quads of samples from a plain per-segment copy.

__device__ __forceinline__ double grid_coord(double dfn, double hnn, double dt) { return fma(dfn, dt, -hnn); }

// The first sample j in [0, L] with S_j >= t (L if none).  dtau is convex in
// j (its series has positive coefficients), so S lies below its chord
// S_0 + m j and above its tangent S_0 + s0 j at j = 0: every j below
// (t - S_0) / m has S_j < t and every j from (t - S_0) / s0 on has S_j >= t.
// The search runs inside that bracket, widened by two samples against
// rounding (inv_m = 1 / m, inv_s0 = 1 / s0).
// The bisection for a series of degree N fixed at compile time (N < 0: any
// degree), so that its loop carries no dispatch on the degree; the
// operations are those of dtau_of.
template <int N>
__device__ __forceinline__ int bisect_at_least(const TauConsts& tc, int lo, int hi, double t, double dfn, double hnn)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double jd = (double)mid;
        double dt;
        if constexpr (N < 0) {
            dt = dtau_of<false>(tc, mid);
        } else if constexpr (N == 0) {
            dt = jd * tc.c;
        } else {
            double acc = tc.bc[N - 1];
#pragma unroll
            for (int k = N - 2; k >= 0; --k) acc = fma(acc, jd, tc.bc[k]);
            dt = acc * jd;
        }
        if (grid_coord(dfn, hnn, dt) < t)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int first_at_least(const TauConsts& tc, int L, double t, double dfn, double hnn,
                                              double inv_m, double inv_s0)
{
    const double d = t + hnn;                     // t - S_0, S_0 = -hnn
    const int lo = (int)fmin(fmax(ceil(d * inv_m) - 2.0, 0.0), (double)L);
    const int hi = (int)fmin(fmax(ceil(d * inv_s0) + 2.0, 0.0), (double)L);
    switch (tc.ndeg) {
#define NR_B(N) \
    case N: return bisect_at_least<N>(tc, lo, hi, t, dfn, hnn);
        NR_B(0) NR_B(1) NR_B(2) NR_B(3) NR_B(4) NR_B(5) NR_B(6) NR_B(7) NR_B(8) NR_B(9) NR_B(10) NR_B(11)
        NR_B(12) NR_B(13) NR_B(14) NR_B(15) NR_B(16)
#undef NR_B
    default: return bisect_at_least<-1>(tc, lo, hi, t, dfn, hnn);
    }
}

template <typename E>
struct alignas(16) Quad {
    E v[4];
};

// Four consecutive samples q .. q+3 (jq = q as a double) of the cell run
// whose Chebyshev variable is u = u1 - 2 S_j (u1 = 1 + 2 U) into the
// moments; MASK: samples outside [js, je) enter with zero strength.
template <typename T, int D, bool CPLX, bool MASK, typename E>
__device__ __forceinline__ void cell_quad(const TauConsts& tc, double top, const E* __restrict__ xs, int q,
                                          double jq, int js, int je, double dfn, double hnn, double u1,
                                          double fcs, const cpx<T>* tab, Moments<T, D>& M)
{
    const Quad<E> xq = *reinterpret_cast<const Quad<E>*>(xs + q);
    double dt[4];
    dtau4(tc, top, jq, dt);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int j = q + e;
        const bool in = MASK ? ((j >= js) & (j < je)) : true;
        const T u = (T)fma(-2.0, grid_coord(dfn, hnn, dt[e]), u1);
        T xr, xi, cr, ci;
        if constexpr (CPLX) {
            xr = in ? xq.v[e].x : T(0);
            xi = in ? xq.v[e].y : T(0);
        } else {
            xr = in ? xq.v[e] : T(0);
            xi = T(0);
        }
        heterodyne_scaled<T, CPLX>(fcs * dt[e], xr, xi, tab, cr, ci);
        M.add(u, cr, ci);
    }
}

template <typename T, int D, bool CPLX>
__device__ __forceinline__ void spread_runs_block(const SpreadArgs& a, const EpilogueOut& o, int64_t lblock)
{
    constexpr int NT = phase_table_entries<T>();   // FP32: no table (hardware sine and cosine)
    using E = typename std::conditional<CPLX, cpx<T>, T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* tab = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* lds = tab + NT;

    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int parts = a.parts;
    const int n = a.n, w = a.w;
    const int wpi = parts < 4 ? parts : 4;
    cpx<T>* grid = lds + wave * grid_stride(a, wpi);
    const cpx<T>* gtab = reinterpret_cast<const cpx<T>*>(a.phase_table);
    for (int k = threadIdx.x; k < NT; k += kBlock) tab[k] = gtab[k];
    for (int c = lane; c < n; c += kWave) grid[c] = cpx<T>{T(0), T(0)};
    __syncthreads();

    int64_t item;
    int part, slot = 0;
    if (parts <= 4) {
        item = lblock * (4 / parts) + wave / parts;
        part = wave % parts;
    } else {
        item = lblock / (parts / 4);
        slot = (int)(lblock % (parts / 4));
        part = slot * 4 + wave;
    }
    const T* __restrict__ A = reinterpret_cast<const T*>(a.taps);

    if (item < a.count) {
        const InstDev d = a.inst[a.first + item];
        TauConsts tc;
        load_tau(tc, d, a.coef, half_width_periods(w, n));
        const double nd = (double)n;
        const int L = d.L;
        // per-sample scales: grid coordinate in cells and phase in table steps
        const double dfn = tc.df * nd, hnn = tc.hn * nd;
        const double fcs = tc.fc * (double)(1 << kPhaseShift<T>);
        const double S1 = grid_coord(dfn, hnn, dtau_of<false>(tc, L > 0 ? L - 1 : 0));
        const double U0 = floor(-hnn), U1 = floor(S1);
        const int rounds = L > 0 ? uniform(((int)(U1 - U0) + kRunsPerRound) / kRunsPerRound) : 0;
        // reciprocal slopes of the chord and of the tangent at j = 0
        const double inv_m = L > 1 ? (double)(L - 1) / (S1 + hnn) : 0.0;
        const double inv_s0 = 1.0 / (dfn * (tc.ndeg > 0 ? tc.bc[0] : tc.c));
        const E* __restrict__ xs = reinterpret_cast<const E*>(a.strain_lm) + d.strain_off;
        // leading series coefficient, kept in a vector register
        double top = tc.ndeg > 0 ? tc.b[tc.ndeg - 1] : 0.0;
        asm volatile("" : "+v"(top));
        for (int r = part; r < rounds; r += parts) {
            // lane v < 63: cell U = U0 + 63 r + v; every lane searches the
            // start of its cell's run (the first sample at or past cell U),
            // lanes v < 63 take the end from lane v + 1, and lane 63 takes
            // no cell (its search gives lane 62's end), so one search per
            // lane and round serves both ends
            const double U = U0 + (double)(kRunsPerRound * r + lane);
            const int js = (r == 0 && lane == 0) ? 0       // S_0 >= U0 = floor(S_0)
                                                 : first_at_least(tc, L, U, dfn, hnn, inv_m, inv_s0);
            int je = dpp_shl1(js);
            if (lane == kWave - 1) je = js;
            const double u1 = fma(2.0, U, 1.0);
            Moments<T, D> M;
            M.zero();
            // whole quads: the first and last quad of a run are masked
            // (samples outside it enter with zero strength; they lie in the
            // padded copy and have finite positions), the ones between are not
            if (je > js) {
                int q = js & ~3;
                double jq = (double)q;
                cell_quad<T, D, CPLX, true>(tc, top, xs, q, jq, js, je, dfn, hnn, u1, fcs, tab, M);
                for (q += 4, jq += 4.0; q + 4 <= je; q += 4, jq += 4.0)
                    cell_quad<T, D, CPLX, false>(tc, top, xs, q, jq, js, je, dfn, hnn, u1, fcs, tab, M);
                if (q < je) cell_quad<T, D, CPLX, true>(tc, top, xs, q, jq, js, je, dfn, hnn, u1, fcs, tab, M);
            }
            // the support of the points of cell U starts at cell U + 1
            flush_round<T, D>(M, (int)U + 1, lane, A, grid, n, w);
        }
    }
    __syncthreads();
    finish_instance<T>(a, o, item, slot, lds, wave, lane, wpi);
}

// Occupancy of the cell-run kernel: six waves per SIMD (at most 80 VGPRs)
// where the FP32 moments of degree up to 7 fit there without spilling; the
// rest is left to the compiler.
template <typename T, int D, bool CPLX>
struct RunsWaves {
    static constexpr int value = (sizeof(T) == 4 && D <= 7) ? 6 : 1;
};

template <typename T, int D, bool CPLX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RunsWaves<T, D, CPLX>::value))) void
spread_runs_kernel(SpreadArgs a, EpilogueOut o)
{
    spread_runs_block<T, D, CPLX>(a, o, logical_block(a));
}

// Class of workgroup b of a multi-class launch (block_off is ascending).
__device__ __forceinline__ int class_of_block(const int64_t* __restrict__ block_off, int ncls, int64_t b)
{
    int c = 0;
    while (c + 1 < ncls && block_off[c + 1] <= b) ++c;
    return uniform(c);
}

template <typename T, int D, bool FUSED, bool CPLX, bool SNAP>
__global__ __launch_bounds__(kBlock) void spread_multi_kernel(const SpreadTable t, EpilogueOut o)
{
    const int c = class_of_block(t.block_off, t.ncls, blockIdx.x);
    spread_block<T, D, FUSED, CPLX, SNAP>(t.a[c], o, (int64_t)blockIdx.x - t.block_off[c]);
}

template <typename T, int D, bool CPLX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RunsWaves<T, D, CPLX>::value))) void
spread_runs_multi_kernel(const SpreadTable t, EpilogueOut o)
{
    const int c = class_of_block(t.block_off, t.ncls, blockIdx.x);
    spread_runs_block<T, D, CPLX>(t.a[c], o, (int64_t)blockIdx.x - t.block_off[c]);
}

// LDS layout of the epilogue kernels: twiddles [n], then per team 2n points,
// then (segment sum) per team kmax FP64 partial sums.
template <typename T>
__device__ __forceinline__ cpx<T>* stage_twiddles(unsigned char* smem, const void* g, int n)
{
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    const cpx<T>* src = reinterpret_cast<const cpx<T>*>(g);
    for (int t = threadIdx.x; t < n; t += kBlock) tw[t] = src[t];
    return tw;
}

// Load an instance's grid (sum of its partial grids, in slot order) into
// the team's buffer.
template <typename T>
__device__ __forceinline__ void load_grid(const EpilogueArgs& a, int64_t local, cpx<T>* buf, int tid, int ts)
{
    const int n = a.fft.n;
    const cpx<T>* g = reinterpret_cast<const cpx<T>*>(a.grid) + local * a.slots * n;
    for (int c = tid; c < n; c += ts) {
        cpx<T> v = g[c];
        for (int q = 1; q < a.slots; ++q) {
            const cpx<T> u = g[(int64_t)q * n + c];
            v.x += u.x;
            v.y += u.y;
        }
        buf[c] = v;
    }
}

template <typename T, typename O>
__device__ __forceinline__ void epilogue_spectra_block(const EpilogueArgs& a, const EpilogueOut& o, int64_t lblock)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.fft.n;
    const int ts = team_size_for(n);
    const int team = threadIdx.x / ts, tid = threadIdx.x % ts;
    const int nteam = kBlock / ts;
    const cpx<T>* tw = stage_twiddles<T>(smem_raw, a.twiddle, n);
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw) + n + (size_t)team * 2 * n;
    const int64_t item = lblock * nteam + team;
    const bool live = item < a.count;
    if (live) load_grid<T>(a, item, buf, tid, ts);
    __syncthreads();
    const cpx<T>* res = fft_team<T>(buf, tw, a.fft, tid, ts);
    if (!live) return;
    const InstDev d = a.inst[a.first + item];
    const T* __restrict__ dec = reinterpret_cast<const T*>(a.dec);
    cpx<O>* sp = reinterpret_cast<cpx<O>*>(o.spectra);
    O* pw = reinterpret_cast<O*>(o.power);
    O* rw = o.rows ? reinterpret_cast<O*>(o.rows) + a.row_base + (int64_t)d.entry * a.kmax : nullptr;
    for (int k = tid; k < d.K; k += ts) {
        int l = k - d.m0;
        if (l < 0) l += n;
        const T f = dec[l];
        const cpx<T> X = cpx<T>{res[l].x * f, res[l].y * f};
        if (sp) sp[d.bin_off + k] = cpx<O>{(O)X.x, (O)X.y};
        const O p = (O)X.x * (O)X.x + (O)X.y * (O)X.y;
        if (pw) pw[d.bin_off + k] = p;
        if (rw) rw[k] = p;
    }
}

// Second pass of the segment sum: the rows of one class template are
// contiguous (template-major list order); threads split them by row in a
// fixed pattern, sum in FP64 and combine the partial sums in order.
template <typename O>
__device__ __forceinline__ void rows_sum_block(const EpilogueArgs& a, const EpilogueOut& o, int64_t lblock)
{
    __shared__ double part[kBlock];
    const int ct = a.tmpl_first + (int)lblock;
    const int64_t lo = a.tmpl_list_off[ct], hi = a.tmpl_list_off[ct + 1];
    if (hi <= lo) return;  // uniform across the workgroup
    const int K = a.inst[a.tmpl_list[lo]].K;
    const O* __restrict__ rows = reinterpret_cast<const O*>(o.rows) + a.row_base;
    O* stat = reinterpret_cast<O*>(o.stat) + a.tmpl_stat_off[ct];
    const int span = K < kBlock ? K : kBlock;
    const int nsub = kBlock / span;
    const int t = threadIdx.x;
    const int sub = t / span, kk = t - sub * span;
    for (int k0 = 0; k0 < K; k0 += span) {
        const int k = k0 + kk;
        double acc = 0.0;
        if (sub < nsub && k < K) {
            for (int64_t e = lo + sub; e < hi; e += nsub) {
                const double wgt = o.seg_weight ? o.seg_weight[a.entry_seg[e]] : 1.0;
                acc += wgt * (double)rows[e * a.kmax + k];
            }
        }
        part[t] = acc;
        __syncthreads();
        if (t < span && k0 + t < K) {
            double s = 0.0;
            for (int q = 0; q < nsub; ++q) s += part[q * span + t];
            stat[k0 + t] = (O)((double)stat[k0 + t] + s);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && o.n_used) o.n_used[a.tmpl_id[ct]] += (int32_t)(hi - lo);
}

template <typename O>
__global__ __launch_bounds__(kBlock) void rows_sum_kernel(EpilogueArgs a, EpilogueOut o)
{
    rows_sum_block<O>(a, o, blockIdx.x);
}

template <typename O>
__global__ __launch_bounds__(kBlock) void rows_sum_multi_kernel(const EpilogueTable t, EpilogueOut o)
{
    const int c = class_of_block(t.block_off[1], t.ncls, blockIdx.x);
    rows_sum_block<O>(t.a[c], o, (int64_t)blockIdx.x - t.block_off[1][c]);
}

// Segment sum: one workgroup per template; its instances inside the chunk
// are shared round-robin by the teams, each team keeps FP64 partial sums,
// and the partials are added in team order, so the result is reproducible.
template <typename T, typename O>
__device__ __forceinline__ void epilogue_sum_block(const EpilogueArgs& a, const EpilogueOut& o, int64_t lblock)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.fft.n;
    const int kmax = a.kmax;
    const int ts = team_size_for(n);
    const int team = threadIdx.x / ts, tid = threadIdx.x % ts;
    const int nteam = kBlock / ts;
    const int ct = a.tmpl_first + (int)lblock;
    int64_t lo = a.tmpl_list_off[ct], hi = a.tmpl_list_off[ct + 1];
    // entries of this chunk: class instances in [first, first + count)
    {
        int64_t l = lo, h = hi;
        while (l < h) {
            const int64_t m = (l + h) >> 1;
            if (a.tmpl_list[m] < a.first) l = m + 1; else h = m;
        }
        const int64_t e0 = l;
        h = hi;
        while (l < h) {
            const int64_t m = (l + h) >> 1;
            if (a.tmpl_list[m] < a.first + a.count) l = m + 1; else h = m;
        }
        lo = e0;
        hi = l;
    }
    const int64_t cnt = hi - lo;
    if (cnt <= 0) return;  // uniform across the workgroup
    const cpx<T>* tw = stage_twiddles<T>(smem_raw, a.twiddle, n);
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw) + n + (size_t)team * 2 * n;
    double* part = reinterpret_cast<double*>(reinterpret_cast<cpx<T>*>(smem_raw) + n + (size_t)nteam * 2 * n);
    double* mine = part + (size_t)team * kmax;
    const InstDev d0 = a.inst[a.tmpl_list[lo]];
    const int K = d0.K;
    for (int k = tid; k < K; k += ts) mine[k] = 0.0;

    const T* __restrict__ dec = reinterpret_cast<const T*>(a.dec);
    const int64_t rounds = (cnt + nteam - 1) / nteam;
    for (int64_t r = 0; r < rounds; ++r) {
        const int64_t e = lo + r * nteam + team;
        const bool live = e < hi;
        int ci = 0;
        if (live) {
            ci = a.tmpl_list[e];
            load_grid<T>(a, ci - a.first, buf, tid, ts);
        }
        __syncthreads();
        const cpx<T>* res = fft_team<T>(buf, tw, a.fft, tid, ts);
        if (live) {
            const InstDev d = a.inst[ci];
            const double wgt = o.seg_weight ? o.seg_weight[d.seg] : 1.0;
            for (int k = tid; k < K; k += ts) {
                int l = k - d.m0;
                if (l < 0) l += n;
                const T f = dec[l];
                const T xr = res[l].x * f, xi = res[l].y * f;
                mine[k] += wgt * ((double)xr * (double)xr + (double)xi * (double)xi);
            }
        }
        __syncthreads();
    }
    O* stat = reinterpret_cast<O*>(o.stat) + a.tmpl_stat_off[ct];
    for (int k = threadIdx.x; k < K; k += kBlock) {
        double s = 0.0;
        for (int t = 0; t < nteam; ++t) s += part[(size_t)t * kmax + k];
        stat[k] = (O)((double)stat[k] + s);
    }
    if (threadIdx.x == 0 && o.n_used) o.n_used[a.tmpl_id[ct]] += (int32_t)cnt;
}

template <typename T, typename O, int SUM>
__global__ __launch_bounds__(kBlock) void epilogue_kernel(EpilogueArgs a, EpilogueOut o)
{
    if (SUM)
        epilogue_sum_block<T, O>(a, o, blockIdx.x);
    else
        epilogue_spectra_block<T, O>(a, o, blockIdx.x);
}

template <typename T, typename O, int SUM>
__global__ __launch_bounds__(kBlock) void epilogue_multi_kernel(const EpilogueTable t, EpilogueOut o)
{
    const int c = class_of_block(t.block_off[SUM], t.ncls, blockIdx.x);
    const EpilogueArgs& a = t.a[c];  // read in place: a private copy would spill the radix list
    const int64_t lb = (int64_t)blockIdx.x - t.block_off[SUM][c];
    if (SUM)
        epilogue_sum_block<T, O>(a, o, lb);
    else
        epilogue_spectra_block<T, O>(a, o, lb);
}

// ------------------------------------------------------- direct baseline --
//
// The plain non-uniform DFT X_k = sum_j x_j exp(-2 pi i f_k dtau_j) on the
// GPU, with no spreading and no FFT: the baseline the NUFFT is measured
// against.  One wave per instance, lanes over samples (coalesced reads of a
// plain copy); per sample the phase of the first bin and the step between
// bins are reduced modulo one cycle in FP64, and the K bins follow by complex
// rotation in the class precision, 16 bins per pass as four interleaved
// rotation chains (steps of r^4) so that consecutive rotations do not wait
// on each other.  The lanes' partial sums are combined by a butterfly of
// lane exchanges.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T, bool CPLX>
__device__ __forceinline__ void direct_block(const SpreadArgs& a, const EpilogueArgs& e, const EpilogueOut& o,
                                             int mode, int out_fp64)
{
    constexpr int KB = 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= a.count) return;  // whole waves; no barriers below
    const InstDev d = a.inst[a.first + item];
    TauConsts tc;
    load_tau(tc, d, a.coef, 0.0);
    using E = typename std::conditional<CPLX, cpx<T>, T>::type;
    const E* __restrict__ xs = reinterpret_cast<const E*>(a.strain_lm) + d.strain_off;
    const double f_lo = d.fc - (double)d.m0 * d.df;
    for (int k0 = 0; k0 < d.K; k0 += KB) {
        T ar[KB], ai[KB];
#pragma unroll
        for (int q = 0; q < KB; ++q) ar[q] = ai[q] = T(0);
        const double f0 = f_lo + (double)k0 * d.df;
        for (int j = lane; j < d.L; j += kWave) {
            const double dt = dtau_of<false>(tc, j);
            const double p0 = __builtin_amdgcn_fract(f0 * dt);
            const double ps = __builtin_amdgcn_fract(d.df * dt);
            T s0, c0, s1, c1;
            if constexpr (sizeof(T) == 4) {
                sincospif((float)(2.0 * p0), &s0, &c0);
                sincospif((float)(2.0 * ps), &s1, &c1);
            } else {
                sincospi(2.0 * p0, &s0, &c0);
                sincospi(2.0 * ps, &s1, &c1);
            }
            // e_q = x exp(-i 2 pi (p0 + q ps)); r = exp(-i 2 pi ps) = (c1, -s1)
            T er[4], ei[4];
            if constexpr (CPLX) {
                const cpx<T> x = xs[j];
                er[0] = x.x * c0 + x.y * s0;
                ei[0] = x.y * c0 - x.x * s0;
            } else {
                const T x = xs[j];
                er[0] = x * c0;
                ei[0] = -x * s0;
            }
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                er[q] = er[q - 1] * c1 + ei[q - 1] * s1;
                ei[q] = ei[q - 1] * c1 - er[q - 1] * s1;
            }
            // r^4 = exp(-i 8 pi ps)
            const T c2 = c1 * c1 - s1 * s1, s2 = T(2) * c1 * s1;
            const T c4 = c2 * c2 - s2 * s2, s4 = T(2) * c2 * s2;
#pragma unroll
            for (int q = 0; q < KB; q += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    ar[q + u] += er[u];
                    ai[q + u] += ei[u];
                    const T nr = er[u] * c4 + ei[u] * s4;
                    ei[u] = ei[u] * c4 - er[u] * s4;
                    er[u] = nr;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KB; ++q) {
            ar[q] = wave_sum(ar[q]);
            ai[q] = wave_sum(ai[q]);
        }
        if (lane == 0) {
            for (int q = 0; q < KB && k0 + q < d.K; ++q) {
                const int k = k0 + q;
                const double pw = (double)ar[q] * (double)ar[q] + (double)ai[q] * (double)ai[q];
                if (mode == 0) {
                    if (out_fp64) {
                        if (o.spectra) reinterpret_cast<cpx<double>*>(o.spectra)[d.bin_off + k] = {(double)ar[q], (double)ai[q]};
                        if (o.power) reinterpret_cast<double*>(o.power)[d.bin_off + k] = pw;
                    } else {
                        if (o.spectra) reinterpret_cast<cpx<float>*>(o.spectra)[d.bin_off + k] = {(float)ar[q], (float)ai[q]};
                        if (o.power) reinterpret_cast<float*>(o.power)[d.bin_off + k] = (float)pw;
                    }
                } else {
                    const int64_t r = e.row_base + (int64_t)d.entry * e.kmax + k;
                    if (out_fp64) reinterpret_cast<double*>(o.rows)[r] = pw;
                    else reinterpret_cast<float*>(o.rows)[r] = (float)pw;
                }
            }
        }
    }
}

template <typename T, bool CPLX>
__global__ __launch_bounds__(kBlock) void direct_kernel(SpreadArgs a, EpilogueArgs e, EpilogueOut o, int mode,
                                                        int out_fp64)
{
    direct_block<T, CPLX>(a, e, o, mode, out_fp64);
}

// ------------------------------------------------------------ utilities --

// Lane-major copies: blockIdx.x picks the class segment, blockIdx.y and the
// thread stride over its entries in order, so the stores are contiguous.
template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void strain_lane_major_kernel(const SegDev* __restrict__ segs,
                                                                   const Ti* __restrict__ src, int cplx)
{
    const SegDev sd = segs[blockIdx.x];
    To* __restrict__ dst = reinterpret_cast<To*>(sd.dst);
    const uint32_t run = (uint32_t)sd.C * kWave;  // entries of 64 lane runs
    const uint32_t total = (uint32_t)sd.parts * run;
    for (uint32_t o = blockIdx.y * kBlock + threadIdx.x; o < total; o += kBlock * gridDim.y) {
        const uint32_t blk = o / run, rem = o - blk * run;
        const uint32_t srow = rem / kWave, lane = rem - srow * kWave;
        const int64_t j = (int64_t)(blk * kWave + lane) * sd.C + srow;
        const int64_t at = sd.dst_off + o;
        if (cplx) {
            To re = To(0), im = To(0);
            if (j < sd.L) {
                re = (To)src[2 * (sd.src_off + j)];
                im = (To)src[2 * (sd.src_off + j) + 1];
            }
            dst[2 * at] = re;
            dst[2 * at + 1] = im;
        } else {
            dst[at] = (j < sd.L) ? (To)src[sd.src_off + j] : To(0);
        }
    }
}

// Validity flags (one thread each) and zero outputs of invalid instances
// (one wave each, lanes along the bins).
template <typename O>
__global__ __launch_bounds__(kBlock) void fill_invalid_kernel(const int32_t* __restrict__ inv,
                                                              const int64_t* __restrict__ bin_off,
                                                              const int32_t* __restrict__ inst_K, int64_t n_inv,
                                                              cpx<O>* sp, O* pw, const uint8_t* __restrict__ mask,
                                                              uint8_t* valid, int64_t n_inst)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (valid && i < n_inst) valid[i] = mask[i];
    const int64_t q = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    if (q < n_inv) {
        const int32_t ii = inv[q];
        const int64_t o = bin_off[ii];
        const int K = inst_K[ii];
        for (int k = threadIdx.x & 63; k < K; k += kWave) {
            if (sp) sp[o + k] = cpx<O>{O(0), O(0)};
            if (pw) pw[o + k] = O(0);
        }
    }
}

template <typename T>
__global__ void finite_scan_kernel(const T* __restrict__ x, int64_t n, int32_t* flag)
{
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------- launches --

// Kernels whose dynamic LDS exceeds 64 KiB must opt in to the larger limit.
template <typename K>
static void allow_lds(K* kernel, size_t bytes)
{
    if (bytes > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t spread_lds_bytes(int fp64, int n, int pong)
{
    const size_t csize = fp64 ? 16 : 8;
    const size_t table = fp64 ? (size_t)phase_table_entries<double>() : (size_t)phase_table_entries<float>();
    return (table + (size_t)(pong ? 8 : 4) * n) * csize;
}

int phase_table_size(int fp64)
{
    return fp64 ? phase_table_entries<double>() : phase_table_entries<float>();
}

size_t epilogue_lds_bytes(int fp64, int n, int K_max, int sum_mode)
{
    const int nteam = kBlock / team_size_for(n);
    size_t b = ((size_t)nteam * 2 + 1) * n * (fp64 ? 16 : 8);
    if (sum_mode) b += (size_t)nteam * K_max * 8;
    return b;
}

hipError_t launch_strain_lane_major(const SegDev* segs, int32_t n_segs, int64_t max_entries, const void* strain,
                                    int strain_fp64, int strain_complex, int dst_fp64, hipStream_t st)
{
    if (n_segs <= 0) return hipSuccess;
    // about 16 entries per thread of the largest segment, at most 64 workgroups per segment
    int64_t gy = (max_entries + kBlock * 16 - 1) / (kBlock * 16);
    if (gy < 1) gy = 1;
    if (gy > 64) gy = 64;
    dim3 grid((unsigned)n_segs, (unsigned)gy), block(kBlock);
    if (strain_fp64 && dst_fp64)
        strain_lane_major_kernel<double, double><<<grid, block, 0, st>>>(segs, (const double*)strain, strain_complex);
    else if (strain_fp64)
        strain_lane_major_kernel<double, float><<<grid, block, 0, st>>>(segs, (const double*)strain, strain_complex);
    else if (dst_fp64)
        strain_lane_major_kernel<float, double><<<grid, block, 0, st>>>(segs, (const float*)strain, strain_complex);
    else
        strain_lane_major_kernel<float, float><<<grid, block, 0, st>>>(segs, (const float*)strain, strain_complex);
    return hipGetLastError();
}

hipError_t launch_direct(const SpreadArgs& a, const EpilogueArgs& e, const EpilogueOut& o, int mode, int fp64,
                         int out_fp64, hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.count + 3) / 4)), block(kBlock);
    if (fp64) {
        if (a.strain_complex) direct_kernel<double, true><<<grid, block, 0, st>>>(a, e, o, mode, out_fp64);
        else direct_kernel<double, false><<<grid, block, 0, st>>>(a, e, o, mode, out_fp64);
    } else {
        if (a.strain_complex) direct_kernel<float, true><<<grid, block, 0, st>>>(a, e, o, mode, out_fp64);
        else direct_kernel<float, false><<<grid, block, 0, st>>>(a, e, o, mode, out_fp64);
    }
    return hipGetLastError();
}

hipError_t launch_tau(const SpreadArgs& a, int fp64, hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    dim3 grid((unsigned)spread_blocks(a.count, a.parts)), block(kBlock);
    if (fp64)
        tau_kernel<double><<<grid, block, 0, st>>>(a);
    else
        tau_kernel<float><<<grid, block, 0, st>>>(a);
    return hipGetLastError();
}

template <typename T, int D, bool FUSED, bool CPLX, bool SNAP>
static void launch_spread_k(const SpreadArgs& a, const EpilogueOut& o, dim3 grid, size_t lds, hipStream_t st)
{
    allow_lds(spread_kernel<T, D, FUSED, CPLX, SNAP>, lds);
    spread_kernel<T, D, FUSED, CPLX, SNAP><<<grid, dim3(kBlock), lds, st>>>(a, o);
}

template <typename T, int D, bool FUSED, bool CPLX, bool SNAP>
static void launch_spread_k(const SpreadTable& m, const EpilogueOut& o, dim3 grid, size_t lds, hipStream_t st)
{
    allow_lds(spread_multi_kernel<T, D, FUSED, CPLX, SNAP>, lds);
    spread_multi_kernel<T, D, FUSED, CPLX, SNAP><<<grid, dim3(kBlock), lds, st>>>(m, o);
}

template <typename T, int D, bool CPLX>
static void launch_runs_k(const SpreadArgs& a, const EpilogueOut& o, dim3 grid, size_t lds, hipStream_t st)
{
    allow_lds(spread_runs_kernel<T, D, CPLX>, lds);
    spread_runs_kernel<T, D, CPLX><<<grid, dim3(kBlock), lds, st>>>(a, o);
}

template <typename T, int D, bool CPLX>
static void launch_runs_k(const SpreadTable& m, const EpilogueOut& o, dim3 grid, size_t lds, hipStream_t st)
{
    allow_lds(spread_runs_multi_kernel<T, D, CPLX>, lds);
    spread_runs_multi_kernel<T, D, CPLX><<<grid, dim3(kBlock), lds, st>>>(m, o);
}

template <typename T, int D, bool SNAP, typename A>
static void launch_spread_s(const A& a, const EpilogueOut& o, int fused, int cplx, dim3 grid, size_t lds,
                            hipStream_t st)
{
    if (fused) {
        if (cplx) launch_spread_k<T, D, true, true, SNAP>(a, o, grid, lds, st);
        else launch_spread_k<T, D, true, false, SNAP>(a, o, grid, lds, st);
    } else {
        if (cplx) launch_spread_k<T, D, false, true, SNAP>(a, o, grid, lds, st);
        else launch_spread_k<T, D, false, false, SNAP>(a, o, grid, lds, st);
    }
}

// cumulative snapshots need a third register set: FP32 classes of moderate degree only
template <typename T, int D>
constexpr bool snap_allowed() { return sizeof(T) == 4 && D <= 12; }

template <typename T, int D, typename A>
static hipError_t launch_spread_d(const A& a, const EpilogueOut& o, int fused, int cplx, int snap, int64_t blocks,
                                  size_t lds, hipStream_t st)
{
    dim3 grid((unsigned)blocks);
    constexpr bool snap_ok = snap_allowed<T, D>();
    if (fused == 2) {
        if (cplx) launch_runs_k<T, D, true>(a, o, grid, lds, st);
        else launch_runs_k<T, D, false>(a, o, grid, lds, st);
    } else if (snap_ok && snap)
        launch_spread_s<T, D, snap_ok>(a, o, fused, cplx, grid, lds, st);
    else
        launch_spread_s<T, D, false>(a, o, fused, cplx, grid, lds, st);
    return hipGetLastError();
}

template <typename T, typename A>
static hipError_t launch_spread_t(const A& a, const EpilogueOut& o, int deg, int fused, int cplx, int snap,
                                  int64_t blocks, size_t lds, hipStream_t st)
{
    switch (deg) {
#define NR_CASE(DD) \
    case DD: return launch_spread_d<T, DD>(a, o, fused, cplx, snap, blocks, lds, st);
        NR_CASE(2) NR_CASE(3) NR_CASE(4) NR_CASE(5) NR_CASE(6) NR_CASE(7) NR_CASE(8) NR_CASE(9)
        NR_CASE(10) NR_CASE(11) NR_CASE(12) NR_CASE(13) NR_CASE(14) NR_CASE(15) NR_CASE(16)
        NR_CASE(17) NR_CASE(18)
#undef NR_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spread(const SpreadArgs& a, int fp64, int deg, int fused, const EpilogueOut& out,
                         hipStream_t st)
{
    if (a.count <= 0) return hipSuccess;
    const int64_t blocks = spread_blocks(a.count, a.parts);
    const size_t lds = spread_lds_bytes(fp64, a.n, a.epi_fused && a.parts == 1);
    return fp64 ? launch_spread_t<double>(a, out, deg, fused, a.strain_complex, a.snap, blocks, lds, st)
                : launch_spread_t<float>(a, out, deg, fused, a.strain_complex, a.snap, blocks, lds, st);
}

hipError_t launch_spread_multi(const SpreadTable& t, int64_t blocks, int fp64, int deg, int fused, int cplx,
                               int snap, size_t lds, const EpilogueOut& out, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (t.ncls < 1 || t.ncls > kGroupMax) return hipErrorInvalidValue;
    return fp64 ? launch_spread_t<double>(t, out, deg, fused, cplx, snap, blocks, lds, st)
                : launch_spread_t<float>(t, out, deg, fused, cplx, snap, blocks, lds, st);
}

int64_t epilogue_blocks(const EpilogueArgs& a, int sum_mode)
{
    if (sum_mode) return a.tmpl_count;
    const int nteam = kBlock / team_size_for(a.fft.n);
    return (a.count + nteam - 1) / nteam;
}

template <typename T, typename O, int SUM>
static hipError_t launch_epi_k(const EpilogueArgs& a, const EpilogueOut& o, int64_t blocks, size_t lds,
                               hipStream_t st)
{
    allow_lds(epilogue_kernel<T, O, SUM>, lds);
    epilogue_kernel<T, O, SUM><<<dim3((unsigned)blocks), dim3(kBlock), lds, st>>>(a, o);
    return hipGetLastError();
}

template <typename T, typename O, int SUM>
static hipError_t launch_epi_multi_k(const EpilogueTable& t, const EpilogueOut& o, int64_t blocks, size_t lds,
                                     hipStream_t st)
{
    allow_lds(epilogue_multi_kernel<T, O, SUM>, lds);
    epilogue_multi_kernel<T, O, SUM><<<dim3((unsigned)blocks), dim3(kBlock), lds, st>>>(t, o);
    return hipGetLastError();
}

template <int SUM>
static hipError_t launch_epi(const EpilogueArgs& a, const EpilogueOut& o, int fp64, int out_fp64, hipStream_t st)
{
    const int64_t blocks = epilogue_blocks(a, SUM);
    if (blocks <= 0 || a.count <= 0) return hipSuccess;
    const size_t lds = epilogue_lds_bytes(fp64, a.fft.n, a.kmax, SUM);
    if (fp64) return launch_epi_k<double, double, SUM>(a, o, blocks, lds, st);
    if (out_fp64) return launch_epi_k<float, double, SUM>(a, o, blocks, lds, st);
    return launch_epi_k<float, float, SUM>(a, o, blocks, lds, st);
}

hipError_t launch_epilogue_spectra(const EpilogueArgs& a, const EpilogueOut& o, int fp64, int out_fp64,
                                   hipStream_t st)
{
    return launch_epi<0>(a, o, fp64, out_fp64, st);
}

hipError_t launch_epilogue_sum(const EpilogueArgs& a, const EpilogueOut& o, int fp64, int out_fp64, hipStream_t st)
{
    return launch_epi<1>(a, o, fp64, out_fp64, st);
}

hipError_t launch_rows_sum(const EpilogueArgs& a, const EpilogueOut& o, int out_fp64, hipStream_t st)
{
    if (a.tmpl_count <= 0) return hipSuccess;
    dim3 grid((unsigned)a.tmpl_count), block(kBlock);
    if (out_fp64)
        rows_sum_kernel<double><<<grid, block, 0, st>>>(a, o);
    else
        rows_sum_kernel<float><<<grid, block, 0, st>>>(a, o);
    return hipGetLastError();
}

hipError_t launch_rows_sum_multi(const EpilogueTable& t, int64_t blocks, EpilogueOut o, int out_fp64,
                                 hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (t.ncls < 1 || t.ncls > kGroupMax) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks), block(kBlock);
    if (out_fp64)
        rows_sum_multi_kernel<double><<<grid, block, 0, st>>>(t, o);
    else
        rows_sum_multi_kernel<float><<<grid, block, 0, st>>>(t, o);
    return hipGetLastError();
}

hipError_t launch_epilogue_multi(const EpilogueTable& t, int64_t blocks, int sum_mode, EpilogueOut o, int fp64,
                                 int out_fp64, size_t lds, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (t.ncls < 1 || t.ncls > kGroupMax) return hipErrorInvalidValue;
    if (sum_mode) {
        if (fp64) return launch_epi_multi_k<double, double, 1>(t, o, blocks, lds, st);
        if (out_fp64) return launch_epi_multi_k<float, double, 1>(t, o, blocks, lds, st);
        return launch_epi_multi_k<float, float, 1>(t, o, blocks, lds, st);
    }
    if (fp64) return launch_epi_multi_k<double, double, 0>(t, o, blocks, lds, st);
    if (out_fp64) return launch_epi_multi_k<float, double, 0>(t, o, blocks, lds, st);
    return launch_epi_multi_k<float, float, 0>(t, o, blocks, lds, st);
}

hipError_t launch_fill_invalid(const int32_t* inv_inst, const int64_t* bin_off,
                               const int32_t* inst_K, int64_t n_inv, void* spectra, void* power,
                               int out_fp64, const uint8_t* mask, uint8_t* valid, int64_t n_inst,
                               hipStream_t st)
{
    const int64_t b_flags = valid ? (n_inst + kBlock - 1) / kBlock : 0;
    const int64_t b_inv = (n_inv + kBlock / kWave - 1) / (kBlock / kWave);
    const int64_t blocks = b_flags > b_inv ? b_flags : b_inv;
    if (blocks <= 0) return hipSuccess;
    dim3 grid((unsigned)blocks), block(kBlock);
    if (out_fp64)
        fill_invalid_kernel<double><<<grid, block, 0, st>>>(inv_inst, bin_off, inst_K, n_inv,
                                                            (cpx<double>*)spectra, (double*)power,
                                                            mask, valid, n_inst);
    else
        fill_invalid_kernel<float><<<grid, block, 0, st>>>(inv_inst, bin_off, inst_K, n_inv,
                                                           (cpx<float>*)spectra, (float*)power,
                                                           mask, valid, n_inst);
    return hipGetLastError();
}

hipError_t launch_finite_scan(const void* strain, int64_t n, int fp64, int32_t* flag,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (fp64)
        finite_scan_kernel<double><<<(unsigned)blocks, 256, 0, st>>>((const double*)strain, n, flag);
    else
        finite_scan_kernel<float><<<(unsigned)blocks, 256, 0, st>>>((const float*)strain, n, flag);
    return hipGetLastError();
}

}  // namespace nr
