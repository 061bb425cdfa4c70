/*
 * Oracle for semicoherent NUFFT resampling -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU evaluation of what the GPU path
 * approximates.  Only the test-suite, the smoke check and the CPU baseline
 * of the benchmark may load this library; the product path never does.
 *
 * Every quantity is the plain definition written out, in higher than double
 * precision:
 *   - beta(f0, Mc)                        Eq. (beta), Sec. II
 *   - u(t) = 1 - (8/3) beta (t - t0)      Eq. (f) / Eq. (new_t), Sec. III.A-B
 *   - tau(t) = -(3/5) u^{5/8} / beta      Eq. (new_t), Sec. III.B
 *   - dtau_j = tau(t_j) - tau(t_s)        (time origin of each segment's DFT
 *                                          at its first sample)
 *     evaluated as a direct difference in __float128 (113-bit significand),
 *     so the cancellation between two values of size 3/(5 beta) is harmless.
 *   - X_k = sum_j x_j exp(-2 pi i f_k dtau_j), f_k = f_lo + k df
 *     (the type-I transform onto the uniform 1/T_coh grid, Sec. III.B),
 *     one term at a time, phase reduced modulo one cycle and summed in
 *     long double.
 *   - P_k = |X_k|^2 and the segment sum S[m][k] = sum_valid w_i P (Sec. III.C,
 *     Eq. (semicoherent_statistic) with equal weights, no normalisation).
 *   - validity of (segment, template): u(t_last) > 0 and
 *     f_0PN(t_last) = f0 u(t_last)^{-3/8} <= f_max (Eq. (f)); f_max <= 0
 *     disables the frequency cut.
 *
 * Mc = 0 denotes the identity map (beta = 0, dtau_j = j/fs).
 * df <= 0 denotes the natural bin spacing 1/T_seg with T_seg = L/fs.
 * Sample times are t_j = t_s + j/fs (no half-sample offset).
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 q_t;
typedef long double ld_t;

/* GM_sun / c^3 from the IAU 2015 nominal GM_sun and the exact speed of light. */
static q_t t_sun_q(void)
{
    const q_t gm = 1.3271244e20Q;
    const q_t c = 299792458.0Q;
    return gm / (c * c * c);
}

/* Eq. (beta): beta = (96/5) pi^{8/3} (G Mc / c^3)^{5/3} f0^{8/3}. */
static q_t beta_q(double mc_msun, double f0)
{
    if (mc_msun == 0.0) return 0.0Q;
    const q_t e83 = 8.0Q / 3.0Q, e53 = 5.0Q / 3.0Q;
    return (96.0Q / 5.0Q) * powq(M_PIq, e83) * powq(t_sun_q() * (q_t)mc_msun, e53) *
           powq((q_t)f0, e83);
}

double nro_beta(double mc_msun, double f0) { return (double)beta_q(mc_msun, f0); }

double nro_t_sun(void) { return (double)t_sun_q(); }

int nro_num_threads(void) { return omp_get_max_threads(); }

/* tau(t) of Eq. (new_t) (t relative to t0). */
static q_t tau_q(q_t beta, q_t t)
{
    q_t u = 1.0Q - (8.0Q / 3.0Q) * beta * t;
    return -(3.0Q / 5.0Q) * powq(u, 5.0Q / 8.0Q) / beta;
}

static q_t dtau_q(q_t beta, double t_start, double fs, int64_t j)
{
    q_t dt = (q_t)j / (q_t)fs;
    if (beta == 0.0Q) return dt;
    return tau_q(beta, (q_t)t_start + dt) - tau_q(beta, (q_t)t_start);
}

/* dtau_j for j = 0..L-1, rounded to double. */
void nro_dtau(double mc_msun, double f0, double t_start, double fs, int64_t L, double* out)
{
    q_t b = beta_q(mc_msun, f0);
    for (int64_t j = 0; j < L; ++j) out[j] = (double)dtau_q(b, t_start, fs, j);
}

/* Validity rule: u(t_last) > 0 and f0 u(t_last)^{-3/8} <= f_max (if f_max > 0). */
static int valid_q(q_t beta, double f0, double f_max, double t_start, double fs, int64_t L)
{
    if (L <= 0) return 0;
    if (beta == 0.0Q) return 1;
    q_t t_last = (q_t)t_start + (q_t)(L - 1) / (q_t)fs;
    q_t u = 1.0Q - (8.0Q / 3.0Q) * beta * t_last;
    if (!(u > 0.0Q)) return 0;
    if (f_max > 0.0) {
        q_t f = (q_t)f0 * powq(u, -3.0Q / 8.0Q);
        if (f > (q_t)f_max) return 0;
    }
    return 1;
}

int nro_valid(double mc_msun, double f0, double f_max, double t_start, double fs, int64_t L)
{
    return valid_q(beta_q(mc_msun, f0), f0, f_max, t_start, fs, L);
}

/*
 * Direct spectrum of one instance at the bins kidx[0..nk-1] (kidx == NULL:
 * bins 0..nk-1).  strain points at the segment's first sample; complex
 * strain is interleaved (re, im).  Returns the validity flag; an invalid
 * instance yields zeros.
 */
int nro_spectrum(const double* strain, int strain_complex, int64_t L, double fs,
                 double t_start, double mc_msun, double f0, double f_lo, double df,
                 double f_max, int32_t nk, const int32_t* kidx, double* out_re,
                 double* out_im)
{
    q_t b = beta_q(mc_msun, f0);
    int ok = valid_q(b, f0, f_max, t_start, fs, L);
    if (!ok) {
        for (int32_t i = 0; i < nk; ++i) out_re[i] = out_im[i] = 0.0;
        return 0;
    }
    if (df <= 0.0) df = fs / (double)L;
    ld_t* dtau = (ld_t*)malloc(sizeof(ld_t) * (size_t)L);
    for (int64_t j = 0; j < L; ++j) dtau[j] = (ld_t)dtau_q(b, t_start, fs, j);
    const ld_t two_pi = 2.0L * 3.14159265358979323846264338327950288L;
    for (int32_t i = 0; i < nk; ++i) {
        int32_t k = kidx ? kidx[i] : i;
        ld_t fk = (ld_t)f_lo + (ld_t)k * (ld_t)df;
        ld_t sr = 0.0L, si = 0.0L;
        for (int64_t j = 0; j < L; ++j) {
            ld_t ph = fk * dtau[j];
            ph -= floorl(ph);
            ld_t s, c;
            sincosl(two_pi * ph, &s, &c);
            /* x_j * exp(-i 2 pi ph) = x_j * (c - i s) */
            ld_t xr = strain_complex ? (ld_t)strain[2 * j] : (ld_t)strain[j];
            ld_t xi = strain_complex ? (ld_t)strain[2 * j + 1] : 0.0L;
            sr += xr * c + xi * s;
            si += xi * c - xr * s;
        }
        out_re[i] = (double)sr;
        out_im[i] = (double)si;
    }
    free(dtau);
    return 1;
}

/*
 * Batch of instances (inst_seg[i], inst_tmpl[i]); spectra written at
 * out_off[i] (complex split into re/im arrays).  OpenMP over instances.
 */
void nro_spectra(const double* strain, int strain_complex, const int64_t* seg_off,
                 const int64_t* seg_len, const double* seg_fs, const double* seg_t,
                 const double* mc, const double* f0, const double* f_lo, const double* df,
                 const int32_t* n_bins, const double* f_max, int64_t n_inst,
                 const int32_t* inst_seg, const int32_t* inst_tmpl, const int64_t* out_off,
                 double* out_re, double* out_im, uint8_t* valid)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_inst; ++i) {
        int32_t s = inst_seg[i], m = inst_tmpl[i];
        const double* x = strain + (strain_complex ? 2 : 1) * seg_off[s];
        int ok = nro_spectrum(x, strain_complex, seg_len[s], seg_fs[s], seg_t[s], mc[m], f0[m],
                              f_lo[m], df[m], f_max[m], n_bins[m], NULL, out_re + out_off[i],
                              out_im + out_off[i]);
        if (valid) valid[i] = (uint8_t)ok;
    }
}

/*
 * Segment sum for every template over all segments:
 *   stat[m][k] = sum_{s valid} w_s |X_{s,m,k}|^2 ,  n_used[m] = #valid s.
 * Segments are added in index order, in long double.  Bins of template m
 * start at stat_off[m].  seg_w == NULL means unit weights.
 */
void nro_semicoherent(const double* strain, int strain_complex, int32_t n_seg,
                      const int64_t* seg_off, const int64_t* seg_len, const double* seg_fs,
                      const double* seg_t, int32_t n_tmpl, const double* mc, const double* f0,
                      const double* f_lo, const double* df, const int32_t* n_bins,
                      const double* f_max, const double* seg_w, const int64_t* stat_off,
                      double* stat, int32_t* n_used)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t m = 0; m < n_tmpl; ++m) {
        int32_t K = n_bins[m];
        ld_t* acc = (ld_t*)calloc((size_t)K, sizeof(ld_t));
        double* re = (double*)malloc(sizeof(double) * (size_t)K);
        double* im = (double*)malloc(sizeof(double) * (size_t)K);
        int32_t used = 0;
        for (int32_t s = 0; s < n_seg; ++s) {
            const double* x = strain + (strain_complex ? 2 : 1) * seg_off[s];
            int ok = nro_spectrum(x, strain_complex, seg_len[s], seg_fs[s], seg_t[s], mc[m],
                                  f0[m], f_lo[m], df[m], f_max[m], K, NULL, re, im);
            if (!ok) continue;
            ld_t w = seg_w ? (ld_t)seg_w[s] : 1.0L;
            for (int32_t k = 0; k < K; ++k)
                acc[k] += w * ((ld_t)re[k] * re[k] + (ld_t)im[k] * im[k]);
            ++used;
        }
        for (int32_t k = 0; k < K; ++k) stat[stat_off[m] + k] = (double)acc[k];
        n_used[m] = used;
        free(acc);
        free(re);
        free(im);
    }
}
