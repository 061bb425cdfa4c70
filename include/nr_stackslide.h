/*
 * nr_stackslide.h -- C ABI of the weighted stack-slide over stored spectra:
 * the semicoherent statistic of Sec. III.C, Eq. (semicoherent_statistic),
 * accumulated along 0PN frequency tracks through per-segment power spectra.
 *
 * Spectra.  Segment i (i = 0 .. n_seg-1) starts at t_i = i t_coh and was
 * resampled with each of n_beta templates of a bank, referenced at its own
 * start (Sec. III.A); power[k][i][j] = |X|^2 of segment i, beta template k,
 * frequency f_j = f_lo + j df (j < n_bins) -- the layout of
 * nufft_resample_execute's power output for a plan over all
 * (template, segment) pairs in template-major order.  Layout 1 stores the
 * same values as power[k][j][i].
 *
 * Tracks.  A semicoherent template theta = (Mc, t0) passes f_start at t0.
 * Segment i is on its track when t_i >= t0 and, with
 * u_i = 1 - (8/3) beta(f_start, Mc) (t_i - t0) (Eq. (f), Eq. (beta)),
 * u_i > 0, f_i = f_start u_i^{-3/8} <= f_max and round((f_i - f_lo)/df)
 * (halves up) is a bin; once a segment fails, all later ones do.  The
 * segment uses the bank template nearest beta(f_i, Mc) = beta(f_start, Mc)/u_i
 * (the lower index on a tie) and that bin.  Its weight (Eq. (weights), white
 * noise, no window) is proportional to f_i^{4/3}, normalised to a unit sum of
 * squares over the track.  With P = norm |X|^2 (Eq. (normalized_power)),
 *     n_sigma(theta) = sum_i w_i (P_i - mu) / sigma,
 * 0 for a track with no segment.  The track grid is n_mc chirp masses times
 * n_seg * t0_steps start times t0 = (i0 - s / t0_steps) t_coh, stored at
 * [c][i0 * t0_steps + s]; t_i - t0 is evaluated as (m + s / t0_steps) t_coh
 * with m = i - i0.
 *
 * Conventions: host arrays are read during the call only; device pointers
 * are caller-owned; work is enqueued on the plan's stream; no exception
 * crosses the ABI; status codes are those of nufft_resample.h.  The plan owns
 * its track tables (built on the device at creation).
 */
#ifndef NR_STACKSLIDE_H
#define NR_STACKSLIDE_H

#include <stdint.h>

#include "nufft_resample.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_seg;      /* segments (>= 1) */
    int32_t n_beta;     /* bank templates (>= 1) */
    int32_t n_bins;     /* bins per spectrum (>= 1) */
    int32_t layout;     /* 0: power[k][i][j]; 1: power[k][j][i] */
    double t_coh;       /* segment duration and spacing, s (> 0) */
    double f_lo, df;    /* frequency of bin 0 and bin spacing, Hz (df > 0) */
    double f_start;     /* track frequency at t0, Hz (> 0) */
    double f_max;       /* tracks end above this frequency, Hz (> f_start) */
    double norm;        /* P = norm |X|^2 (> 0); 2 / (L sigma_x^2) for white noise */
    double mu, sigma;   /* background mean and standard deviation of P (sigma > 0) */
} nr_ss_geometry;

typedef struct nr_ss_s* nr_ss_plan;

/* Tracks of n_mc chirp masses mc[] (host, Msun, > 0) by n_seg * t0_steps
 * start times (1 <= t0_steps <= 64), over a bank of ascending beta values
 * beta_bank[] (host, > 0).  stream: hipStream_t (NULL: the null stream).
 * Errors: NR_ERR_INVALID_ARG for any violated bound (nothing allocated),
 * NR_ERR_OUT_OF_MEMORY, NR_ERR_DEVICE. */
nr_status nr_ss_create(nr_ss_plan* out, const nr_ss_geometry* g, const double* beta_bank,
                       const double* mc, int32_t n_mc, int32_t t0_steps, void* stream);

/* n_sigma[n_mc][n_seg * t0_steps] (device float) from power (device float, the
 * geometry's layout, n_beta * n_seg * n_bins values); n_used (device int32,
 * same shape, or NULL) receives each track's segment count. */
nr_status nr_ss_execute(nr_ss_plan p, const float* power, float* n_sigma, int32_t* n_used);

/* The paper's partial sums for spectra that do not fit the device at once
 * (Sec. VI: a year of spectra is about 200 GB; the statistic is summed over
 * ranges of segments kept in memory one at a time): the contribution of the
 * segments seg_begin .. seg_begin + seg_count - 1 to every track, ADDED to
 * n_sigma (+=) and n_used (+=, or NULL).  power holds exactly those segments,
 * in the geometry's layout with seg_count in place of n_seg (segment i at
 * position i - seg_begin).  Each track's weights are normalised over the whole
 * track, so summing the ranges of a partition of [0, n_seg) in any order gives
 * nr_ss_execute's n_sigma up to float rounding and its n_used exactly (start
 * from zeroed outputs).  NR_ERR_INVALID_ARG unless 0 <= seg_begin and
 * 1 <= seg_count <= n_seg - seg_begin. */
nr_status nr_ss_execute_range(nr_ss_plan p, const float* power, int32_t seg_begin, int32_t seg_count,
                              float* n_sigma, int32_t* n_used);

/* The plan's track tables, copied to the host (synchronous): for chirp mass
 * c, start offset s and lag m (segment i0 + m of a track starting in segment
 * i0): k[(c * t0_steps + s) * n_seg + m], j[...], w2sum[...] (running sum of
 * the squared unnormalised weights f^{8/3} through lag m) for m < len[c * t0_steps + s];
 * any pointer may be NULL. */
nr_status nr_ss_tables(nr_ss_plan p, int32_t* k, int32_t* j, double* w2sum, int32_t* len);

/* power_kji[k][j][i] = power_kij[k][i][j] (device float arrays), on stream. */
nr_status nr_ss_transpose(const float* power_kij, int32_t n_beta, int32_t n_seg, int32_t n_bins,
                          float* power_kji, void* stream);

/* Message of the last failure on p (p == NULL: of the last failed create or
 * transpose on this thread). */
const char* nr_ss_last_error(nr_ss_plan p);

/* Free the plan (synchronises its stream).  NULL is a no-op. */
void nr_ss_destroy(nr_ss_plan p);

#ifdef __cplusplus
}
#endif

#endif /* NR_STACKSLIDE_H */
