/*
 * nr_strobo.h -- C ABI of the stroboscopic-resampling baseline (Sec. III.B,
 * App. A): the comparison method the NUFFT replaces.  A segment sampled at
 * fs_o (O times the rate of the resampled series) is read at the sample
 * nearest to each point tau_m = m / fs_o of a uniform grid in the resampled
 * time of Eq. (new_t) (nearest-neighbour interpolation, a rectangular
 * kernel), for every m with tau_m <= tau(t_last) - tau(0).  The time of a
 * grid point inverts Eq. (new_t) with the segment start as reference:
 * t = (3 / (8 beta)) (1 - (1 - tau / a)^{8/5}), a = 3 / (5 beta), beta of
 * Eq. (beta) (Mc = 0: t = tau); the nearest sample is rint(t fs_o).
 *
 * The library produces the tau-uniform series folded modulo N (N = fs_o / df
 * for the bin spacing df the caller wants), so that an N-point FFT of the
 * fold gives sum_m y_m exp(-2 pi i f tau_m) exactly at f = q df; the caller
 * runs that FFT (the baseline uses the vendor FFT library through torch) and
 * divides by O for the scale of the NUFFT sum over the original samples.
 *
 * Conventions as in nufft_resample.h: host scalars, caller-owned device
 * arrays, work enqueued on the given stream, no exception crosses the ABI.
 */
#ifndef NR_STROBO_H
#define NR_STROBO_H

#include <stdint.h>

#include "nufft_resample.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size M of the tau grid of a segment of n_samples (>= 1) at fs_o (> 0) for
 * the template (mc_msun >= 0, f0 > 0); NR_ERR_INVALID_ARG if the segment
 * reaches coalescence. */
nr_status nr_strobo_points(double fs_o, int64_t n_samples, double mc_msun, double f0, int64_t* m_out);

/* For each of n_seg segments stored one after another (segment s at
 * x + s * n_samples samples), out[s * fold + r] = sum of y_m over
 * m = r, r + fold, ... < M (complex float, interleaved; fold >= 1), with y_m
 * the nearest sample of the segment (device, float; real when x_complex == 0,
 * else interleaved complex) to the grid point's time (0 outside the
 * segment).  Each segment is its own time reference; each slot adds its
 * terms in increasing m. */
nr_status nr_strobo_fold(const void* x, int32_t x_complex, int64_t n_samples, int32_t n_seg, double fs_o,
                         double mc_msun, double f0, int64_t fold, void* out, void* stream);

/* Message of the last failure on this thread. */
const char* nr_strobo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NR_STROBO_H */
