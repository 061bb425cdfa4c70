/*
 * nr_proposal.h -- C ABI of the learned proposal's ranking and refinement
 * steps (the statistic, the ranking of regions and the selection of the
 * regions that are re-searched on the finer chirp-mass grid).
 *
 * The statistic ranked and refined is the semicoherent sum of Sec. III.C
 * (Eq. (semicoherent_statistic) with unit weights): for a template with
 * summed power S_k over N segments, the standardised value
 *     z_k = (S_k * norm - N) / sqrt(N),   norm = 1 / (L sigma^2),
 * is zero-mean and unit-variance under white Gaussian noise of variance
 * sigma^2 (|X_k|^2 norm of one segment is exponentially distributed with
 * unit mean, the chi-square with two degrees of freedom of Sec. III.C scaled
 * by one half), and z = 0 when N = 0.
 *
 * The region features (nr_mlp_region_features) and the network (nr_mlp_*)
 * are declared in nr_mlp.h; this header adds the steps around them:
 *   nr_prop_max_z  -- the largest z of each group of templates (a coarse
 *                     template's own score, or a refined region's best fine
 *                     template), and where it is;
 *   nr_prop_topk   -- the k best-scoring regions of each row of scores.
 *
 * Conventions: all array arguments are device pointers owned by the caller;
 * work is enqueued on `stream` (hipStream_t; NULL: the null stream) and the
 * call returns after enqueueing; no exception crosses the ABI; status codes
 * are those of nufft_resample.h, with the message of the last failure on
 * this thread in nr_prop_last_error.  Results are bitwise reproducible.
 */
#ifndef NR_PROPOSAL_H
#define NR_PROPOSAL_H

#include <stdint.h>

#include "nufft_resample.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Largest z over each group of `group` consecutive templates and their K bins:
 *   stat[t * K + k]   summed |X|^2 of template t, bin k (float);
 *   n_used[t]         segments in that sum;
 *   zmax[g]           max over templates t in [g group, (g + 1) group) and
 *                     k < K of z_{t,k}, computed in FP64 and rounded to float;
 *   arg[g] (or NULL)  (t - g group) * K + k of that maximum, the lowest such
 *                     index on ties.
 * NaN sums take no part; a group without a number gives zmax NaN and arg -1.
 * n_groups >= 0 (0: no work), 1 <= group <= 64, 1 <= K <= 4096, norm > 0.
 * NR_ERR_INVALID_ARG for a NULL array (with n_groups > 0) or a size out of range.
 */
nr_status nr_prop_max_z(const float* stat, const int32_t* n_used, int64_t n_groups, int32_t group,
                        int32_t K, double norm, float* zmax, int32_t* arg, void* stream);

/*
 * The k largest of each row of scores, best first:
 *   scores[r * n + i]  float score of item i of row r;
 *   idx[r * k + j]     item of rank j in row r: scores decrease with j and
 *                      equal scores keep ascending item order; -0 counts as
 *                      +0, and NaN ranks below every number.
 * rows >= 0 (0: no work), 1 <= n <= 16384, 1 <= k <= n.
 * NR_ERR_INVALID_ARG for a NULL array (with rows > 0) or a size out of range.
 */
nr_status nr_prop_topk(const float* scores, int64_t rows, int32_t n, int32_t k, int32_t* idx,
                       void* stream);

/* Message of the last failure of a call of this header on this thread. */
const char* nr_prop_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NR_PROPOSAL_H */
