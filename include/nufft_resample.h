/*
 * nufft_resample.h -- C ABI of the MI355X (gfx950) semicoherent NUFFT
 * resampling library.
 *
 * What it computes (the paper's coherent stage, Sec. III.A-C):
 *
 *   For every instance = (segment i, template m) the uniformly sampled strain
 *   x_j, j = 0..L-1, of the segment is placed at the Newtonian resampled times
 *     tau(t) = -(3/5) u(t)^{5/8} / beta,   u(t) = 1 - (8/3) beta (t - t0)
 *   (Eq. (new_t), Sec. III.B; beta(f0, Mc) of Eq. (beta), Sec. II), with
 *   sample times t_j = t_start + j / fs relative to the reference time t0,
 *   and the type-I transform
 *     X_k = sum_j x_j exp(-2 pi i f_k (tau(t_j) - tau(t_start))),
 *     f_k = f_lo + k df,  k = 0..K-1
 *   is evaluated onto the uniform frequency grid (Sec. III.B: one transform
 *   evaluates every f0 across the band).  The power is P_k = |X_k|^2 and the
 *   segment sum S[m][k] = sum over valid segments of w_i P_k (Sec. III.C,
 *   Eq. (semicoherent_statistic) with unnormalised power).
 *
 *   The DFT time origin of each segment is its first sample, so X carries
 *   no global phase; the power does not depend on that choice.
 *
 *   An instance is VALID iff u(t_last) > 0 and, when f_max > 0, the 0PN
 *   frequency f0 u(t_last)^{-3/8} of Eq. (f) at the last sample does not
 *   exceed f_max.  Invalid instances produce zeros and valid = 0 and are
 *   left out of the segment sum.
 *
 *   Mc = 0 selects the identity map (tau = t): a plain non-uniform ->
 *   uniform DFT of the segment.
 *
 * How (type-I NUFFT, Sec. III.B and App. A: interpolate with a kernel onto
 * a uniform grid, FFT, deconvolve): heterodyne by the band centre, spread
 * with the "exponential of semicircle" kernel onto an upsampled periodic
 * grid, FFT, divide by the kernel's Fourier transform.  The accuracy target
 * `tol` is the relative l2 error of an instance's K bins against the exact
 * sum.  FP64 arithmetic is used for tau and for the reduction of f * tau
 * modulo one cycle in every precision class.
 *
 * Conventions
 *   - Host pointers: segment / template / instance descriptions and option
 *     structs (read during the call only).
 *   - Device pointers: strain, outputs, weights.  The caller owns them (for
 *     example torch tensors); the library never frees them.
 *   - The plan owns its device workspace and frees it in destroy.
 *   - execute / semicoherent_sum are asynchronous on the plan's stream; they
 *     return after enqueueing.  Synchronise the stream before reading.
 *   - A plan must not be used from two host threads at once, and two calls
 *     on one plan must not overlap on different streams.
 *   - No C++ exception crosses this ABI; every failure is a status code with
 *     a message from nufft_resample_last_error.
 *   - All argument validation happens before any device work is enqueued.
 */
#ifndef NUFFT_RESAMPLE_H
#define NUFFT_RESAMPLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nr_plan_s* nr_plan;

typedef enum {
    NR_OK = 0,
    NR_ERR_INVALID_ARG = 1,      /* a size, index, value or pointer is out of its domain */
    NR_ERR_TOL_UNATTAINABLE = 2, /* strict mode: tolerance below what the precision reaches */
    NR_ERR_OUT_OF_MEMORY = 3,    /* workspace cap too small, or device allocation failed */
    NR_ERR_DEVICE = 4,           /* a HIP runtime call failed */
    NR_ERR_NONFINITE_INPUT = 5   /* check_finite: NaN or Inf in the strain */
} nr_status;

typedef enum {
    NR_FP32 = 0, /* spread / FFT / power in FP32 (tau and phase reduction in FP64) */
    NR_FP64 = 1, /* everything in FP64 */
    NR_AUTO = 2  /* per instance: FP32 when its tol >= 1e-6, else FP64 */
} nr_precision;

typedef enum {
    NR_METHOD_AUTO = 0,   /* per instance: NR_METHOD_CELLRUN when its time series spends
                             at least 24 samples (12 in plans of 4096 or more
                             instances) in each grid cell it visits or its
                             spreader workgroup needs at most 1/5 of a compute unit's
                             LDS; else NR_METHOD_FUSED */
    NR_METHOD_STAGED = 1, /* tau kernel writes a point stream; spreader reads it */
    NR_METHOD_FUSED = 2,  /* the spreader evaluates tau itself; no point stream; each
                             lane takes a fixed run of consecutive samples */
    NR_METHOD_CELLRUN = 3, /* fused; each lane takes the samples of one visit of the
                             time series to one grid cell (found by binary search on
                             the monotone cell index), so lanes never change cell
                             inside a run and flush together.
                             FP64 classes of the fused methods take instances whose
                             heterodyne phase spans fewer than 2^30 phase-table steps
                             (256 per cycle: about 4e6 cycles of the band centre over
                             the segment); longer FP64 spans, and instances whose tau
                             needs the log1p/expm1 form, use NR_METHOD_STAGED (FP32
                             classes take the phase's cosine and sine from the
                             hardware and have no such limit) */
    NR_METHOD_DIRECT = 4  /* baseline: the plain non-uniform DFT on the GPU, every
                             (sample, bin) term, no spreading and no FFT; never
                             chosen automatically; its segment sums need the plan's
                             power rows to fit the workspace */
} nr_method;

/* One segment of uniformly sampled strain (Sec. III: T_obs split into T_coh segments). */
typedef struct {
    int64_t sample_offset; /* index of the segment's first sample in the strain array */
    int64_t n_samples;     /* L >= 1 */
    double fs;             /* sample rate in Hz, > 0 */
    double t_start;        /* time of the first sample relative to t0, in s */
} nr_segment;

/* One resampling template (beta from Eq. (beta)) and its frequency grid. */
typedef struct {
    double mc_msun; /* chirp mass in solar masses, >= 0; 0 = identity map */
    double f0;      /* template frequency at t0 in Hz (> 0 when mc_msun > 0) */
    double f_lo;    /* frequency of bin 0 in Hz */
    double df;      /* bin spacing in Hz; <= 0 means 1/T_seg = fs/L of each segment */
    int32_t n_bins; /* K >= 1 */
    int32_t reserved;
    double f_max;   /* validity cut on the 0PN frequency at the last sample; <= 0: none */
} nr_template;

/* One explicit (segment, template) pair for ragged batches. */
typedef struct {
    int32_t segment;
    int32_t template_id;
    double tol; /* <= 0: the plan tolerance */
} nr_instance;

typedef struct {
    int32_t precision;          /* nr_precision */
    int32_t method;             /* nr_method */
    double sigma;               /* grid upsampling factor in [1.25, 4]; <= 0: 2.0 */
    int32_t strain_complex;     /* 0: real strain; 1: interleaved complex (re, im) */
    int32_t strict;             /* 1: unattainable tolerances are errors, not clamped: an FP32
                                   tolerance below 1e-6 without NR_AUTO, an FP64 tolerance
                                   below 1e-12, or one below 4x the error of the FP64
                                   heterodyne phase, about 2 pi (degree + 3) 2^-53 times the
                                   cycles of the band centre over the segment */
    int32_t check_finite;       /* 1: execute scans the strain and synchronises */
    int32_t parts;              /* waves per instance in the spreader: 1, 2, 4, 8 or 16
                                   (8 and 16 span 2 and 4 workgroups whose partial grids
                                   the epilogue adds); 0: automatic (more waves per
                                   instance when the plan is too small to fill the GPU) */
    int32_t profile;            /* 1: time every kernel launch with HIP events */
    int32_t use_graph;          /* 1: capture each call's launches in a HIP graph, keyed by
                                   its pointer arguments, and replay it on later calls with
                                   the same pointers (needs a non-null stream; ignored with
                                   profile or check_finite) */
    int64_t strain_length;      /* samples in the strain array; 0: not checked */
    int64_t max_workspace_bytes;/* device workspace cap; 0: 8 GiB */
    void* stream;               /* hipStream_t of every enqueue; NULL: the null stream */
    const char* tune_cache;     /* autotuner cache file read before and written after tuning;
                                   NULL: keep results in memory only */
    int32_t tune;               /* 1: at plan creation, time the candidate spreader
                                   configurations (parts, flush period, fused or staged) of
                                   every shape (precision, kernel width, grid size, samples)
                                   on a small synthetic batch and use the fastest */
    int32_t flush_period;       /* steps between collective flushes of the spreader (1..64,
                                   power of two); 0: chosen from the sample density */
    int32_t moment_mode;        /* spreader moments: 0 automatic, 1 restarted per grid cell,
                                   2 cumulative with snapshots (FP32 classes, degree <= 12) */
    int32_t epilogue;           /* 2: classes of at most four waves per instance run the FFT,
                                   deconvolution and power inside the spreader's workgroup (the
                                   grid never leaves LDS; App. A's interpolate-FFT-deconvolve as
                                   one kernel), unless the FFT's second buffer would cost the
                                   spreader workgroups per compute unit; 1: always a separate
                                   epilogue kernel reading the grids from memory; 0: as 2 in
                                   plans of at least 4096 waves, counted at the default waves
                                   per instance (one up to 16,384 samples, two up to 32,768,
                                   four beyond), else as 1 */
} nr_options;

typedef struct {
    int64_t n_inst;          /* instances in the plan */
    int64_t n_valid;         /* valid instances */
    int64_t total_bins;      /* sum of K over instances: length of spectra / power */
    int64_t stat_bins;       /* sum of K over templates: length of the segment-sum output */
    int64_t valid_points;    /* sum of L over valid instances */
    int64_t workspace_bytes; /* device bytes owned by the plan */
    int32_t n_classes;       /* kernel classes (precision, kernel width, grid size, parts) */
    int32_t out_fp64;        /* 1: outputs are double / complex double; 0: float */
    int32_t method;          /* nr_method of the first class (classes may differ when tuned) */
    int32_t n_chunks;        /* spread launches per call: the chunks of every class, or,
                                when every class fits one chunk and all grids fit the
                                workspace together, the groups of classes that share a
                                kernel and are launched together */
} nr_plan_info;

typedef struct {
    int32_t fp64;       /* 1: FP64 class */
    int32_t w;          /* kernel width in grid cells */
    int32_t n;          /* upsampled grid size (2^a 3^b 5^c) */
    int32_t degree;     /* Chebyshev degree of the per-cell kernel polynomials */
    int32_t parts;      /* waves per instance in the spreader */
    int32_t n_radix;    /* FFT passes */
    int32_t radix[8];   /* FFT radices, first pass first */
    double beta_es;     /* ES shape parameter */
    int64_t n_inst;     /* valid instances in the class */
    int64_t n_points;   /* sum of L over them */
    int32_t method;          /* NR_METHOD_STAGED, NR_METHOD_FUSED or NR_METHOD_CELLRUN */
    int32_t flush_period;    /* spreader steps between collective flushes */
    int32_t snap;            /* 1: cumulative spreader moments with snapshots; 0: per cell */
    int32_t epi_fused;       /* 1: the spreader runs the FFT / deconvolution / power */
    int64_t series_terms;    /* sum over instances of L x (degree of the tau series) */
    int64_t fallback_points; /* samples of instances using the log1p/expm1 form of tau */
} nr_class_info;

/* Kernel time per stage, accumulated over launches since the last read. */
typedef enum {
    NR_STAGE_LAYOUT = 0,   /* lane-major strain copy */
    NR_STAGE_TAU = 1,      /* point stream (staged method) */
    NR_STAGE_SPREAD = 2,   /* spreading (fused method: tau + spreading) */
    NR_STAGE_EPILOGUE = 3, /* FFT, deconvolution, power / segment sum, invalid fill */
    NR_N_STAGES = 4
} nr_stage;

typedef struct {
    double ms[NR_N_STAGES];       /* summed kernel durations in milliseconds */
    int64_t launches[NR_N_STAGES];/* kernel launches timed */
} nr_stage_times;

/* Default options: NR_FP32, NR_METHOD_AUTO, sigma 2, real strain, non-strict. */
void nufft_resample_default_options(nr_options* opt);

/*
 * Build a plan (host work plus device allocations; no kernel runs).
 *   segs[n_segs], tmpls[n_tmpls]: host arrays.
 *   inst: NULL for the full product, instance index = template * n_segs + segment
 *         (template-major); else an explicit list of n_inst pairs.
 *   tol:  target relative l2 error per instance, in (0, 0.1].
 * On success *out holds the plan; on failure *out is NULL (the message is
 * then available from nufft_resample_last_error(NULL)).
 */
nr_status nufft_resample_plan(nr_plan* out, const nr_segment* segs, int32_t n_segs,
                              const nr_template* tmpls, int32_t n_tmpls,
                              const nr_instance* inst, int64_t n_inst, double tol,
                              const nr_options* opt);

/*
 * Spectra of every instance.
 *   strain:  device, float (NR_FP32 plans) or double (NR_FP64 / NR_AUTO),
 *            real or interleaved complex per the options.
 *   spectra: device complex [total_bins] (interleaved re, im) or NULL.
 *   power:   device real [total_bins] or NULL.
 *   valid:   device uint8 [n_inst] or NULL.
 *   Instance i's K bins start at bin offset i of nufft_resample_bin_offsets.
 *   Output element type: float for NR_FP32 plans, double otherwise.
 */
nr_status nufft_resample_execute(nr_plan p, const void* strain, void* spectra, void* power,
                                 uint8_t* valid);

/*
 * Segment sum, accumulated into the caller's buffers:
 *   stat[stat_off[m] + k] += sum over the plan's valid instances of template
 *   m, in instance order, of seg_weight[segment] * |X_k|^2;
 *   n_used[m] += number of those instances.
 *   stat: device, [stat_bins], float or double like the outputs.
 *   seg_weight: device double [n_segs] or NULL (unit weights).
 *   n_used: device int32 [n_tmpls] or NULL.
 * The per-template order is fixed, so results are bitwise reproducible.
 * Every instance of one template must fall in one kernel class.
 */
nr_status nufft_resample_semicoherent_sum(nr_plan p, const void* strain,
                                          const double* seg_weight, void* stat,
                                          int32_t* n_used);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * segment sum of nufft_resample_semicoherent_sum for the plan that
 * nufft_resample_plan would build from the same arguments, planned, run and
 * released inside this one call without any device allocation.  Every
 * device buffer of that plan (instance tables, the lane-major strain copy,
 * grids, power rows) is carved from one static scratch array of
 * NR_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; no hipMalloc, hipFree, stream, event or graph is
 * created.
 *   segs ... opt: as for nufft_resample_plan, except that opt->profile,
 *       opt->use_graph and opt->tune must be 0 (NR_ERR_INVALID_ARG), side
 *       streams are not used, and grids, point stream and power rows are
 *       budgeted within half the scratch (opt->max_workspace_bytes may only
 *       lower that); opt may be NULL (defaults, null stream).
 *   strain, seg_weight, stat, n_used: as for nufft_resample_semicoherent_sum
 *       (device pointers; stat and n_used are accumulated into).
 * The call synchronises opt->stream before planning (an earlier call on that
 * stream may still read the scratch) and returns after the sum has
 * completed.  Every call on one GPU shares that GPU's scratch, which keeps
 * the last call's contents: calls that overlap on one GPU (from other host
 * threads, or on other streams) race and must be serialised by the caller.
 * NR_ERR_OUT_OF_MEMORY when the plan needs more than the scratch; other
 * failures as for plan / semicoherent_sum, with the message in
 * nufft_resample_last_error(NULL).
 */
#define NR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
nr_status nufft_resample_semicoherent_sum_static(const nr_segment* segs, int32_t n_segs,
                                                 const nr_template* tmpls, int32_t n_tmpls,
                                                 const nr_instance* inst, int64_t n_inst, double tol,
                                                 const nr_options* opt, const void* strain,
                                                 const double* seg_weight, void* stat, int32_t* n_used);

/*
 * Per-stage kernel times of a plan created with profile = 1: waits for the
 * recorded launches to finish (synchronising), returns their summed
 * durations and starts a new accumulation.  All zeros when profiling is off.
 */
nr_status nufft_resample_stage_times(nr_plan p, nr_stage_times* out);

/* Plan summary. */
nr_status nufft_resample_query(nr_plan p, nr_plan_info* info);

/* Description of kernel class c, 0 <= c < n_classes. */
nr_status nufft_resample_query_class(nr_plan p, int32_t c, nr_class_info* info);

/* Host array [n_inst + 1] of bin offsets into spectra / power. */
nr_status nufft_resample_bin_offsets(nr_plan p, int64_t* offsets);

/* Host array [n_tmpls + 1] of bin offsets into the segment-sum output. */
nr_status nufft_resample_stat_offsets(nr_plan p, int64_t* offsets);

/* Host array [n_inst] of validity flags (the same rule as execute's output). */
nr_status nufft_resample_valid_mask(nr_plan p, uint8_t* valid);

/*
 * Kernel parameters a plan picks for one instance with this tolerance,
 * upsampling factor, precision and bin count (host only; no device needed):
 * fp64, w, beta_es, n, degree, radix plan.  parts / n_inst / n_points are
 * left 1 / 0 / 0.  NR_ERR_INVALID_ARG for out-of-domain arguments.
 */
nr_status nufft_resample_kernel_params(double tol, double sigma, int32_t precision, int32_t n_bins,
                                       nr_class_info* info);

/*
 * Fourier transform of the ES spreading kernel of width w (grid cells),
 *   psi_hat(xi) = integral over |x| <= w/2 of exp(beta_es (sqrt(1 - (2x/w)^2) - 1)) cos(xi x) dx,
 * by Gauss-Legendre quadrature (the deconvolution factors are 1/psi_hat(2 pi m / n)).
 * Host only.  NaN for w outside [2, 16] or beta_es <= 0.
 */
double nufft_resample_kernel_ft(int32_t w, double beta_es, double xi);

/* beta(f0, Mc) of Eq. (beta), Sec. II, in s^-1, as the plan computes it
 * (GM_sun/c^3 from the IAU 2015 nominal GM_sun).  Host only; NaN for Mc < 0 or f0 <= 0. */
double nufft_resample_chirp_beta(double mc_msun, double f0);

/* Message of the last failure on p (p == NULL: of the last failed plan
 * creation on this thread).  Valid until the next call on p. */
const char* nufft_resample_last_error(nr_plan p);

/* Free the plan and its workspace (synchronises its stream).  NULL is a no-op. */
void nufft_resample_destroy(nr_plan p);

#ifdef __cplusplus
}
#endif

#endif /* NUFFT_RESAMPLE_H */
