// Internal definitions shared by the host plan code and the gfx950 kernels.
#pragma once

#include <cstdint>
#include <string>

#include <hip/hip_runtime.h>

#include "../../include/nufft_resample.h"

namespace nr {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlock = 256;      // four waves per workgroup
constexpr int kMaxRadix = 8;     // FFT passes
constexpr int kMaxDeg = 18;      // highest Chebyshev degree of the per-cell kernel polynomials
constexpr int kMaxHorner = 28;   // highest degree of the tau series before the log1p/expm1 form

// Cell-run spreader: a wave deals one run (cell) per lane and round to all
// lanes but the last, whose search of the next run's start ends the others.
constexpr int kRunsPerRound = kWave - 1;

// Per valid instance of a kernel class.  Lane-major point order: the
// instance's L samples are cut into V = 64 * parts contiguous runs of C
// samples; run v holds samples v*C .. v*C+C-1, and sample (v, s) lives at
// entry (v / 64) * (C * 64) + s * 64 + (v % 64) of the instance's point
// stream and of its segment's lane-major strain copy.  Lane l of the wave
// for part p therefore walks run p*64+l in sample order while every load
// of the wave is one contiguous 64-entry row.
struct InstDev {
    double a;           // tau scale (3/(5 beta)) u_s^{5/8}
    double c;           // series variable per sample, (8/3) beta / (u_s fs); identity: 1/fs
    double df;          // frequency period of the upsampled grid (bin spacing)
    double fc;          // heterodyne frequency: f_lo + floor(K/2) df
    int64_t strain_off; // first entry of the segment's lane-major strain copy
    int64_t bin_off;    // first output bin of the instance
    int64_t pt_off;     // first entry of the instance in the class point-stream layout
    int32_t L;          // samples
    int32_t C;          // samples per lane run
    int32_t K;          // output bins
    int32_t m0;         // floor(K/2): bin k holds mode m = k - m0
    int32_t inst;       // plan instance index
    int32_t seg;        // segment index
    int32_t ndeg;       // tau: 0 identity; > 0 Horner degree in the sample index; < 0 log1p/expm1
    int32_t coef_off;   // first Horner coefficient of this instance
    int32_t entry;      // position in the class's template-major instance list
};

// One segment of a class: where its samples are and where its lane-major copy goes.
struct SegDev {
    void* dst;          // the class's lane-major strain buffer
    int64_t src_off;    // first sample in the caller's strain
    int64_t dst_off;    // first entry of the lane-major copy
    int32_t L;
    int32_t C;
    int32_t parts;      // waves per instance of the class
    int32_t pad_;
};


struct FftPlanDev {
    int32_t n;
    int32_t nr;              // number of passes
    int32_t radix[kMaxRadix];
};
// Arguments of the tau and spreading kernels for one chunk of one class.
struct SpreadArgs {
    const InstDev* inst;     // class instances
    const double* coef;      // Horner coefficients
    const void* taps;        // [w][deg+1] Chebyshev coefficients of the per-cell kernel pieces
    const void* strain_lm;   // lane-major strain copy of the class (real or complex)
    const void* phase_table; // exp(2 pi i k / N), k < N (N = phase_table_size)
    void* points;            // staged point stream (chunk-relative)
    void* grid;              // [chunk instances][slots][n] complex
    int64_t first;           // first class instance of the chunk
    int64_t count;           // instances in the chunk
    int64_t pt_base;         // pt_off of the first instance of the chunk
    int32_t n;               // grid size
    int32_t w;               // kernel width
    int32_t parts;           // waves per instance (1, 2, 4, 8 or 16)
    int32_t flush_period;    // steps between collective flushes (power of two)
    int32_t strain_complex;
    int32_t snap;            // 1: cumulative moments with snapshots; 0: per-cell moments
    // fused epilogue (epi_fused = 1): the spreader itself runs the FFT of each
    // instance's grid in LDS, deconvolves and writes the outputs of the call
    // (EpilogueOut::mode); the grid never leaves LDS
    int32_t epi_fused;
    int32_t kmax;            // largest K of the class (power-row stride)
    int64_t row_base;        // first element of the class's power rows
    const void* dec;         // [n] real deconvolution factors indexed by mode mod n
    const void* twiddle;     // [n] complex exp(-2 pi i t / n)
    FftPlanDev fft;
    // single-class launches: logical workgroup of each hardware workgroup
    // (NULL: the identity)
    const int32_t* block_order;
};

// Workgroups of one launch of a class chunk, and grid slots per instance:
// up to four waves of an instance share a workgroup; an instance with more
// waves spans parts / 4 workgroups, each writing its own partial grid.
__host__ __device__ inline int grid_slots(int parts) { return parts > 4 ? parts / 4 : 1; }
__host__ __device__ inline int64_t spread_blocks(int64_t count, int parts)
{
    return parts > 4 ? count * (parts / 4) : (count * parts + 3) / 4;
}

struct EpilogueArgs {
    const InstDev* inst;
    const void* grid;        // [chunk instances][slots][n] complex (partial grids are summed)
    const void* dec;         // [n] real deconvolution factors indexed by mode mod n
    const void* twiddle;     // [n] complex exp(-2 pi i t / n)
    FftPlanDev fft;
    int64_t first;
    int64_t count;
    // segment-sum mode
    const int32_t* tmpl_list;      // class instances of each class template, ascending
    const int64_t* tmpl_list_off;  // [n class templates + 1]
    const int64_t* tmpl_stat_off;  // stat offset of each class template
    const int32_t* tmpl_id;        // plan template id of each class template
    int32_t tmpl_first;            // class templates handled by this launch
    int32_t tmpl_count;
    int32_t slots;                 // partial grids per instance
    int32_t kmax;                  // largest K of the class (LDS sizing of the segment sum)
    // two-pass segment sum: power rows of the class, one per list entry
    int64_t row_base;              // first element of the class's rows (row e at row_base + e kmax)
    const int32_t* entry_seg;      // segment of each list entry
};

// Per-call pointers of the epilogue (the same for every class of a plan).
struct EpilogueOut {
    void* spectra;
    void* power;
    const double* seg_weight;
    void* stat;
    int32_t* n_used;
    void* rows;              // power rows of the two-pass segment sum (first pass output)
    int32_t mode;            // spreaders of fused classes: 0 write the grid (a separate epilogue
                             // follows), 1 power rows, 2 spectra and/or power at the bin offsets
    int32_t out_fp64;        // outputs and rows are double (else float)
};

// Launch wrappers (defined in nr_kernels.hip).
// max_entries: the largest parts * C * 64 of the segments (sizes the grid).
hipError_t launch_strain_lane_major(const SegDev* segs, int32_t n_segs, int64_t max_entries, const void* strain,
                                    int strain_fp64, int strain_complex, int dst_fp64, hipStream_t st);
// One launch over up to kGroupMax classes of the same kernel instantiation:
// their arguments travel in the kernel arguments (so that the kernel knows
// every pointer in them addresses global memory), block_off[c] is the first
// workgroup of class c.
constexpr int kGroupMax = 8;
struct SpreadTable {
    SpreadArgs a[kGroupMax];
    int64_t block_off[kGroupMax];
    int32_t ncls;
};
hipError_t launch_spread_multi(const SpreadTable& t, int64_t blocks, int fp64, int deg, int fused, int cplx,
                               int snap, size_t lds, const EpilogueOut& out, hipStream_t st);
// The same for the epilogue: block_off[m][c] is the first workgroup of class
// c in mode m (0 spectra or power rows, 1 segment sum or row sums).
struct EpilogueTable {
    EpilogueArgs a[kGroupMax];
    int64_t block_off[2][kGroupMax];
    int32_t ncls;
};
hipError_t launch_epilogue_multi(const EpilogueTable& t, int64_t blocks, int sum_mode, EpilogueOut out, int fp64,
                                 int out_fp64, size_t lds, hipStream_t st);
int64_t epilogue_blocks(const EpilogueArgs& a, int sum_mode);
hipError_t launch_tau(const SpreadArgs& a, int fp64, hipStream_t st);
// The direct non-uniform DFT baseline: mode 0 writes spectra/power at the
// instances' bin offsets, mode 1 power rows for the two-pass segment sum.
hipError_t launch_direct(const SpreadArgs& a, const EpilogueArgs& e, const EpilogueOut& o, int mode, int fp64,
                         int out_fp64, hipStream_t st);
// fused: 0 staged (reads the point stream), 1 fused sample runs, 2 fused cell runs.
hipError_t launch_spread(const SpreadArgs& a, int fp64, int deg, int fused, const EpilogueOut& out,
                         hipStream_t st);
hipError_t launch_epilogue_spectra(const EpilogueArgs& a, const EpilogueOut& out, int fp64,
                                   int out_fp64, hipStream_t st);
// Second pass of the two-pass segment sum: stat += weighted sums of the
// power rows of each class template (one workgroup per template).
hipError_t launch_rows_sum(const EpilogueArgs& a, const EpilogueOut& out, int out_fp64, hipStream_t st);
hipError_t launch_rows_sum_multi(const EpilogueTable& t, int64_t blocks, EpilogueOut out, int out_fp64,
                                 hipStream_t st);
hipError_t launch_epilogue_sum(const EpilogueArgs& a, const EpilogueOut& out, int fp64, int out_fp64,
                               hipStream_t st);
hipError_t launch_fill_invalid(const int32_t* inv_inst, const int64_t* bin_off,
                               const int32_t* inst_K, int64_t n_inv, void* spectra,
                               void* power, int out_fp64, const uint8_t* mask, uint8_t* valid,
                               int64_t n_inst, hipStream_t st);
hipError_t launch_finite_scan(const void* strain, int64_t n, int fp64, int32_t* flag,
                              hipStream_t st);
// LDS of a spreader workgroup: phase table and one grid per wave; with
// pong = 1 (fused epilogue, one wave per instance) a second grid per wave
// holds the other half of the FFT's ping-pong.
size_t spread_lds_bytes(int fp64, int n, int pong = 0);
int phase_table_size(int fp64);
constexpr int kHornerPad = 16;   // zero coefficients appended to every class's tau series
size_t epilogue_lds_bytes(int fp64, int n, int K_max, int sum_mode);

// Set the message of nufft_resample_last_error(NULL) on this thread; returns code.
nr_status report_create_error(nr_status code, const std::string& msg);

// Plan (every device buffer carved from [base, base + bytes)), segment sum and
// release, with no device allocation; the arguments are those of
// nufft_resample_plan and nufft_resample_semicoherent_sum.  Synchronises the
// options' stream before and after.  Messages go to nufft_resample_last_error(NULL).
nr_status semicoherent_sum_in_arena(void* base, size_t bytes, const nr_segment* segs, int32_t n_segs,
                                    const nr_template* tmpls, int32_t n_tmpls, const nr_instance* inst,
                                    int64_t n_inst, double tol, const nr_options* opt, const void* strain,
                                    const double* seg_weight, void* stat, int32_t* n_used);

}  // namespace nr
