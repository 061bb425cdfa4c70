// Host plan runtime of the semicoherent NUFFT resampling library: argument
// validation, per-instance resampling constants, kernel-class grouping,
// NUFFT parameters, workspace and launch sequencing.  See
// include/nufft_resample.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/nufft_resample.h"
#include "nr_internal.hpp"
#include "nr_params.hpp"

using namespace nr;

namespace {

thread_local std::string g_create_error;

struct NrError : std::runtime_error {
    nr_status code;
    NrError(nr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(nr_status c, const std::string& m) { throw NrError(c, m); }

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) fail(NR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device memory of the plans built on this thread: NULL for hipMalloc, else
// a bump allocator over memory the caller provides (the static-scratch entry
// point), from which buffers are carved and never freed.
struct Arena {
    char* base;
    size_t size, used;
};
thread_local Arena* g_arena = nullptr;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool owned = false;   // allocated with hipMalloc (else carved from an arena)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned)
    {
        o.p = nullptr;
        o.bytes = 0;
        o.owned = false;
    }
    ~DevBuf()
    {
        if (p && owned) (void)hipFree(p);
    }
    void alloc(size_t b, const char* what)
    {
        if (b == 0) b = 16;
        if (g_arena) {
            const size_t at = (g_arena->used + 255) & ~size_t(255);
            if (at > g_arena->size || b > g_arena->size - at)
                fail(NR_ERR_OUT_OF_MEMORY, std::string("the plan needs more than the ") +
                                               std::to_string(g_arena->size) + "-byte static scratch (at " + what +
                                               ": " + std::to_string(at + b) + " bytes)");
            p = g_arena->base + at;
            g_arena->used = at + b;
            bytes = b;
            owned = false;
            return;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            fail(NR_ERR_OUT_OF_MEMORY, std::string("device allocation of ") + std::to_string(b) +
                                           " bytes for " + what + " failed: " + hipGetErrorString(e));
        }
        bytes = b;
        owned = true;
    }
    template <typename T>
    void upload(const std::vector<T>& v, const char* what)
    {
        alloc(v.size() * sizeof(T), what);
        if (!v.empty()) hip_check(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), what);
    }
};

struct Chunk {
    int64_t first, count, pt_base;
    int32_t tmpl_first, tmpl_count;
    int64_t order_off = -1;            // first entry of its workgroup order in Class::d_order (-1: none)
};

struct Class {
    int fp64, w, n, deg, parts;
    int method = NR_METHOD_FUSED;
    int snap = 0;
    int fuse_epi = 0;                  // the spreader runs the FFT / deconvolution / power itself
    int radix_code = 0;                // FFT radix plan (radix_code digits); 0: fft_radices(n)
    int kmax = 0;                      // largest K of the class
    int64_t grid_off = 0;              // batched mode: the class's grids and point stream
    int64_t pts_off = 0;               //   inside the plan's buffers (bytes)
    double beta_es;
    std::vector<int> radix;
    std::vector<InstDev> inst;         // class instances, ascending plan index
    std::vector<double> coef;          // Horner coefficients
    std::vector<SegDev> segs;          // lane-major strain layout (dst set once allocated)
    int64_t strain_entries = 0;        // lane-major entries (complex counts once)
    int64_t n_points = 0;              // sum of L
    int64_t pt_entries = 0;            // point-stream entries (runs padded to C samples)
    std::vector<Chunk> chunks;
    // segment-sum bookkeeping
    std::vector<int32_t> tmpl_id, tmpl_list;
    std::vector<int64_t> tmpl_list_off, tmpl_stat_off;
    // device copies
    int flush_period = 16;
    std::vector<int32_t> entry_seg;    // segment of each template-major list entry
    int64_t row_base = 0;              // two-pass sum: first element of the class's power rows
    DevBuf d_inst, d_coef, d_taps, d_dec, d_tw, d_phase, d_strain, d_tmpl_id, d_tmpl_list,
        d_tmpl_list_off, d_tmpl_stat_off, d_entry_seg, d_order;
};

// XCD-aware workgroup order.  The GPU deals the workgroups of a launch to its
// eight XCDs in turn (workgroup b to XCD b mod 8), and each XCD has its own
// L2; in list order every XCD would meet every segment and fetch the whole
// strain.  Large single-class launches instead sort their logical workgroups
// by segment and give each XCD one contiguous share of that order, so each L2
// meets mostly its own segments (measured on the 1 h workload: strain fetched
// about 2.8 times instead of 8, since a full GPU does not keep strict turns).
constexpr int kXcds = 8;
constexpr int64_t kOrderMinBlocks = 2048;

void build_block_order(Class& c)
{
    std::vector<int32_t> order;
    for (Chunk& ch : c.chunks) {
        ch.order_off = -1;
        if (c.method == NR_METHOD_DIRECT) continue;
        const int64_t G = spread_blocks(ch.count, c.parts);
        if (G < kOrderMinBlocks || G > INT32_MAX) continue;
        std::vector<std::pair<int32_t, int32_t>> key((size_t)G);   // (segment of the first item, block)
        bool several = false;
        for (int64_t b = 0; b < G; ++b) {
            const int64_t item = c.parts <= 4 ? b * (4 / c.parts) : b / (c.parts / 4);
            key[b] = {c.inst[ch.first + item].seg, (int32_t)b};
            several = several || key[b].first != key[0].first;
        }
        if (!several) continue;
        std::sort(key.begin(), key.end());
        ch.order_off = (int64_t)order.size();
        order.resize(order.size() + (size_t)G);
        int32_t* o = order.data() + ch.order_off;
        const int64_t q = G / kXcds, r = G % kXcds;
        for (int64_t b = 0; b < G; ++b) {
            const int64_t x = b % kXcds;       // XCD of hardware workgroup b, and its turn there
            o[b] = key[x * q + std::min(x, r) + b / kXcds].second;
        }
    }
    if (!order.empty()) c.d_order.upload(order, "workgroup order");
}

// The class tables of grouped launches travel in the kernel arguments
// (limited to 4 KiB).
static_assert(sizeof(SpreadTable) <= 2048 && sizeof(EpilogueTable) + sizeof(EpilogueOut) <= 2048,
              "class tables must fit the kernel argument segment");

// Classes launched together: one kernel instantiation and one LDS
// occupancy tier, each class's arguments in a table of the kernel arguments.
struct Group {
    std::vector<int> cls;
    int fp64 = 0, deg = 0, fused = 1, snap = 0;
    int fuse_epi = 0;                  // epilogue groups: classes whose spreader writes the outputs
    size_t lds[2] = {0, 0};            // spread: [0]; epilogue: [0] spectra, [1] segment sum
    int64_t blocks[2] = {0, 0};
    SpreadTable spread{};              // class tables (kernel arguments)
    EpilogueTable epi{};
};

}  // namespace

struct nr_plan_s {
    std::string err;
    nr_options opt{};
    int radix_override = 0;           // autotuner mini-plans: radix_code of every class
    hipStream_t stream = nullptr;
    int32_t n_segs = 0, n_tmpls = 0;
    int64_t n_inst = 0;
    std::vector<nr_segment> segs;
    std::vector<nr_template> tmpls;
    std::vector<int32_t> inst_seg, inst_tmpl, inst_K;
    std::vector<uint8_t> valid;
    std::vector<int64_t> bin_off, stat_off;
    std::vector<std::unique_ptr<Class>> classes;
    int out_fp64 = 0, strain_fp64 = 0, method = NR_METHOD_FUSED;
    int64_t n_valid = 0, valid_points = 0;
    DevBuf d_points, d_grid, d_mask, d_bin_off, d_inst_K, d_invalid, d_flag;
    // lane-major layout of every class, by destination precision
    std::vector<SegDev> lm_segs[2];
    int64_t lm_max_entries[2] = {0, 0};
    DevBuf d_lm_segs[2];
    // batched mode: every class in one chunk with its own grid region, the
    // classes launched in groups instead of one after another
    bool batched = false;
    bool two_pass = false;             // segment sum through power rows (P.d_rows)
    DevBuf d_rows;
    std::vector<Group> spread_groups, epi_groups;
    // side streams of a batched plan: independent groups run on them at the
    // same time, forked from and joined back to the plan's stream by events
    // (which HIP graph capture records as dependencies)
    std::vector<hipStream_t> side;
    hipEvent_t ev_fork[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> ev_join[2];
    int64_t n_invalid = 0;
    int64_t workspace = 0;
    int n_chunks = 0;
    // profiling: (stage, start, end) events of launches not yet read
    struct Timed {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    // captured launch sequences, keyed by call kind and pointer arguments
    struct Graph {
        int kind;
        const void* key[5];
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    ~nr_plan_s()
    {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        for (auto& t : timed) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        for (auto e : event_pool) (void)hipEventDestroy(e);
        for (int k = 0; k < 2; ++k) {
            if (ev_fork[k]) (void)hipEventDestroy(ev_fork[k]);
            for (auto e : ev_join[k]) (void)hipEventDestroy(e);
        }
        for (auto s : side) (void)hipStreamDestroy(s);
    }
};

namespace {

// ---------------------------------------------------------------- checks --

bool finite(double x) { return std::isfinite(x); }

void validate(const nr_segment* segs, int32_t n_segs, const nr_template* tmpls, int32_t n_tmpls,
              const nr_instance* inst, int64_t n_inst, double tol, const nr_options& o)
{
    if (!segs || n_segs <= 0) fail(NR_ERR_INVALID_ARG, "n_segs must be >= 1 with a segment array");
    if (!tmpls || n_tmpls <= 0) fail(NR_ERR_INVALID_ARG, "n_tmpls must be >= 1 with a template array");
    if (!(tol > 0.0 && tol <= 0.1) || !finite(tol)) fail(NR_ERR_INVALID_ARG, "tol must be in (0, 0.1]");
    if (o.precision < NR_FP32 || o.precision > NR_AUTO) fail(NR_ERR_INVALID_ARG, "unknown precision");
    if (o.method < NR_METHOD_AUTO || o.method > NR_METHOD_DIRECT) fail(NR_ERR_INVALID_ARG, "unknown method");
    if (o.sigma > 0.0 && !(o.sigma >= 1.25 && o.sigma <= 4.0))
        fail(NR_ERR_INVALID_ARG, "sigma must be in [1.25, 4]");
    if (o.parts != 0 && o.parts != 1 && o.parts != 2 && o.parts != 4 && o.parts != 8 && o.parts != 16)
        fail(NR_ERR_INVALID_ARG, "parts must be 0, 1, 2, 4, 8 or 16");
    if (o.strain_length < 0 || o.max_workspace_bytes < 0) fail(NR_ERR_INVALID_ARG, "negative size option");
    if (o.moment_mode < 0 || o.moment_mode > 2) fail(NR_ERR_INVALID_ARG, "moment_mode must be 0, 1 or 2");
    if (o.epilogue < 0 || o.epilogue > 2) fail(NR_ERR_INVALID_ARG, "epilogue must be 0, 1 or 2");
    if (o.flush_period < 0 || o.flush_period > 64 || (o.flush_period & (o.flush_period - 1)))
        fail(NR_ERR_INVALID_ARG, "flush_period must be 0 or a power of two up to 64");
    for (int32_t s = 0; s < n_segs; ++s) {
        const nr_segment& g = segs[s];
        if (g.n_samples < 1 || g.n_samples > (int64_t(1) << 30))
            fail(NR_ERR_INVALID_ARG, "segment " + std::to_string(s) + ": n_samples out of range");
        if (g.sample_offset < 0) fail(NR_ERR_INVALID_ARG, "segment " + std::to_string(s) + ": negative offset");
        if (!(g.fs > 0.0) || !finite(g.fs)) fail(NR_ERR_INVALID_ARG, "segment " + std::to_string(s) + ": fs must be > 0");
        if (!finite(g.t_start)) fail(NR_ERR_INVALID_ARG, "segment " + std::to_string(s) + ": t_start not finite");
        if (o.strain_length > 0 && g.sample_offset + g.n_samples > o.strain_length)
            fail(NR_ERR_INVALID_ARG, "segment " + std::to_string(s) + " runs past the strain");
    }
    for (int32_t m = 0; m < n_tmpls; ++m) {
        const nr_template& t = tmpls[m];
        const std::string id = "template " + std::to_string(m);
        if (!(t.mc_msun >= 0.0) || !finite(t.mc_msun)) fail(NR_ERR_INVALID_ARG, id + ": mc_msun must be >= 0");
        if (t.mc_msun > 0.0 && (!(t.f0 > 0.0) || !finite(t.f0))) fail(NR_ERR_INVALID_ARG, id + ": f0 must be > 0");
        if (t.n_bins < 1 || t.n_bins > (1 << 20)) fail(NR_ERR_INVALID_ARG, id + ": n_bins out of range");
        if (!finite(t.f_lo) || !finite(t.df) || !finite(t.f_max)) fail(NR_ERR_INVALID_ARG, id + ": non-finite frequency");
    }
    if (inst) {
        if (n_inst <= 0) fail(NR_ERR_INVALID_ARG, "n_inst must be >= 1 with an instance list");
        for (int64_t i = 0; i < n_inst; ++i) {
            if (inst[i].segment < 0 || inst[i].segment >= n_segs || inst[i].template_id < 0 ||
                inst[i].template_id >= n_tmpls)
                fail(NR_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": index out of range");
            if (!finite(inst[i].tol) || inst[i].tol > 0.1)
                fail(NR_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": tol must be <= 0.1");
        }
    } else if ((int64_t)n_segs * n_tmpls > (int64_t(1) << 31) - 1) {
        fail(NR_ERR_INVALID_ARG, "too many instances");
    }
}

// ------------------------------------------------------------ resampling --

struct InstHost {
    bool valid;
    double beta;
    long double a, c;  // tau scale and series variable per sample
    double y_max;
};

// Validity rule and tau constants of one instance (long double host math);
// beta is the template's Eq. (beta) value.
InstHost instance_constants(const nr_segment& g, const nr_template& t, double beta)
{
    InstHost h{};
    h.beta = beta;
    if (h.beta == 0.0) {
        h.valid = true;
        h.c = 1.0L / (long double)g.fs;
        return h;
    }
    const long double b = h.beta;
    const long double us = 1.0L - (8.0L / 3.0L) * b * (long double)g.t_start;
    const long double t_last = (long double)g.t_start + (long double)(g.n_samples - 1) / (long double)g.fs;
    const long double ul = 1.0L - (8.0L / 3.0L) * b * t_last;
    h.valid = (ul > 0.0L) && (us > 0.0L);
    if (h.valid && t.f_max > 0.0) {
        const long double f = (long double)t.f0 * powl(ul, -3.0L / 8.0L);
        if (f > (long double)t.f_max) h.valid = false;
    }
    if (!h.valid) return h;
    h.a = (3.0L / (5.0L * b)) * powl(us, 5.0L / 8.0L);
    h.c = (8.0L / 3.0L) * b / (us * (long double)g.fs);
    h.y_max = (double)(h.c * (long double)(g.n_samples - 1));
    return h;
}

// Horner coefficients b_k (k = 1..d) of dtau(j) = a sum_k e_k (c j)^k, the
// binomial series of 1 - (1 - y)^{5/8}; returns d, or -1 when the series
// needs more than kMaxHorner terms for the requested phase accuracy.
// e_k of 1 - (1 - y)^{5/8} = sum_k e_k y^k (all positive): e_1 = 5/8,
// e_k = e_{k-1} (k - 1 - 5/8) / k.
const std::vector<long double>& binomial_e()
{
    static const std::vector<long double> e = [] {
        std::vector<long double> v(kMaxHorner + 2, 0.0L);
        v[1] = 0.625L;
        for (int k = 2; k <= kMaxHorner + 1; ++k) v[k] = v[k - 1] * ((long double)(k - 1) - 0.625L) / (long double)k;
        return v;
    }();
    return e;
}

int horner_series(const InstHost& h, double f_ref, double cyc_tol, std::vector<double>& out)
{
    const long double y = h.y_max;
    if (y <= 0.0L) {
        out.push_back((double)(h.a * 0.625L * h.c));
        return 1;
    }
    if (y >= 0.9L) return -1;
    const std::vector<long double>& e = binomial_e();
    int d = -1;
    long double yk1 = y * y;  // y^{k+1}
    const long double scale = h.a * (long double)f_ref / (1.0L - y);
    for (int k = 1; k <= kMaxHorner; ++k) {
        // terms are positive and fall at least geometrically with ratio y
        if (scale * e[k + 1] * yk1 <= (long double)cyc_tol) {
            d = k;
            break;
        }
        yk1 *= y;
    }
    if (d < 0) return -1;
    long double ck = 1.0L;
    for (int k = 1; k <= d; ++k) {
        ck *= h.c;
        out.push_back((double)(h.a * e[k] * ck));
    }
    return d;
}

// The method an option value stands for (AUTO: the fused sample-run spreader).
int resolve_method(int m)
{
    return m == NR_METHOD_AUTO ? NR_METHOD_FUSED : m;
}

// Spreader code of a class for the launchers: 0 staged, 1 fused sample
// runs, 2 fused cell runs.
int spread_code(int method)
{
    return method == NR_METHOD_STAGED ? 0 : method == NR_METHOD_CELLRUN ? 2 : 1;
}

// Grid cells that one instance's time series visits: its unwrapped cell
// index spans about n df dtau(L - 1) cells, plus the two ends.
double cells_visited(const InstHost& h, int64_t L, int n, double df)
{
    long double span;
    if (h.beta == 0.0)
        span = h.c * (long double)(L - 1);
    else
        span = h.a * (1.0L - powl(1.0L - (long double)h.y_max, 0.625L));
    return (double)((long double)n * (long double)df * span + 2.0L);
}

// Rounds of cell runs (one per lane) that one cell-run instance needs.
int cellrun_rounds(const InstHost& h, int64_t L, int n, double df)
{
    return (int)std::min(1e6, std::ceil(cells_visited(h, L, n, df) / kRunsPerRound));
}

int default_parts(int64_t L)
{
    if (L <= 16384) return 1;
    if (L <= 32768) return 2;
    return 4;
}

// Waves per cell-run instance (its rounds are dealt to its waves in turn).
// Plans too small to fill the GPU (plan_waves at one wave per instance):
// more waves, up to 16 and one round each, while the plan has fewer than
// 8192 waves, then only while every wave keeps four rounds (a wave's fixed
// cost, zeroing and reducing its grid copy, is then amortised); otherwise
// the sample-run rule, keeping at least four rounds per wave.
int cellrun_parts(int rounds, bool small_plan, int64_t L, int64_t plan_waves)
{
    int p = 1;
    if (small_plan) {
        while (p * 2 <= 16 && p * 2 <= rounds && (plan_waves * p < 8192 || rounds >= 4 * p * 2)) p *= 2;
    } else {
        while (p * 2 <= default_parts(L) && rounds >= 4 * p * 2) p *= 2;
    }
    return p;
}

// Automatic spreader: cell runs, unless the time series spends fewer than
// kCellRunMinDensity samples in each cell it visits AND the spreader's LDS
// leaves fewer than five workgroups per compute unit (sparse runs pay more
// for the run search and partly used quads than they save, and that
// search's dependent chain needs resident waves to hide behind).  The
// density bar is lower in plans with at least 4096 instances: measured on
// the beta bank (8280 instances, 12.8 samples per cell, n = 1200) cell runs
// with four waves per instance take 1.01 ms per step against 1.11 ms for
// sample runs, while on the 512-instance ragged batch the same switch for its
// 12.8-sample classes costs 0.318 -> 0.350 ms.
constexpr double kCellRunMinDensity = 24.0;
constexpr double kCellRunMinDensityLarge = 12.0;
constexpr int64_t kLargePlanWaves = 4096;
constexpr size_t kCellRunMaxSparseLds = kLdsBytes / 5;
// Longest heterodyne phase span, in phase-table steps, of an FP64 instance on
// the fused spreaders (half the range of their 32-bit table-step conversion;
// FP32 classes have no table and no such limit).
constexpr double kFusedMaxPhaseSteps = 1073741824.0;

// LDS occupancy tier: workgroups per compute unit that the LDS allows.
int lds_tier(size_t bytes)
{
    return (int)std::min<size_t>(8, kLdsBytes / std::max<size_t>(bytes, 1));
}

// Waves per instance when the whole plan has too few waves to fill the chip:
// enough to bring the samples per lane down to about 64 (at most 16 waves).
int small_plan_parts(int64_t L)
{
    int p = default_parts(L);
    while (p < 16 && (L + (int64_t)kWave * p - 1) / ((int64_t)kWave * p) > 64) p *= 2;
    return p;
}

struct ClassKey {
    int fp64, w, n, parts, method, flush, snap, radix;
    bool operator<(const ClassKey& o) const
    {
        return std::tie(fp64, w, n, parts, method, flush, snap, radix) <
               std::tie(o.fp64, o.w, o.n, o.parts, o.method, o.flush, o.snap, o.radix);
    }
};

// ------------------------------------------------------------- autotuner --

// Spreader configuration and FFT radix plan of one shape (precision, kernel
// width, grid, samples).
struct Tuned {
    int method, parts, flush, snap;
    double us_per_inst;
    int radix;   // radix_code of the fastest FFT plan (0: the default order)
};
// batch 0: tuned for throughput on a mini-plan that fills the GPU; > 0: for a
// plan too small to fill it, on a mini-plan of that many instances.
struct ShapeKey {
    int fp64, w, n;
    int64_t L, batch;
    bool operator<(const ShapeKey& o) const
    {
        return std::tie(fp64, w, n, L, batch) < std::tie(o.fp64, o.w, o.n, o.L, o.batch);
    }
};

std::mutex g_tune_mutex;
std::map<ShapeKey, Tuned> g_tuned;             // process-wide results
std::map<std::string, bool> g_cache_loaded;    // cache files already read

void load_tune_cache(const char* path)
{
    if (!path || g_cache_loaded[path]) return;
    g_cache_loaded[path] = true;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    // one shape per line; the radix plan (tenth field) and the small-plan
    // batch (eleventh) may be absent
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        ShapeKey k;
        Tuned t{};
        long long L, batch = 0;
        const int got = std::sscanf(line, "%d %d %d %lld %d %d %d %d %lf %d %lld", &k.fp64, &k.w, &k.n, &L,
                                    &t.method, &t.parts, &t.flush, &t.snap, &t.us_per_inst, &t.radix, &batch);
        if (got < 9) continue;
        if (got < 10) t.radix = 0;
        if (got < 11) batch = 0;
        k.batch = batch;
        const std::vector<int> r = radix_from_code(t.radix);
        int prod = 1;
        for (int q : r) prod = (q >= 2 && q <= 5 && prod <= k.n) ? prod * q : -1;
        if (t.radix != 0 && prod != k.n) t.radix = 0;   // not a plan of this size: use the default
        k.L = L;
        g_tuned[k] = t;
    }
    std::fclose(f);
}

void save_tune_cache(const char* path)
{
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto& kv : g_tuned)
        std::fprintf(f, "%d %d %d %lld %d %d %d %d %.6f %d %lld\n", kv.first.fp64, kv.first.w, kv.first.n,
                     (long long)kv.first.L, kv.second.method, kv.second.parts, kv.second.flush, kv.second.snap,
                     kv.second.us_per_inst, kv.second.radix, (long long)kv.first.batch);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

template <typename T>
std::vector<T> cast_vec(const std::vector<long double>& v)
{
    std::vector<T> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
    return o;
}

void build_class_tables(Class& c, double tol_cls, double sigma)
{
    // Chebyshev pieces of the kernel and the degree that reaches the target
    std::vector<long double> taps;
    c.deg = kernel_pieces(c.w, c.beta_es, tol_cls, kMaxDeg, taps);
    // deconvolution factors 1/psi_hat(2 pi l' / n), l' = min(l, n - l)
    std::vector<long double> dec(c.n);
    for (int l = 0; l < c.n; ++l) {
        const int lp = std::min(l, c.n - l);
        dec[l] = 1.0L / es_fourier(c.w, c.beta_es, 2.0L * 3.14159265358979323846264338327950288L * lp / c.n);
    }
    std::vector<long double> tw(2 * (size_t)c.n);
    for (int t = 0; t < c.n; ++t) {
        const long double ang = -2.0L * 3.14159265358979323846264338327950288L * t / c.n;
        tw[2 * t] = cosl(ang);
        tw[2 * t + 1] = sinl(ang);
    }
    c.radix = c.radix_code ? radix_from_code(c.radix_code) : fft_radices(c.n);
    // coarse heterodyne phasors exp(2 pi i k / N)
    const int NT = phase_table_size(c.fp64);
    std::vector<long double> ph(2 * (size_t)NT);
    for (int k = 0; k < NT; ++k) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * k / NT;
        ph[2 * k] = cosl(ang);
        ph[2 * k + 1] = sinl(ang);
    }
    if (c.fp64) {
        c.d_taps.upload(cast_vec<double>(taps), "kernel pieces");
        c.d_dec.upload(cast_vec<double>(dec), "deconvolution");
        c.d_tw.upload(cast_vec<double>(tw), "twiddles");
        c.d_phase.upload(cast_vec<double>(ph), "phase table");
    } else {
        c.d_taps.upload(cast_vec<float>(taps), "kernel pieces");
        c.d_dec.upload(cast_vec<float>(dec), "deconvolution");
        c.d_tw.upload(cast_vec<float>(tw), "twiddles");
        c.d_phase.upload(cast_vec<float>(ph), "phase table");
    }
    (void)sigma;
}

Tuned tuned_config(const nr_options& base, const nr_segment& g, const nr_template& t, double tol, int fp64,
                   int w, int n, int64_t small_batch);
void build_groups(nr_plan_s& P);

void create_plan(nr_plan_s& P, const nr_segment* segs, int32_t n_segs, const nr_template* tmpls,
                 int32_t n_tmpls, const nr_instance* inst, int64_t n_inst, double tol)
{
    const nr_options& o = P.opt;
    validate(segs, n_segs, tmpls, n_tmpls, inst, n_inst, tol, o);
    const double sigma = o.sigma > 0.0 ? o.sigma : 2.0;
    P.stream = (hipStream_t)o.stream;
    P.n_segs = n_segs;
    P.n_tmpls = n_tmpls;
    P.segs.assign(segs, segs + n_segs);
    P.tmpls.assign(tmpls, tmpls + n_tmpls);
    P.n_inst = inst ? n_inst : (int64_t)n_segs * n_tmpls;
    P.out_fp64 = o.precision != NR_FP32;
    P.strain_fp64 = P.out_fp64;
    P.method = resolve_method(o.method);

    const int64_t N = P.n_inst;
    P.inst_seg.resize(N);
    P.inst_tmpl.resize(N);
    P.inst_K.resize(N);
    P.valid.assign(N, 0);
    P.bin_off.resize(N + 1);
    std::vector<double> inst_tol(N, tol);
    for (int64_t i = 0; i < N; ++i) {
        if (inst) {
            P.inst_seg[i] = inst[i].segment;
            P.inst_tmpl[i] = inst[i].template_id;
            if (inst[i].tol > 0.0) inst_tol[i] = inst[i].tol;
        } else {
            P.inst_seg[i] = (int32_t)(i % n_segs);
            P.inst_tmpl[i] = (int32_t)(i / n_segs);
        }
        P.inst_K[i] = P.tmpls[P.inst_tmpl[i]].n_bins;
    }
    P.bin_off[0] = 0;
    for (int64_t i = 0; i < N; ++i) P.bin_off[i + 1] = P.bin_off[i] + P.inst_K[i];
    P.stat_off.resize(n_tmpls + 1);
    P.stat_off[0] = 0;
    for (int32_t m = 0; m < n_tmpls; ++m) P.stat_off[m + 1] = P.stat_off[m] + P.tmpls[m].n_bins;

    // Precision class and tolerance checks
    for (int64_t i = 0; i < N; ++i) {
        const double t = inst_tol[i];
        if (o.precision == NR_FP32 && t < kFp32MinTol && o.strict)
            fail(NR_ERR_TOL_UNATTAINABLE, "instance " + std::to_string(i) + ": FP32 cannot reach tol " +
                                              std::to_string(t) + " (minimum 1e-6); use NR_FP64 or NR_AUTO");
        if (t < kFp64MinTol && o.strict)
            fail(NR_ERR_TOL_UNATTAINABLE, "instance " + std::to_string(i) + ": tol below 1e-12");
    }

    std::map<ClassKey, size_t> class_of;
    std::map<ClassKey, double> class_tol;
    // largest grid whose spreader LDS (grids plus phase table) fits a workgroup
    int n_max_of[2];
    for (int f = 0; f < 2; ++f) {
        int lo = 1, hi = 1 << 16;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            const bool fits = spread_lds_bytes(f, mid) <= kLdsBytes &&
                              epilogue_lds_bytes(f, mid, mid, 1) <= kLdsBytes;
            if (fits) lo = mid; else hi = mid - 1;
        }
        n_max_of[f] = lo;
    }
    // plans with few waves: spread each instance over more waves
    bool small_plan = false;
    int64_t plan_waves = 0;
    if (o.parts == 0) {
        int64_t waves = 0;
        for (int64_t i = 0; i < N && waves < 16384; ++i) waves += default_parts(P.segs[P.inst_seg[i]].n_samples);
        small_plan = waves < 16384;
        plan_waves = waves;
    }
    std::vector<double> tmpl_beta(n_tmpls);
    for (int32_t m = 0; m < n_tmpls; ++m) tmpl_beta[m] = chirp_beta(P.tmpls[m].mc_msun, P.tmpls[m].f0);
    // tuning a plan too small to fill the GPU: how many valid instances each
    // shape (precision, width, grid, samples) has
    std::map<std::array<int64_t, 4>, int64_t> shape_count;
    if (o.tune && small_plan) {
        for (int64_t i = 0; i < N; ++i) {
            const nr_segment& g = P.segs[P.inst_seg[i]];
            const nr_template& t = P.tmpls[P.inst_tmpl[i]];
            if (!instance_constants(g, t, tmpl_beta[P.inst_tmpl[i]]).valid) continue;
            const int fp64 = (o.precision == NR_FP64 || (o.precision == NR_AUTO && inst_tol[i] < kFp32MinTol)) ? 1 : 0;
            const double tol_eff = std::max(inst_tol[i], fp64 ? kFp64MinTol : kFp32MinTol);
            const int w = kernel_width(tol_eff, sigma);
            const int n = fft_size(std::max((int64_t)std::ceil(sigma * t.n_bins - 1e-9), (int64_t)2 * w));
            ++shape_count[{fp64, w, n, g.n_samples}];
        }
    }
    // kernel width per distinct tolerance, and the last class looked up
    std::map<std::pair<double, int>, int> width_of;
    ClassKey last_key{-1, -1, -1, -1, -1, -1, -1, -1};
    std::vector<double> series;
    size_t last_ci = 0;
    for (int64_t i = 0; i < N; ++i) {
        const nr_segment& g = P.segs[P.inst_seg[i]];
        const nr_template& t = P.tmpls[P.inst_tmpl[i]];
        const InstHost h = instance_constants(g, t, tmpl_beta[P.inst_tmpl[i]]);
        if (!h.valid) continue;
        P.valid[i] = 1;
        ++P.n_valid;
        P.valid_points += g.n_samples;
        int fp64 = o.precision == NR_FP64 ? 1 : 0;
        if (o.precision == NR_AUTO && inst_tol[i] < kFp32MinTol) fp64 = 1;
        const double tol_eff = std::max(inst_tol[i], fp64 ? kFp64MinTol : kFp32MinTol);
        const int w = kernel_width(tol_eff, sigma);
        const int K = t.n_bins;
        int n;
        {
            auto wk = width_of.find({sigma * K, w});
            if (wk == width_of.end()) {
                n = fft_size(std::max((int64_t)std::ceil(sigma * K - 1e-9), (int64_t)2 * w));
                width_of[{sigma * K, w}] = n;
            } else {
                n = wk->second;
            }
        }
        const int n_max = n_max_of[fp64];
        if (n > n_max)
            fail(NR_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": grid size " + std::to_string(n) +
                                         " exceeds the supported maximum " + std::to_string(n_max) +
                                         " (lower n_bins or sigma)");
        // tau series of the instance (ndeg < 0: the log1p/expm1 form)
        const double df_i = t.df > 0.0 ? t.df : g.fs / (double)g.n_samples;
        series.clear();
        int ndeg = 0;
        double phase_steps = 0.0;   // heterodyne phase span in phase-table steps
        if (h.beta != 0.0) {
            const double f_ref = std::fabs(t.f_lo) + (double)K * df_i + df_i;
            ndeg = horner_series(h, f_ref, fp64 ? 1e-14 : 1e-11, series);
        }
        {
            // The heterodyne phase fc dtau is evaluated in FP64: the tau
            // series (or log1p/expm1) and the product with fc each add a few
            // units in the last place, so the phase in cycles carries a
            // relative error of about (degree + 3) 2^-53, which grows with
            // the cycles the segment spans.  An instance whose phase error
            // would exceed a quarter of its tolerance cannot reach it in any
            // precision class: an error in strict plans (otherwise the
            // phase error bounds what the instance attains).  The phase must
            // also stay below 2^38 cycles, far inside the range of the
            // kernels' FP64 rounding to the nearest cycle or table step.
            const long double span = h.beta == 0.0 ? h.c * (long double)(g.n_samples - 1)
                                                    : h.a * (1.0L - powl(1.0L - (long double)h.y_max, 0.625L));
            const double fc = t.f_lo + (double)(K / 2) * df_i;
            const double cycles = std::fabs(fc) * (double)span;
            phase_steps = cycles * (double)phase_table_size(fp64);
            if (cycles * 1024.0 >= 281474976710656.0)
                fail(NR_ERR_INVALID_ARG, "instance " + std::to_string(i) +
                                             ": heterodyne frequency x duration too large (over 2^38 cycles)");
            const double terms = (ndeg > 0 ? ndeg : ndeg == 0 ? 1 : 8) + 3;
            const double phase_err = 2.0 * M_PI * cycles * terms * 0x1p-53;
            if (o.strict && phase_err > 0.25 * tol_eff)
                fail(NR_ERR_TOL_UNATTAINABLE,
                     "instance " + std::to_string(i) + ": the FP64 heterodyne phase over " +
                         std::to_string(cycles) + " cycles is accurate to about " + std::to_string(phase_err) +
                         " rad, too coarse for tolerance " + std::to_string(tol_eff));
        }
        int method = resolve_method(o.method);
        if (o.method == NR_METHOD_AUTO &&
            ((double)g.n_samples >= (small_plan && plan_waves < kLargePlanWaves ? kCellRunMinDensity
                                                                                : kCellRunMinDensityLarge) *
                                        cells_visited(h, g.n_samples, n, df_i) ||
             spread_lds_bytes(fp64, n) <= kCellRunMaxSparseLds))
            method = NR_METHOD_CELLRUN;
        int parts = o.parts ? o.parts : small_plan ? small_plan_parts(g.n_samples) : default_parts(g.n_samples);
        if (method == NR_METHOD_CELLRUN && o.parts == 0)
            parts = cellrun_parts(cellrun_rounds(h, g.n_samples, n, df_i), small_plan, g.n_samples, plan_waves);
        int flush = o.flush_period;
        int snap = o.moment_mode == 2 ? 1 : 0;
        int radix = P.radix_override;
        if (o.tune) {
            const int64_t sb = small_plan ? shape_count[{fp64, w, n, g.n_samples}] : 0;
            const Tuned tu = tuned_config(o, g, t, tol_eff, fp64, w, n, sb);
            method = tu.method;
            flush = tu.flush;
            snap = tu.snap;
            radix = tu.radix;
            if (tu.parts > 0)
                parts = tu.parts;
            else if (o.parts == 0)   // automatic waves per instance for the tuned method
                parts = method == NR_METHOD_CELLRUN
                            ? cellrun_parts(cellrun_rounds(h, g.n_samples, n, df_i), small_plan, g.n_samples,
                                            plan_waves)
                            : small_plan_parts(g.n_samples);
        }
        // the fused spreaders and the direct baseline carry only the series
        // form of tau; instances that need log1p/expm1 get their points from
        // the tau kernel
        if (ndeg < 0) method = NR_METHOD_STAGED;
        // the FP64 fused spreaders pick the phase-table entry through a 32-bit
        // conversion of the phase in table steps; longer phase spans take the
        // staged path, whose tau kernel reduces the phase modulo one cycle
        // (FP32 classes: phase_steps is 0, they have no table)
        if (phase_steps >= kFusedMaxPhaseSteps && method != NR_METHOD_DIRECT) method = NR_METHOD_STAGED;
        if (method == NR_METHOD_CELLRUN) snap = 0;  // moments restart with every run
        ClassKey key{fp64, w, n, parts, method, flush, snap, radix};
        size_t ci;
        const bool same = !(key < last_key) && !(last_key < key);
        auto it = same ? class_of.end() : class_of.find(key);
        if (same) {
            ci = last_ci;
            if (tol_eff < class_tol[key]) class_tol[key] = tol_eff;
        } else if (it == class_of.end()) {
            ci = P.classes.size();
            class_of[key] = ci;
            class_tol[key] = tol_eff;
            auto c = std::make_unique<Class>();
            c->fp64 = fp64;
            c->w = w;
            c->n = n;
            c->parts = parts;
            c->method = method;
            c->flush_period = flush;
            c->snap = snap;
            c->radix_code = radix;
            c->beta_es = es_beta(w, sigma);
            P.classes.push_back(std::move(c));
        } else {
            ci = it->second;
            class_tol[key] = std::min(class_tol[key], tol_eff);
        }
        last_key = key;
        last_ci = ci;
        Class& c = *P.classes[ci];
        InstDev d{};
        const double df = t.df > 0.0 ? t.df : g.fs / (double)g.n_samples;
        d.df = df;
        d.m0 = K / 2;
        d.fc = t.f_lo + (double)d.m0 * df;
        d.L = (int32_t)g.n_samples;
        // cell runs and the direct baseline read a plain copy of the segment
        // (lane-major layout with C = 1)
        d.C = (method == NR_METHOD_CELLRUN || method == NR_METHOD_DIRECT)
                  ? 1
                  : (int32_t)((g.n_samples + (int64_t)kWave * parts - 1) / ((int64_t)kWave * parts));
        d.K = K;
        d.inst = (int32_t)i;
        d.seg = P.inst_seg[i];
        d.a = (double)h.a;
        d.c = (double)h.c;
        d.ndeg = ndeg;
        if (ndeg > 0) {
            d.coef_off = (int32_t)c.coef.size();
            c.coef.insert(c.coef.end(), series.begin(), series.end());
        }
        c.inst.push_back(d);
        c.kmax = std::max(c.kmax, K);
        c.n_points += g.n_samples;
    }
    for (auto& kv : class_of) build_class_tables(*P.classes[kv.second], class_tol[kv.first], sigma);

    // Lane-major strain layout per class, point-stream offsets, templates
    const size_t psize_f = 8, psize_d = 16;
    int64_t grid_chunk_bytes = 0, point_chunk_bytes = 0, grid_total = 0, point_total = 0;
    const int64_t cap = o.max_workspace_bytes > 0 ? o.max_workspace_bytes : (int64_t(8) << 30);
    int64_t fixed_bytes = 0;
    for (auto& cp : P.classes) {
        Class& c = *cp;
        std::vector<int64_t> seg_at(P.n_segs, -1);
        const int esize = (c.fp64 ? 8 : 4) * (o.strain_complex ? 2 : 1);
        int64_t pt = 0;
        std::vector<int32_t> tmpl_at(P.n_tmpls, -1);
        std::vector<std::vector<int32_t>> lists;
        for (size_t k = 0; k < c.inst.size(); ++k) {
            InstDev& d = c.inst[k];
            if (seg_at[d.seg] < 0) {
                SegDev sd{};
                sd.src_off = P.segs[d.seg].sample_offset;
                sd.dst_off = c.strain_entries;
                sd.L = d.L;
                sd.C = d.C;
                sd.parts = (c.method == NR_METHOD_CELLRUN || c.method == NR_METHOD_DIRECT)
                               ? (int32_t)((d.L + kWave - 1) / kWave)
                               : c.parts;
                c.segs.push_back(sd);
                seg_at[d.seg] = sd.dst_off;
                c.strain_entries += (int64_t)sd.parts * d.C * kWave;
            }
            d.strain_off = seg_at[d.seg];
            d.pt_off = pt;
            pt += (int64_t)c.parts * d.C * kWave;
            d.bin_off = P.bin_off[d.inst];
            const int32_t pm = P.inst_tmpl[d.inst];
            if (tmpl_at[pm] < 0) {
                tmpl_at[pm] = (int32_t)c.tmpl_id.size();
                c.tmpl_id.push_back(pm);
                c.tmpl_stat_off.push_back(P.stat_off[pm]);
                lists.emplace_back();
            }
            lists[tmpl_at[pm]].push_back((int32_t)k);
        }
        c.pt_entries = pt;
        c.tmpl_list_off.push_back(0);
        for (auto& l : lists) {
            for (int32_t k : l) {
                c.inst[k].entry = (int32_t)c.tmpl_list.size();
                c.entry_seg.push_back(c.inst[k].seg);
                c.tmpl_list.push_back(k);
            }
            c.tmpl_list_off.push_back((int64_t)c.tmpl_list.size());
        }
        // collective flush period: about half the samples a lane spends in one cell
        if (c.flush_period <= 0) {
            long double pts_per_cell = 0.0L;
            for (const InstDev& d : c.inst) {
                const long double span = std::max(1.0L, (long double)d.df * d.L / (long double)P.segs[d.seg].fs);
                pts_per_cell += (long double)d.L / ((long double)c.n * span);
            }
            pts_per_cell /= std::max<size_t>(c.inst.size(), 1);
            int f = 1;
            while (f < 64 && 2.0L * f * 2.0L <= pts_per_cell) f *= 2;
            c.flush_period = f;
        }
        // class template of each class instance, to bound each chunk's template range
        std::vector<int32_t> ct_of(c.inst.size());
        for (size_t t = 0; t < lists.size(); ++t)
            for (int32_t k : lists[t]) ct_of[k] = (int32_t)t;
        fixed_bytes += c.strain_entries * esize;
        // chunks bounded by the workspace cap
        // the direct baseline needs no grid
        const int64_t gsize =
            c.method == NR_METHOD_DIRECT ? 0 : (int64_t)c.n * (c.fp64 ? 16 : 8) * grid_slots(c.parts);
        const int64_t psz = c.method == NR_METHOD_STAGED ? (c.fp64 ? psize_d : psize_f) : 0;
        const int64_t budget = std::max<int64_t>(cap / 2, 1);
        int64_t k0 = 0;
        while (k0 < (int64_t)c.inst.size()) {
            int64_t k1 = k0, gb = 0, pb = 0;
            int32_t tlo = INT32_MAX, thi = -1;
            while (k1 < (int64_t)c.inst.size()) {
                const int64_t pts = (int64_t)c.parts * c.inst[k1].C * kWave;
                if (k1 > k0 && (gb + gsize + pb + pts * psz > budget || k1 - k0 >= (int64_t(1) << 28))) break;
                gb += gsize;
                pb += pts * psz;
                tlo = std::min(tlo, ct_of[k1]);
                thi = std::max(thi, ct_of[k1]);
                ++k1;
            }
            Chunk ch{k0, k1 - k0, c.inst[k0].pt_off, tlo, thi - tlo + 1};
            c.chunks.push_back(ch);
            grid_chunk_bytes = std::max(grid_chunk_bytes, gb);
            point_chunk_bytes = std::max(point_chunk_bytes, pb);
            grid_total += gb;
            point_total += pb;
            k0 = k1;
        }
        P.n_chunks += (int)c.chunks.size();
        // fused epilogue: the instance's waves share one workgroup (at most
        // four waves), the FFT's second buffer (one more grid per wave when an
        // instance has one wave) costs no workgroups per compute unit, and the
        // plan has at least 4096 waves.  Measured: the 1 h workload (60-cell
        // grids) runs as fast either way with half the memory traffic, the
        // beta bank (8280 instances of four waves, 1200 cells) 1 % faster; in
        // the 512-instance ragged batch, too small to fill the GPU, every
        // workgroup's transform lengthens the launch it ends (0.32 -> 0.38 ms)
        {
            const bool wanted =
                (o.epilogue == 0 && (!small_plan || plan_waves >= kLargePlanWaves)) || o.epilogue == 2;
            const bool fits = c.method != NR_METHOD_DIRECT && c.parts <= 4 &&
                              lds_tier(spread_lds_bytes(c.fp64, c.n, c.parts == 1)) >=
                                  lds_tier(spread_lds_bytes(c.fp64, c.n, 0));
            c.fuse_epi = wanted && fits ? 1 : 0;
        }
        build_block_order(c);
        // device tables
        c.d_inst.upload(c.inst, "instances");
        c.coef.resize(c.coef.size() + kHornerPad, 0.0);  // whole-width register loads stay in bounds
        c.d_coef.upload(c.coef, "tau series");
        c.d_strain.alloc((size_t)c.strain_entries * esize, "lane-major strain");
        for (SegDev& sd : c.segs) {
            sd.dst = c.d_strain.p;
            P.lm_segs[c.fp64].push_back(sd);
            P.lm_max_entries[c.fp64] = std::max(P.lm_max_entries[c.fp64], (int64_t)sd.parts * sd.C * kWave);
        }
        c.d_tmpl_id.upload(c.tmpl_id, "templates");
        c.d_tmpl_list.upload(c.tmpl_list, "template lists");
        c.d_tmpl_list_off.upload(c.tmpl_list_off, "template lists");
        c.d_tmpl_stat_off.upload(c.tmpl_stat_off, "template offsets");
        c.d_entry_seg.upload(c.entry_seg, "list segments");
        P.workspace += (int64_t)(c.d_inst.bytes + c.d_coef.bytes + c.d_strain.bytes +
                                 c.d_phase.bytes + c.d_taps.bytes + c.d_dec.bytes + c.d_tw.bytes + c.d_tmpl_id.bytes +
                                 c.d_tmpl_list.bytes + c.d_tmpl_list_off.bytes + c.d_tmpl_stat_off.bytes +
                                 c.d_entry_seg.bytes + c.d_order.bytes);
    }
    if (fixed_bytes + grid_chunk_bytes + point_chunk_bytes > cap)
        fail(NR_ERR_OUT_OF_MEMORY, "workspace of " + std::to_string(fixed_bytes + grid_chunk_bytes + point_chunk_bytes) +
                                       " bytes exceeds max_workspace_bytes " + std::to_string(cap));
    // Batched mode when every class fits one chunk and all grids fit together.
    bool one_chunk = true, any_direct = false;
    for (auto& cp : P.classes) {
        one_chunk = one_chunk && cp->chunks.size() <= 1;
        any_direct = any_direct || cp->method == NR_METHOD_DIRECT;
    }
    P.batched = P.classes.size() > 1 && one_chunk && !any_direct && fixed_bytes + grid_total + point_total <= cap &&
                grid_total + point_total <= std::max<int64_t>(cap / 2, 1);
    if (P.batched) {
        int64_t go = 0, po = 0;
        for (auto& cp : P.classes) {
            Class& c = *cp;
            c.grid_off = go;
            c.pts_off = po;
            const int64_t gsize = (int64_t)c.n * (c.fp64 ? 16 : 8) * grid_slots(c.parts);
            go += (int64_t)c.inst.size() * gsize;
            if (c.method == NR_METHOD_STAGED)
                po += c.pt_entries * (c.fp64 ? (int64_t)psize_d : (int64_t)psize_f);
            go = (go + 255) & ~int64_t(255);
            po = (po + 255) & ~int64_t(255);
        }
        grid_chunk_bytes = go;
        point_chunk_bytes = po;
    }
    // Two-pass segment sum (power rows, then per-template row sums) when
    // every class fits one chunk and the rows fit the workspace.
    {
        int64_t rows = 0;
        for (auto& cp : P.classes) {
            cp->row_base = rows;
            rows += (int64_t)cp->inst.size() * cp->kmax;
        }
        const int64_t rbytes = rows * (P.out_fp64 ? 8 : 4);
        P.two_pass = one_chunk && !P.classes.empty() &&
                     fixed_bytes + grid_chunk_bytes + point_chunk_bytes + rbytes <= cap;
        if (P.two_pass) P.d_rows.alloc((size_t)rbytes, "power rows");
        if (any_direct && !P.two_pass)
            fail(NR_ERR_OUT_OF_MEMORY, "the direct method needs every class in one chunk with its power rows "
                                       "inside max_workspace_bytes");
    }
    P.d_grid.alloc((size_t)grid_chunk_bytes, "grid");
    if (point_chunk_bytes > 0) P.d_points.alloc((size_t)point_chunk_bytes, "point stream");
    for (int f = 0; f < 2; ++f) P.d_lm_segs[f].upload(P.lm_segs[f], "segments");
    if (P.batched) {
        build_groups(P);
        P.n_chunks = (int)P.spread_groups.size();
        const size_t most = std::max(P.spread_groups.size(), P.epi_groups.size());
        // plans built in an arena create no streams or events
        const int n_side = g_arena ? 0 : (int)std::min<size_t>(3, most > 0 ? most - 1 : 0);
        for (int i = 0; i < n_side; ++i) {
            hipStream_t st;
            hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "side stream");
            P.side.push_back(st);
        }
        for (int k = 0; k < 2 && n_side > 0; ++k) {
            hip_check(hipEventCreateWithFlags(&P.ev_fork[k], hipEventDisableTiming), "fork event");
            for (int i = 0; i < n_side; ++i) {
                hipEvent_t e;
                hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "join event");
                P.ev_join[k].push_back(e);
            }
        }
    }
    if (!P.classes.empty()) P.method = P.classes[0]->method;
    P.d_mask.upload(P.valid, "mask");
    std::vector<int32_t> invalid;
    for (int64_t i = 0; i < N; ++i)
        if (!P.valid[i]) invalid.push_back((int32_t)i);
    P.n_invalid = (int64_t)invalid.size();
    P.d_invalid.upload(invalid, "invalid list");
    P.d_bin_off.upload(P.bin_off, "bin offsets");
    P.d_inst_K.upload(P.inst_K, "bins");
    P.d_flag.alloc(sizeof(int32_t), "flag");
    P.workspace += (int64_t)(P.d_grid.bytes + P.d_points.bytes + P.d_mask.bytes + P.d_invalid.bytes + P.d_rows.bytes +
                             P.d_lm_segs[0].bytes + P.d_lm_segs[1].bytes +
                             P.d_bin_off.bytes + P.d_inst_K.bytes + P.d_flag.bytes);
}

// ------------------------------------------------------------ execution --

hipEvent_t take_event(nr_plan_s& P)
{
    if (!P.event_pool.empty()) {
        hipEvent_t e = P.event_pool.back();
        P.event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "event create");
    return e;
}

// Launch through f, bracketed by events when the plan profiles.
template <typename F>
void timed_launch(nr_plan_s& P, int stage, F&& f, const char* what)
{
    if (!P.opt.profile) {
        hip_check(f(), what);
        return;
    }
    hipEvent_t a = take_event(P), b = take_event(P);
    hip_check(hipEventRecord(a, P.stream), "event record");
    hip_check(f(), what);
    hip_check(hipEventRecord(b, P.stream), "event record");
    P.timed.push_back({stage, a, b});
}

SpreadArgs spread_args(const nr_plan_s& P, const Class& c, const Chunk& ch)
{
    SpreadArgs a{};
    a.inst = (const InstDev*)c.d_inst.p;
    a.coef = (const double*)c.d_coef.p;
    a.taps = c.d_taps.p;
    a.strain_lm = c.d_strain.p;
    a.phase_table = c.d_phase.p;
    a.points = (char*)P.d_points.p + c.pts_off;
    a.grid = (char*)P.d_grid.p + c.grid_off;
    a.first = ch.first;
    a.count = ch.count;
    a.pt_base = ch.pt_base;
    a.n = c.n;
    a.w = c.w;
    a.parts = c.parts;
    a.flush_period = c.flush_period;
    a.snap = c.snap;
    a.strain_complex = P.opt.strain_complex;
    a.epi_fused = c.fuse_epi;
    a.kmax = c.kmax;
    a.row_base = c.row_base;
    a.dec = c.d_dec.p;
    a.twiddle = c.d_tw.p;
    a.fft.n = c.n;
    a.fft.nr = (int32_t)c.radix.size();
    for (size_t r = 0; r < c.radix.size(); ++r) a.fft.radix[r] = c.radix[r];
    a.block_order = ch.order_off >= 0 ? (const int32_t*)c.d_order.p + ch.order_off : nullptr;
    return a;
}

EpilogueArgs epilogue_args(const nr_plan_s& P, const Class& c, const Chunk& ch)
{
    EpilogueArgs e{};
    e.inst = (const InstDev*)c.d_inst.p;
    e.grid = (const char*)P.d_grid.p + c.grid_off;
    e.dec = c.d_dec.p;
    e.twiddle = c.d_tw.p;
    e.fft.n = c.n;
    e.fft.nr = (int32_t)c.radix.size();
    for (size_t r = 0; r < c.radix.size(); ++r) e.fft.radix[r] = c.radix[r];
    e.first = ch.first;
    e.count = ch.count;
    e.tmpl_list = (const int32_t*)c.d_tmpl_list.p;
    e.tmpl_list_off = (const int64_t*)c.d_tmpl_list_off.p;
    e.tmpl_stat_off = (const int64_t*)c.d_tmpl_stat_off.p;
    e.tmpl_id = (const int32_t*)c.d_tmpl_id.p;
    e.tmpl_first = ch.tmpl_first;
    e.tmpl_count = ch.tmpl_count;
    e.slots = grid_slots(c.parts);
    e.kmax = c.kmax;
    e.row_base = c.row_base;
    e.entry_seg = (const int32_t*)c.d_entry_seg.p;
    return e;
}


void build_groups(nr_plan_s& P)
{
    // spread: same kernel instantiation and LDS tier
    std::map<std::array<int, 5>, size_t> sg;
    // epilogue groups: a segment sum adds into its templates' statistics
    // without atomics, so the classes of one group have disjoint templates
    std::map<std::array<int, 3>, std::vector<size_t>> eg;
    std::vector<std::vector<char>> eg_tmpls;
    for (size_t ci = 0; ci < P.classes.size(); ++ci) {
        const Class& c = *P.classes[ci];
        if (c.inst.empty()) continue;
        const int fused = spread_code(c.method);
        const int snap = (c.snap && !c.fp64 && c.deg <= 12) ? 1 : 0;
        // fused and separate-epilogue classes share launches (the flag is per
        // class in the launch table); their epilogue groups stay apart
        const size_t sl = spread_lds_bytes(c.fp64, c.n, c.fuse_epi && c.parts == 1);
        const std::array<int, 5> sk{c.fp64, c.deg, fused, snap, lds_tier(sl)};
        auto it = sg.find(sk);
        if (it != sg.end() && P.spread_groups[it->second].cls.size() >= (size_t)kGroupMax) {
            sg.erase(it);    // full: later classes of this kind start a new group
            it = sg.end();
        }
        if (it == sg.end()) {
            it = sg.emplace(sk, P.spread_groups.size()).first;
            P.spread_groups.emplace_back();
            Group& g = P.spread_groups.back();
            g.fp64 = c.fp64;
            g.deg = c.deg;
            g.fused = fused;
            g.snap = snap;
        }
        Group& g = P.spread_groups[it->second];
        g.cls.push_back((int)ci);
        g.lds[0] = std::max(g.lds[0], sl);
        const size_t el = epilogue_lds_bytes(c.fp64, c.n, c.kmax, 1);
        const std::array<int, 3> ek{c.fp64, lds_tier(el), c.fuse_epi};
        std::vector<size_t>& cand = eg[ek];
        size_t gi = SIZE_MAX;
        for (size_t q : cand) {
            if (P.epi_groups[q].cls.size() >= (size_t)kGroupMax) continue;
            bool clash = false;
            for (int32_t t : c.tmpl_id) clash = clash || eg_tmpls[q][t];
            if (!clash) {
                gi = q;
                break;
            }
        }
        if (gi == SIZE_MAX) {
            gi = P.epi_groups.size();
            cand.push_back(gi);
            P.epi_groups.emplace_back();
            P.epi_groups.back().fp64 = c.fp64;
            P.epi_groups.back().fuse_epi = c.fuse_epi;
            eg_tmpls.emplace_back((size_t)P.n_tmpls, (char)0);
        }
        for (int32_t t : c.tmpl_id) eg_tmpls[gi][t] = 1;
        Group& e = P.epi_groups[gi];
        e.cls.push_back((int)ci);
        e.lds[0] = std::max(e.lds[0], epilogue_lds_bytes(c.fp64, c.n, c.kmax, 0));
        e.lds[1] = std::max(e.lds[1], el);
    }
    for (Group& g : P.spread_groups) {
        int64_t off = 0;
        g.spread.ncls = (int32_t)g.cls.size();
        for (size_t q = 0; q < g.cls.size(); ++q) {
            const Class& c = *P.classes[g.cls[q]];
            g.spread.a[q] = spread_args(P, c, c.chunks[0]);
            g.spread.a[q].block_order = nullptr;     // grouped launches keep list order
            g.spread.block_off[q] = off;
            off += spread_blocks(c.chunks[0].count, c.parts);
        }
        g.blocks[0] = off;
    }
    for (Group& g : P.epi_groups) {
        int64_t off[2] = {0, 0};
        g.epi.ncls = (int32_t)g.cls.size();
        for (size_t q = 0; q < g.cls.size(); ++q) {
            const Class& c = *P.classes[g.cls[q]];
            g.epi.a[q] = epilogue_args(P, c, c.chunks[0]);
            for (int m = 0; m < 2; ++m) {
                g.epi.block_off[m][q] = off[m];
                off[m] += epilogue_blocks(g.epi.a[q], m);
            }
        }
        for (int m = 0; m < 2; ++m) g.blocks[m] = off[m];
    }
}

void check_finite(nr_plan_s& P, const void* strain)
{
    if (!P.opt.check_finite) return;
    int64_t total = 0;
    for (auto& g : P.segs) total = std::max(total, g.sample_offset + g.n_samples);
    if (P.opt.strain_complex) total *= 2;
    hip_check(hipMemsetAsync(P.d_flag.p, 0, sizeof(int32_t), P.stream), "flag reset");
    hip_check(launch_finite_scan(strain, total, P.strain_fp64, (int32_t*)P.d_flag.p, P.stream), "finite scan");
    int32_t flag = 0;
    hip_check(hipMemcpyAsync(&flag, P.d_flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, P.stream), "flag read");
    hip_check(hipStreamSynchronize(P.stream), "finite scan");
    if (flag) fail(NR_ERR_NONFINITE_INPUT, "strain contains NaN or Inf");
}

// tau (staged classes) and spreading of one chunk; out: the call's outputs
// for classes whose spreader runs the epilogue (out.mode 0: grids only).
void run_front(nr_plan_s& P, Class& c, const Chunk& ch, const EpilogueOut& out)
{
    SpreadArgs a = spread_args(P, c, ch);
    if (c.method == NR_METHOD_STAGED)
        timed_launch(P, NR_STAGE_TAU, [&] { return launch_tau(a, c.fp64, P.stream); }, "tau kernel");
    timed_launch(P, NR_STAGE_SPREAD,
                 [&] { return launch_spread(a, c.fp64, c.deg, spread_code(c.method), out, P.stream); },
                 "spread kernel");
}

// The call's outputs as the spreaders see them (mode: 0 grids, 1 power rows,
// 2 spectra / power).
EpilogueOut spread_out(const nr_plan_s& P, EpilogueOut out, int mode)
{
    out.mode = mode;
    out.out_fp64 = P.out_fp64;
    return out;
}

// Lane-major strain copies of every class (one launch per destination precision).
void lane_major(nr_plan_s& P, const void* strain)
{
    for (int f = 0; f < 2; ++f)
        if (!P.lm_segs[f].empty())
            timed_launch(P, NR_STAGE_LAYOUT, [&] {
                return launch_strain_lane_major((const SegDev*)P.d_lm_segs[f].p, (int32_t)P.lm_segs[f].size(),
                                                P.lm_max_entries[f], strain, P.strain_fp64, P.opt.strain_complex,
                                                f, P.stream);
            }, "strain layout");
}

// Side streams usable for k independent launch sequences (0 when profiling:
// the stage timers bracket launches on the plan's stream).
int side_count(const nr_plan_s& P, size_t k)
{
    if (P.opt.profile || P.side.empty() || k < 2) return 0;
    return (int)std::min(P.side.size(), k - 1);
}

void fork_side(nr_plan_s& P, int which, int n)
{
    if (n == 0) return;
    hip_check(hipEventRecord(P.ev_fork[which], P.stream), "fork");
    for (int i = 0; i < n; ++i) hip_check(hipStreamWaitEvent(P.side[i], P.ev_fork[which], 0), "fork");
}

void join_side(nr_plan_s& P, int which, int n)
{
    for (int i = 0; i < n; ++i) {
        hip_check(hipEventRecord(P.ev_join[which][i], P.side[i]), "join");
        hip_check(hipStreamWaitEvent(P.stream, P.ev_join[which][i], 0), "join");
    }
}

// Stream of the i-th of several independent sequences.
hipStream_t lane_stream(const nr_plan_s& P, size_t i, int n)
{
    const size_t r = i % (size_t)(n + 1);
    return r == 0 ? P.stream : P.side[r - 1];
}

// Batched mode: per spread group, the tau kernel of its staged classes and
// then one spread launch; independent groups run on side streams.
void run_front_batched(nr_plan_s& P, const EpilogueOut& out)
{
    const int ns = side_count(P, P.spread_groups.size());
    fork_side(P, 0, ns);
    for (size_t gi = 0; gi < P.spread_groups.size(); ++gi) {
        Group& g = P.spread_groups[gi];
        hipStream_t st = lane_stream(P, gi, ns);
        for (int ci : g.cls) {
            Class& c = *P.classes[ci];
            if (c.method != NR_METHOD_STAGED || c.chunks.empty()) continue;
            SpreadArgs a = spread_args(P, c, c.chunks[0]);
            timed_launch(P, NR_STAGE_TAU, [&] { return launch_tau(a, c.fp64, st); }, "tau kernel");
        }
        if (g.cls.size() == 1) {
            Class& c = *P.classes[g.cls[0]];
            SpreadArgs a = spread_args(P, c, c.chunks[0]);
            timed_launch(P, NR_STAGE_SPREAD, [&] { return launch_spread(a, c.fp64, c.deg, g.fused, out, st); },
                         "spread kernel");
            continue;
        }
        timed_launch(P, NR_STAGE_SPREAD, [&] {
            return launch_spread_multi(g.spread, g.blocks[0], g.fp64, g.deg, g.fused, P.opt.strain_complex, g.snap,
                                       g.lds[0], out, st);
        }, "spread kernel");
    }
    join_side(P, 0, ns);
}

// Batched mode: one epilogue launch per group (mode 0 spectra, 1 segment
// sum).  Spectra groups write disjoint bins and run side by side; segment
// sums of different groups may add into the same templates and stay in order.
void run_epilogue_batched(nr_plan_s& P, int mode, const EpilogueOut& out)
{
    // spectra / power rows of fused classes came out of their spreaders
    std::vector<size_t> todo;
    for (size_t gi = 0; gi < P.epi_groups.size(); ++gi)
        if (mode || !P.epi_groups[gi].fuse_epi) todo.push_back(gi);
    const int ns = mode ? 0 : side_count(P, todo.size());
    fork_side(P, 1, ns);
    for (size_t ti = 0; ti < todo.size(); ++ti) {
        Group& g = P.epi_groups[todo[ti]];
        hipStream_t st = lane_stream(P, ti, ns);
        if (g.cls.size() == 1) {
            Class& c = *P.classes[g.cls[0]];
            EpilogueArgs e = epilogue_args(P, c, c.chunks[0]);
            timed_launch(P, NR_STAGE_EPILOGUE, [&] {
                return mode ? launch_epilogue_sum(e, out, c.fp64, P.out_fp64, st)
                            : launch_epilogue_spectra(e, out, c.fp64, P.out_fp64, st);
            }, mode ? "segment sum" : "epilogue");
            continue;
        }
        timed_launch(P, NR_STAGE_EPILOGUE, [&] {
            return launch_epilogue_multi(g.epi, g.blocks[mode], mode, out, g.fp64, P.out_fp64, g.lds[mode], st);
        }, mode ? "segment sum" : "epilogue");
    }
    join_side(P, 1, ns);
}

void execute_launches(nr_plan_s& P, const void* strain, void* spectra, void* power, uint8_t* valid);

// Run enqueue() directly, or through a HIP graph captured on the first call
// with these pointer arguments and replayed afterwards.
template <typename F>
void run_graphed(nr_plan_s& P, int kind, std::initializer_list<const void*> args, F&& enqueue)
{
    const bool can = P.opt.use_graph && P.stream != nullptr && !P.opt.profile && !P.opt.check_finite;
    if (!can) {
        enqueue();
        return;
    }
    const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int k = 0;
    for (const void* a : args) key[k++] = a;
    for (auto& g : P.graphs)
        if (g.kind == kind && std::equal(key, key + 5, g.key)) {
            hip_check(hipGraphLaunch(g.exec, P.stream), "graph launch");
            return;
        }
    hip_check(hipStreamBeginCapture(P.stream, hipStreamCaptureModeRelaxed), "begin capture");
    hipGraph_t graph = nullptr;
    try {
        enqueue();
    } catch (...) {
        (void)hipStreamEndCapture(P.stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    hip_check(hipStreamEndCapture(P.stream, &graph), "end capture");
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e, "graph instantiate");
    if (P.graphs.size() >= 8) {
        (void)hipGraphExecDestroy(P.graphs.front().exec);
        P.graphs.erase(P.graphs.begin());
    }
    nr_plan_s::Graph g{kind, {}, exec};
    std::copy(key, key + 5, g.key);
    P.graphs.push_back(g);
    hip_check(hipGraphLaunch(exec, P.stream), "graph launch");
}

void execute(nr_plan_s& P, const void* strain, void* spectra, void* power, uint8_t* valid)
{
    if (!strain) fail(NR_ERR_INVALID_ARG, "strain is NULL");
    check_finite(P, strain);
    run_graphed(P, 0, {strain, spectra, power, valid}, [&] { execute_launches(P, strain, spectra, power, valid); });
}

void execute_launches(nr_plan_s& P, const void* strain, void* spectra, void* power, uint8_t* valid)
{
    EpilogueOut out{};
    out.spectra = spectra;
    out.power = power;
    lane_major(P, strain);
    const EpilogueOut sout = spread_out(P, out, 2);
    if (P.batched) {
        if (spectra || power) {
            run_front_batched(P, sout);
            run_epilogue_batched(P, 0, out);
        }
    } else {
        for (auto& cp : P.classes) {
            Class& c = *cp;
            for (const Chunk& ch : c.chunks) {
                EpilogueArgs e = epilogue_args(P, c, ch);
                if (c.method == NR_METHOD_DIRECT) {
                    SpreadArgs a = spread_args(P, c, ch);
                    if (spectra || power)
                        timed_launch(P, NR_STAGE_SPREAD, [&] {
                            return launch_direct(a, e, out, 0, c.fp64, P.out_fp64, P.stream);
                        }, "direct sum");
                    continue;
                }
                if (!(spectra || power)) continue;
                run_front(P, c, ch, sout);
                if (!c.fuse_epi)
                    timed_launch(P, NR_STAGE_EPILOGUE,
                                 [&] { return launch_epilogue_spectra(e, out, c.fp64, P.out_fp64, P.stream); },
                                 "epilogue");
            }
        }
    }
    if (spectra || power || valid)
        timed_launch(P, NR_STAGE_EPILOGUE, [&] {
            return launch_fill_invalid((const int32_t*)P.d_invalid.p, (const int64_t*)P.d_bin_off.p,
                                       (const int32_t*)P.d_inst_K.p, (spectra || power) ? P.n_invalid : 0,
                                       spectra, power, P.out_fp64, (const uint8_t*)P.d_mask.p, valid,
                                       P.n_inst, P.stream);
        }, "invalid fill");
}

void semicoherent_launches(nr_plan_s& P, const void* strain, const double* w, void* stat, int32_t* n_used);

void semicoherent(nr_plan_s& P, const void* strain, const double* w, void* stat, int32_t* n_used)
{
    if (!strain || !stat) fail(NR_ERR_INVALID_ARG, "strain and stat must not be NULL");
    check_finite(P, strain);
    run_graphed(P, 1, {strain, w, stat, n_used}, [&] { semicoherent_launches(P, strain, w, stat, n_used); });
}

void semicoherent_launches(nr_plan_s& P, const void* strain, const double* w, void* stat, int32_t* n_used)
{
    EpilogueOut out{};
    out.seg_weight = w;
    out.stat = stat;
    out.n_used = n_used;
    lane_major(P, strain);
    if (P.two_pass) {
        // first pass: power rows (spectra-mode epilogue); second: row sums
        EpilogueOut rows{};
        rows.rows = P.d_rows.p;
        out.rows = P.d_rows.p;
        const EpilogueOut srows = spread_out(P, rows, 1);
        if (P.batched) {
            run_front_batched(P, srows);
            run_epilogue_batched(P, 0, rows);
            for (Group& g : P.epi_groups) {
                if (g.cls.size() == 1) {
                    Class& c = *P.classes[g.cls[0]];
                    EpilogueArgs e = epilogue_args(P, c, c.chunks[0]);
                    timed_launch(P, NR_STAGE_EPILOGUE, [&] { return launch_rows_sum(e, out, P.out_fp64, P.stream); },
                                 "segment sum");
                    continue;
                }
                timed_launch(P, NR_STAGE_EPILOGUE, [&] {
                    return launch_rows_sum_multi(g.epi, g.blocks[1], out, P.out_fp64, P.stream);
                }, "segment sum");
            }
            return;
        }
        for (auto& cp : P.classes) {
            Class& c = *cp;
            for (const Chunk& ch : c.chunks) {
                EpilogueArgs e = epilogue_args(P, c, ch);
                if (c.method == NR_METHOD_DIRECT) {
                    SpreadArgs a = spread_args(P, c, ch);
                    timed_launch(P, NR_STAGE_SPREAD, [&] {
                        return launch_direct(a, e, rows, 1, c.fp64, P.out_fp64, P.stream);
                    }, "direct sum");
                } else {
                    run_front(P, c, ch, srows);
                    if (!c.fuse_epi)
                        timed_launch(P, NR_STAGE_EPILOGUE,
                                     [&] { return launch_epilogue_spectra(e, rows, c.fp64, P.out_fp64, P.stream); },
                                     "epilogue");
                }
                timed_launch(P, NR_STAGE_EPILOGUE, [&] { return launch_rows_sum(e, out, P.out_fp64, P.stream); },
                             "segment sum");
            }
        }
        return;
    }
    const EpilogueOut sgrid = spread_out(P, out, 0);
    if (P.batched) {
        run_front_batched(P, sgrid);
        run_epilogue_batched(P, 1, out);
        return;
    }
    for (auto& cp : P.classes) {
        Class& c = *cp;
        for (const Chunk& ch : c.chunks) {
            run_front(P, c, ch, sgrid);
            EpilogueArgs e = epilogue_args(P, c, ch);
            timed_launch(P, NR_STAGE_EPILOGUE,
                         [&] { return launch_epilogue_sum(e, out, c.fp64, P.out_fp64, P.stream); }, "segment sum");
        }
    }
}

// Time one spreader configuration on a synthetic batch of identical instances.
double time_config(const nr_options& base, const nr_segment& g, const nr_template& t, double tol, int fp64,
                   int method, int parts, int flush, int snap, const void* strain, void* stat, int32_t* used,
                   int64_t batch)
{
    nr_options o2 = base;
    o2.tune = 0;
    o2.tune_cache = nullptr;
    o2.parts = parts;
    o2.flush_period = flush;
    o2.moment_mode = snap ? 2 : 1;
    o2.method = method;
    o2.precision = fp64 ? NR_FP64 : NR_FP32;
    o2.profile = 0;
    o2.use_graph = 0;
    o2.check_finite = 0;
    o2.strain_length = 0;
    o2.max_workspace_bytes = 0;
    nr_segment s1 = g;
    s1.sample_offset = 0;
    std::vector<nr_instance> il((size_t)batch, nr_instance{0, 0, tol});
    nr_plan_s mini;
    mini.opt = o2;
    create_plan(mini, &s1, 1, &t, 1, il.data(), batch, tol);
    semicoherent(mini, strain, nullptr, stat, used);  // warm-up
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "event");
    hip_check(hipEventCreate(&b), "event");
    hip_check(hipEventRecord(a, mini.stream), "event");
    for (int r = 0; r < 3; ++r) semicoherent(mini, strain, nullptr, stat, used);
    hip_check(hipEventRecord(b, mini.stream), "event");
    hip_check(hipEventSynchronize(b), "event");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, a, b), "event");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return 1e3 * ms / 3.0 / (double)batch;
}

// Grid size the plan gives this template's instances.
int fft_size_of_template(const nr_template& t, const nr_segment& g, double sigma_opt, double tol, int fp64)
{
    (void)g;
    const double sigma = sigma_opt > 0.0 ? sigma_opt : 2.0;
    const int w = kernel_width(std::max(tol, fp64 ? kFp64MinTol : kFp32MinTol), sigma);
    return fft_size(std::max((int64_t)std::ceil(sigma * t.n_bins - 1e-9), (int64_t)2 * w));
}

// Epilogue time per instance (microseconds) of one radix plan, with the
// separate epilogue kernel and the given spreader configuration.
double time_fft_plan(const nr_options& base, const nr_segment& g, const nr_template& t, double tol, int fp64,
                     const Tuned& cfg, int radix, const void* strain, void* stat, int32_t* used, int64_t batch)
{
    nr_options o2 = base;
    o2.tune = 0;
    o2.tune_cache = nullptr;
    o2.parts = cfg.parts;
    o2.flush_period = cfg.flush;
    o2.moment_mode = cfg.snap ? 2 : 1;
    o2.method = cfg.method;
    o2.precision = fp64 ? NR_FP64 : NR_FP32;
    o2.profile = 1;
    o2.use_graph = 0;
    o2.check_finite = 0;
    o2.strain_length = 0;
    o2.max_workspace_bytes = 0;
    o2.epilogue = 1;
    nr_segment s1 = g;
    s1.sample_offset = 0;
    std::vector<nr_instance> il((size_t)batch, nr_instance{0, 0, tol});
    nr_plan_s mini;
    mini.opt = o2;
    mini.radix_override = radix;
    create_plan(mini, &s1, 1, &t, 1, il.data(), batch, tol);
    semicoherent(mini, strain, nullptr, stat, used);  // warm-up
    nr_stage_times st{};
    nufft_resample_stage_times(&mini, &st);
    for (int r = 0; r < 3; ++r) semicoherent(mini, strain, nullptr, stat, used);
    nufft_resample_stage_times(&mini, &st);
    return 1e3 * st.ms[NR_STAGE_EPILOGUE] / 3.0 / (double)batch;
}

// small_batch > 0: the shape's instances in a plan too small to fill the GPU;
// the mini-plans then hold that many and keep the automatic waves per
// instance (which spread small plans over more waves), so that the timings
// reflect that plan's latency rather than a full GPU's throughput.
Tuned tune_shape(const nr_options& base, const nr_segment& g, const nr_template& t, double tol, int fp64,
                 int64_t small_batch)
{
    const int64_t L = g.n_samples;
    int64_t batch = (int64_t(1) << 25) / std::max<int64_t>(L, 1);
    batch = std::min<int64_t>(4096, std::max<int64_t>(256, batch));
    if (small_batch > 0) batch = std::min<int64_t>(small_batch, 4096);
    // synthetic N(0,1) strain (values do not change the cost)
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd;
    DevBuf strain, stat, used;
    if (fp64) {
        std::vector<double> h((size_t)L);
        for (auto& v : h) v = nd(rng);
        strain.upload(h, "tuning strain");
    } else {
        std::vector<float> h((size_t)L);
        for (auto& v : h) v = (float)nd(rng);
        strain.upload(h, "tuning strain");
    }
    stat.alloc((size_t)t.n_bins * 8, "tuning output");
    used.alloc(sizeof(int32_t), "tuning output");
    hip_check(hipMemset(stat.p, 0, (size_t)t.n_bins * 8), "tuning output");
    Tuned best{NR_METHOD_FUSED, default_parts(L), 0, 0, INFINITY, 0};
    for (int method : {NR_METHOD_FUSED, NR_METHOD_STAGED, NR_METHOD_CELLRUN})
        for (int parts : {1, 2, 4, 0}) {
            if ((parts == 0) != (small_batch > 0)) continue;   // 0: automatic, small plans only
            if (parts > 1 && L < (int64_t)kWave * parts * 16) continue;
            for (int flush : {4, 16, 64})
                for (int snap : {0, 1}) {
                    if (snap && fp64) continue;  // cumulative snapshots are an FP32-class option
                    // cell runs flush once per run and restart their moments
                    if (method == NR_METHOD_CELLRUN && (flush != 16 || snap)) continue;
                    const double us = time_config(base, g, t, tol, fp64, method, parts, flush, snap, strain.p,
                                                  stat.p, (int32_t*)used.p, batch);
                    if (us < best.us_per_inst) best = Tuned{method, parts, flush, snap, us, 0};
                }
        }
    // FFT radix plan: the epilogue alone, timed for every candidate order
    const std::vector<std::vector<int>> cand = fft_radix_candidates(fft_size_of_template(t, g, base.sigma, tol, fp64));
    double best_fft = INFINITY;
    for (const std::vector<int>& r : cand) {
        const double us = time_fft_plan(base, g, t, tol, fp64, best, radix_code(r), strain.p, stat.p,
                                        (int32_t*)used.p, batch);
        if (us < best_fft) {
            best_fft = us;
            best.radix = r == cand[0] ? 0 : radix_code(r);
        }
    }
    return best;
}

Tuned tuned_config(const nr_options& base, const nr_segment& g, const nr_template& t, double tol, int fp64,
                   int w, int n, int64_t small_batch)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    load_tune_cache(base.tune_cache);
    const ShapeKey key{fp64, w, n, g.n_samples, small_batch};
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
    const Tuned tu = tune_shape(base, g, t, tol, fp64, small_batch);
    g_tuned[key] = tu;
    save_tune_cache(base.tune_cache);
    return tu;
}

template <typename F>
nr_status guarded(nr_plan_s* P, F&& f)
{
    try {
        f();
        if (P) P->err.clear();
        return NR_OK;
    } catch (const NrError& e) {
        if (P) P->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        if (P) P->err = "host allocation failed";
        return NR_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        if (P) P->err = e.what();
        return NR_ERR_DEVICE;
    }
}

}  // namespace

namespace nr {

nr_status report_create_error(nr_status code, const std::string& msg)
{
    g_create_error = msg;
    return code;
}

nr_status semicoherent_sum_in_arena(void* base, size_t bytes, const nr_segment* segs, int32_t n_segs,
                                    const nr_template* tmpls, int32_t n_tmpls, const nr_instance* inst,
                                    int64_t n_inst, double tol, const nr_options* opt, const void* strain,
                                    const double* seg_weight, void* stat, int32_t* n_used)
{
    nr_options o;
    if (opt)
        o = *opt;
    else
        nufft_resample_default_options(&o);
    if (o.profile || o.use_graph || o.tune) {
        g_create_error = "profile, use_graph and tune need device allocations: they must be 0 here";
        return NR_ERR_INVALID_ARG;
    }
    if (!base || bytes < 4096) {
        g_create_error = "no static scratch";
        return NR_ERR_DEVICE;
    }
    // grids, point stream and power rows within half the scratch; the tables
    // and the lane-major strain take the rest
    const int64_t budget = (int64_t)(bytes / 2);
    o.max_workspace_bytes = o.max_workspace_bytes > 0 ? std::min<int64_t>(o.max_workspace_bytes, budget) : budget;
    const hipStream_t st = (hipStream_t)o.stream;
    // a previous call on this stream may still read the scratch
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        g_create_error = std::string("stream synchronisation: ") + hipGetErrorString(e);
        return NR_ERR_DEVICE;
    }
    std::unique_ptr<nr_plan_s> P;
    try {
        P.reset(new nr_plan_s());
    } catch (...) {
        g_create_error = "host allocation failed";
        return NR_ERR_OUT_OF_MEMORY;
    }
    P->opt = o;
    Arena arena{static_cast<char*>(base), bytes, 0};
    g_arena = &arena;
    nr_status s = guarded(P.get(), [&] { create_plan(*P, segs, n_segs, tmpls, n_tmpls, inst, n_inst, tol); });
    g_arena = nullptr;
    if (s == NR_OK) s = guarded(P.get(), [&] { semicoherent(*P, strain, seg_weight, stat, n_used); });
    if (s != NR_OK) g_create_error = P->err;
    // the sum reads the scratch: finish before it can be reused
    e = hipStreamSynchronize(st);
    if (s == NR_OK && e != hipSuccess) {
        g_create_error = std::string("segment sum: ") + hipGetErrorString(e);
        s = NR_ERR_DEVICE;
    }
    return s;
}

}  // namespace nr

extern "C" {

void nufft_resample_default_options(nr_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = NR_FP32;
    opt->method = NR_METHOD_AUTO;
    opt->sigma = 2.0;
}

nr_status nufft_resample_plan(nr_plan* out, const nr_segment* segs, int32_t n_segs,
                              const nr_template* tmpls, int32_t n_tmpls, const nr_instance* inst,
                              int64_t n_inst, double tol, const nr_options* opt)
{
    if (!out) {
        g_create_error = "out is NULL";
        return NR_ERR_INVALID_ARG;
    }
    *out = nullptr;
    nr_plan_s* P = nullptr;
    try {
        P = new nr_plan_s();
    } catch (...) {
        g_create_error = "host allocation failed";
        return NR_ERR_OUT_OF_MEMORY;
    }
    if (opt)
        P->opt = *opt;
    else
        nufft_resample_default_options(&P->opt);
    nr_status st = guarded(P, [&] { create_plan(*P, segs, n_segs, tmpls, n_tmpls, inst, n_inst, tol); });
    if (st != NR_OK) {
        g_create_error = P->err;
        delete P;
        return st;
    }
    *out = P;
    return NR_OK;
}

nr_status nufft_resample_execute(nr_plan p, const void* strain, void* spectra, void* power,
                                 uint8_t* valid)
{
    if (!p) return NR_ERR_INVALID_ARG;
    return guarded(p, [&] { execute(*p, strain, spectra, power, valid); });
}

nr_status nufft_resample_semicoherent_sum(nr_plan p, const void* strain, const double* seg_weight,
                                          void* stat, int32_t* n_used)
{
    if (!p) return NR_ERR_INVALID_ARG;
    return guarded(p, [&] { semicoherent(*p, strain, seg_weight, stat, n_used); });
}

nr_status nufft_resample_stage_times(nr_plan p, nr_stage_times* out)
{
    if (!p || !out) return NR_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    return guarded(p, [&] {
        for (auto& t : p->timed) {
            hip_check(hipEventSynchronize(t.b), "event sync");
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, t.a, t.b), "event time");
            out->ms[t.stage] += ms;
            out->launches[t.stage] += 1;
            p->event_pool.push_back(t.a);
            p->event_pool.push_back(t.b);
        }
        p->timed.clear();
    });
}

nr_status nufft_resample_query(nr_plan p, nr_plan_info* info)
{
    if (!p || !info) return NR_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_inst = p->n_inst;
    info->n_valid = p->n_valid;
    info->total_bins = p->bin_off.back();
    info->stat_bins = p->stat_off.back();
    info->valid_points = p->valid_points;
    info->workspace_bytes = p->workspace;
    info->n_classes = (int32_t)p->classes.size();
    info->out_fp64 = p->out_fp64;
    info->method = p->method;
    info->n_chunks = p->n_chunks;
    return NR_OK;
}

nr_status nufft_resample_query_class(nr_plan p, int32_t ci, nr_class_info* info)
{
    if (!p || !info || ci < 0 || ci >= (int32_t)p->classes.size()) {
        if (p) p->err = "class index out of range";
        return NR_ERR_INVALID_ARG;
    }
    const Class& c = *p->classes[ci];
    std::memset(info, 0, sizeof(*info));
    info->fp64 = c.fp64;
    info->w = c.w;
    info->n = c.n;
    info->degree = c.deg;
    info->parts = c.parts;
    info->n_radix = (int32_t)c.radix.size();
    for (size_t r = 0; r < c.radix.size() && r < 8; ++r) info->radix[r] = c.radix[r];
    info->beta_es = c.beta_es;
    info->method = c.method;
    info->flush_period = c.flush_period;
    info->snap = c.snap;
    info->epi_fused = c.fuse_epi;
    info->n_inst = (int64_t)c.inst.size();
    info->n_points = c.n_points;
    for (const InstDev& d : c.inst) {
        if (d.ndeg > 0) info->series_terms += (int64_t)d.L * d.ndeg;
        if (d.ndeg < 0) info->fallback_points += d.L;
    }
    return NR_OK;
}

nr_status nufft_resample_bin_offsets(nr_plan p, int64_t* offsets)
{
    if (!p || !offsets) return NR_ERR_INVALID_ARG;
    std::memcpy(offsets, p->bin_off.data(), p->bin_off.size() * sizeof(int64_t));
    return NR_OK;
}

nr_status nufft_resample_stat_offsets(nr_plan p, int64_t* offsets)
{
    if (!p || !offsets) return NR_ERR_INVALID_ARG;
    std::memcpy(offsets, p->stat_off.data(), p->stat_off.size() * sizeof(int64_t));
    return NR_OK;
}

nr_status nufft_resample_valid_mask(nr_plan p, uint8_t* valid)
{
    if (!p || !valid) return NR_ERR_INVALID_ARG;
    std::memcpy(valid, p->valid.data(), p->valid.size());
    return NR_OK;
}

nr_status nufft_resample_kernel_params(double tol, double sigma, int32_t precision, int32_t n_bins,
                                       nr_class_info* info)
{
    if (!info || !(tol > 0.0 && tol <= 0.1) || n_bins < 1 || precision < NR_FP32 || precision > NR_AUTO ||
        (sigma > 0.0 && !(sigma >= 1.25 && sigma <= 4.0))) {
        g_create_error = "invalid kernel parameter query";
        return NR_ERR_INVALID_ARG;
    }
    if (sigma <= 0.0) sigma = 2.0;
    std::memset(info, 0, sizeof(*info));
    const int fp64 = precision == NR_FP64 || (precision == NR_AUTO && tol < kFp32MinTol);
    const double tol_eff = std::max(tol, fp64 ? kFp64MinTol : kFp32MinTol);
    info->fp64 = fp64;
    info->w = kernel_width(tol_eff, sigma);
    info->beta_es = es_beta(info->w, sigma);
    info->n = fft_size(std::max((long long)std::ceil(sigma * n_bins - 1e-9), (long long)2 * info->w));
    std::vector<long double> taps;
    info->degree = kernel_pieces(info->w, info->beta_es, tol_eff, kMaxDeg, taps);
    const std::vector<int> r = fft_radices(info->n);
    info->n_radix = (int32_t)r.size();
    for (size_t k = 0; k < r.size() && k < 8; ++k) info->radix[k] = r[k];
    info->parts = 1;
    return NR_OK;
}

double nufft_resample_kernel_ft(int32_t w, double beta_es, double xi)
{
    if (w < 2 || w > 16 || !(beta_es > 0.0)) return NAN;
    return (double)es_fourier(w, beta_es, (long double)xi);
}

double nufft_resample_chirp_beta(double mc_msun, double f0)
{
    if (!(mc_msun >= 0.0) || !(f0 > 0.0)) return NAN;
    return chirp_beta(mc_msun, f0);
}

const char* nufft_resample_last_error(nr_plan p)
{
    return p ? p->err.c_str() : g_create_error.c_str();
}

void nufft_resample_destroy(nr_plan p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    delete p;
}

}  // extern "C"
