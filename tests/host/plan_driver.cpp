// Host driver for the address / undefined-behaviour sanitizer build of the
// plan code (csrc/nr_plan.cpp, host parts instrumented): plans the 1 h
// semicoherent workload (120 segments x 64 chirp masses x 20 sub-bands) and
// asks for kernel parameters.  Without a GPU the plan stops at its first
// device allocation with NR_ERR_OUT_OF_MEMORY after validating and building
// every instance's constants and every class's tables; with one it runs to the
// end.  Exit status 0 unless an unexpected status comes back.
#include <cstdio>
#include <vector>
#include "nufft_resample.h"
int main() {
    std::vector<nr_segment> segs(120);
    for (int i = 0; i < 120; ++i) segs[i] = {(int64_t)i * 7680, 7680, 256.0, 30.0 * i};
    std::vector<nr_template> t(64 * 20);
    for (int m = 0; m < 64; ++m) for (int b = 0; b < 20; ++b) {
        nr_template& q = t[m * 20 + b];
        q.mc_msun = 5e-4 * __builtin_pow(200.0, m / 63.0); q.f0 = 40.5 + b; q.f_lo = 40 + b; q.df = 1.0 / 30; q.n_bins = 30; q.reserved = 0; q.f_max = 60;
    }
    nr_options o; nufft_resample_default_options(&o);
    nr_plan p = nullptr;
    nr_status s = nufft_resample_plan(&p, segs.data(), 120, t.data(), (int)t.size(), nullptr, 0, 1e-6, &o);
    std::printf("plan status %d: %s\n", (int)s, s == NR_OK ? "" : nufft_resample_last_error(nullptr));
    int bad = (s != NR_OK && s != NR_ERR_OUT_OF_MEMORY && s != NR_ERR_DEVICE);
    nr_class_info ci;
    for (double tol : {1e-2, 1e-6, 1e-9})
        bad += nufft_resample_kernel_params(tol, 2.0, NR_AUTO, 600, &ci) != NR_OK;
    // rejected arguments
    bad += nufft_resample_plan(&p, segs.data(), 0, t.data(), 1, nullptr, 0, 1e-6, &o) != NR_ERR_INVALID_ARG;
    o.sigma = 9.0;
    bad += nufft_resample_plan(&p, segs.data(), 1, t.data(), 1, nullptr, 0, 1e-6, &o) != NR_ERR_INVALID_ARG;
    if (p) nufft_resample_destroy(p);
    std::printf("%d unexpected statuses\n", bad);
    return bad ? 1 : 0;
}
