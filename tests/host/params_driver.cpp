// Host driver for the address / undefined-behaviour sanitizer build of the
// plan's parameter code (csrc/nr_params.cpp): every function over its domain
// and past its edges.  Prints one line per check group; exits non-zero on a
// failed check.
#include <cmath>
#include <cstdio>
#include <vector>

#include "nr_params.hpp"

int main()
{
    int bad = 0;
    for (double tol : {1e-1, 1e-2, 1e-3, 1e-6, 1e-9, 1e-12, 1e-15}) {
        for (double sigma : {1.25, 2.0, 3.0, 4.0}) {
            const int w = nr::kernel_width(tol, sigma);
            if (w < 2 || w > 16) ++bad;
            const double b = nr::es_beta(w, sigma);
            std::vector<long double> pieces;
            const int deg = nr::kernel_pieces(w, b, tol, 18, pieces);
            if (deg < 1 || deg > 18 || pieces.size() != (size_t)w * (deg + 1)) ++bad;
            const long double ft = nr::es_fourier(w, b, 0.5L);
            if (!(ft > 0.0L) || !std::isfinite((double)ft)) ++bad;
        }
    }
    std::printf("widths and pieces: %d failures\n", bad);
    for (long long m : {1LL, 2LL, 7LL, 60LL, 61LL, 1199LL, 4801LL, 65537LL}) {
        const int n = nr::fft_size(m);
        std::vector<int> r = nr::fft_radices(n);
        long long prod = 1;
        for (int q : r) prod *= q;
        if (n < m || prod != n) ++bad;
    }
    std::printf("fft sizes: %d failures\n", bad);
    for (double mc : {0.0, 1e-6, 5e-4, 1e-1, 10.0})
        for (double f0 : {1.0, 50.0, 2000.0}) {
            const double b = nr::chirp_beta(mc, f0);
            if (!(b >= 0.0) || !std::isfinite(b)) ++bad;
        }
    for (double z : {-2.0, -1.0, 0.0, 0.5, 1.0, 2.0})
        if (!std::isfinite((double)nr::es_value(23.0, z))) ++bad;
    std::printf("beta and kernel values: %d failures\n", bad);
    return bad ? 1 : 0;
}
