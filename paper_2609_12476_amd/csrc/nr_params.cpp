// Host-side NUFFT and resampling parameters.
#include "nr_params.hpp"

#include <algorithm>
#include <functional>
#include <cmath>
#include <vector>

namespace nr {

namespace {
const long double kPi = 3.14159265358979323846264338327950288L;

// Calibrated relative l2 error of the ES kernel at sigma = 2 with
// beta = 2.30 w, w = 2..16: the worst over K = 30, 600 and 2400 modes and
// three draws of random points and strengths of a plain FP64 NUFFT with exact
// kernel values against the direct sums, times 1.25 and rounded up to two
// digits (written by paper_2609_12476_amd/calibrate_es.py, seed 0).
const double kErrSigma2[17] = {1.0,    1.0,    9.0e-2, 1.1e-2, 9.9e-4, 1.8e-4,
                               1.6e-5, 1.5e-6, 1.4e-7, 1.7e-8, 3.2e-9, 3.1e-10,
                               3.3e-11, 2.3e-12, 4.0e-13, 3.0e-13, 3.0e-13};

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_N.
void gauss_legendre(int N, std::vector<long double>& x, std::vector<long double>& w)
{
    x.resize(N);
    w.resize(N);
    for (int i = 0; i < N; ++i) {
        long double z = cosl(kPi * (i + 0.75L) / (N + 0.5L));
        long double dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= N; ++k) {
                const long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = N * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}
}  // namespace

double chirp_beta(double mc_msun, double f0)
{
    if (mc_msun == 0.0) return 0.0;
    // GM_sun / c^3 from the IAU 2015 nominal GM_sun and the exact speed of light.
    const long double c = 299792458.0L;
    const long double t_sun = 1.3271244e20L / (c * c * c);
    return (double)((96.0L / 5.0L) * powl(kPi, 8.0L / 3.0L) * powl(t_sun * mc_msun, 5.0L / 3.0L) *
                    powl((long double)f0, 8.0L / 3.0L));
}

double kernel_error(int w, double sigma)
{
    if (w < 2) return 1.0;
    if (std::fabs(sigma - 2.0) < 1e-12 && w <= 16) return kErrSigma2[w];
    // exp(-pi w sqrt(1 - 1/sigma)) with a safety factor 10
    return 10.0 * std::exp(-M_PI * w * std::sqrt(1.0 - 1.0 / sigma));
}

int kernel_width(double tol, double sigma)
{
    for (int w = 2; w <= 16; ++w)
        if (kernel_error(w, sigma) <= 0.5 * tol) return w;
    return 16;
}

double es_beta(int w, double sigma)
{
    // 2.30 w at sigma = 2, scaled with the usable fraction 1 - 1/(2 sigma)
    return 2.30 * w * (1.0 - 1.0 / (2.0 * sigma)) / 0.75;
}

long double es_value(double beta, long double z)
{
    if (fabsl(z) > 1.0L) return 0.0L;
    return expl((long double)beta * (sqrtl(1.0L - z * z) - 1.0L));
}

long double es_fourier(int w, double beta, long double xi)
{
    // With z = sin(theta) the integrand exp(beta (cos theta - 1)) cos(xi h sin theta) cos theta
    // is smooth on [-pi/2, pi/2], so Gauss-Legendre converges geometrically.
    static thread_local std::vector<long double> gx, gw;
    if (gx.empty()) gauss_legendre(160, gx, gw);
    const long double h = 0.5L * w;
    long double s = 0.0L;
    for (size_t i = 0; i < gx.size(); ++i) {
        const long double th = 0.5L * kPi * gx[i];
        const long double ct = cosl(th);
        s += gw[i] * expl((long double)beta * (ct - 1.0L)) * cosl(xi * h * sinl(th)) * ct;
    }
    return h * 0.5L * kPi * s;
}

int kernel_pieces(int w, double beta, double tol, int max_deg, std::vector<long double>& out)
{
    const int N = 96;  // Chebyshev interpolation nodes per piece
    const long double h = 0.5L * w;
    std::vector<long double> coef((size_t)w * N);
    for (int t = 0; t < w; ++t) {
        std::vector<long double> f(N);
        for (int k = 0; k < N; ++k) {
            const long double u = cosl(kPi * (k + 0.5L) / N);
            const long double fr = 0.5L * (u + 1.0L);
            f[k] = es_value(beta, (t + fr - h) / h);
        }
        for (int p = 0; p < N; ++p) {
            long double s = 0.0L;
            for (int k = 0; k < N; ++k) s += f[k] * cosl(p * kPi * (k + 0.5L) / N);
            coef[(size_t)t * N + p] = (p == 0 ? 1.0L : 2.0L) * s / N;
        }
    }
    const int M = 257;
    const long double target = tol / 20.0;
    int best_deg = max_deg;
    long double best_err = INFINITY;
    for (int D = 2; D <= max_deg; ++D) {
        long double err = 0.0L;
        for (int t = 0; t < w; ++t) {
            for (int i = 0; i < M; ++i) {
                const long double fr = (long double)i / (M - 1);
                const long double u = 2.0L * fr - 1.0L;
                long double t0 = 1.0L, t1 = u, v = coef[(size_t)t * N] + coef[(size_t)t * N + 1] * u;
                for (int p = 2; p <= D; ++p) {
                    const long double t2 = 2.0L * u * t1 - t0;
                    v += coef[(size_t)t * N + p] * t2;
                    t0 = t1;
                    t1 = t2;
                }
                // the exact piece on the closed interval; its end values at
                // fr = 0 (t = 0) and fr = 1 (t = w-1) touch the support edge
                const long double ex = es_value(beta, (t + fr - h) / h);
                err = std::max(err, fabsl(v - ex));
            }
        }
        if (err < best_err) {
            best_err = err;
            best_deg = D;
        }
        if (err <= target) {
            best_deg = D;
            break;
        }
    }
    out.assign((size_t)w * (best_deg + 1), 0.0L);
    for (int t = 0; t < w; ++t)
        for (int p = 0; p <= best_deg; ++p) out[(size_t)t * (best_deg + 1) + p] = coef[(size_t)t * N + p];
    return best_deg;
}

int fft_size(long long m)
{
    if (m < 1) m = 1;
    for (long long n = m;; ++n) {
        long long r = n;
        for (int p : {2, 3, 5})
            while (r % p == 0) r /= p;
        if (r == 1) return (int)n;
    }
}

std::vector<int> fft_radices(int n)
{
    std::vector<int> r;
    while (n % 4 == 0) {
        r.push_back(4);
        n /= 4;
    }
    if (n % 2 == 0) {
        r.push_back(2);
        n /= 2;
    }
    while (n % 3 == 0) {
        r.push_back(3);
        n /= 3;
    }
    while (n % 5 == 0) {
        r.push_back(5);
        n /= 5;
    }
    return r;
}

std::vector<std::vector<int>> fft_radix_candidates(int n)
{
    const std::vector<int> d = fft_radices(n);
    std::vector<std::vector<int>> c{d};
    c.emplace_back(d.rbegin(), d.rend());
    std::vector<int> s = d;
    std::sort(s.begin(), s.end(), std::greater<int>());
    c.push_back(s);
    std::sort(s.begin(), s.end());
    c.push_back(s);
    std::vector<int> twos;
    for (int q : d) {
        if (q == 4) {
            twos.push_back(2);
            twos.push_back(2);
        } else {
            twos.push_back(q);
        }
    }
    c.push_back(twos);
    std::vector<std::vector<int>> out;
    for (auto& r : c)
        if (r.size() <= 8 && std::find(out.begin(), out.end(), r) == out.end()) out.push_back(r);
    return out;
}

int radix_code(const std::vector<int>& r)
{
    int code = 0;
    for (int q : r) code = code * 10 + q;
    return code;
}

std::vector<int> radix_from_code(int code)
{
    std::vector<int> r;
    for (; code > 0; code /= 10) r.insert(r.begin(), code % 10);
    return r;
}

}  // namespace nr
