// Host-side NUFFT and resampling parameters (no device code).
#pragma once

#include <cstddef>
#include <vector>

namespace nr {

constexpr double kFp32MinTol = 1e-6;   // FP32 spreading/FFT reach about 1e-6 relative l2
constexpr double kFp64MinTol = 1e-12;  // below this the kernel width table ends
// LDS of one gfx950 workgroup; the spreader's four per-wave grid copies and
// its phase table must fit, which bounds the upsampled grid size.
constexpr size_t kLdsBytes = 160 * 1024;

// beta(f0, Mc) of Eq. (beta) in s^-1 (0 for Mc = 0).
double chirp_beta(double mc_msun, double f0);

// Smallest ES kernel width whose calibrated relative error is <= tol / 2.
int kernel_width(double tol, double sigma);

// ES shape parameter for width w at upsampling sigma.
double es_beta(int w, double sigma);

// Upper bound on the relative l2 error of width w at upsampling sigma.
double kernel_error(int w, double sigma);

// Chebyshev coefficients of the w kernel pieces psi((t + fr - w/2)/(w/2)),
// fr in [0, 1], t = 0..w-1, in the variable u = 2 fr - 1, truncated at the
// smallest degree whose sup error is <= tol / 20 (at most max_deg).
// Returns the degree; out holds w * (degree + 1) coefficients, tap-major.
int kernel_pieces(int w, double beta, double tol, int max_deg, std::vector<long double>& out);

// Fourier transform of the ES kernel of width w (grid units):
//   psi_hat(xi) = int_{-w/2}^{w/2} exp(beta (sqrt(1 - (2x/w)^2) - 1)) cos(xi x) dx.
long double es_fourier(int w, double beta, long double xi);

// ES kernel value at z in [-1, 1].
long double es_value(double beta, long double z);

// Smallest 2^a 3^b 5^c >= m.
int fft_size(long long m);

// Radix passes of a 2^a 3^b 5^c size: fours, then a two, threes, fives.
std::vector<int> fft_radices(int n);

// Orders of radix passes the autotuner times for size n (the default order of
// fft_radices first, then its reverse, descending and ascending orders and the
// fours split into twos; duplicates removed).
std::vector<std::vector<int>> fft_radix_candidates(int n);

// A radix plan as decimal digits, first pass most significant (at most 8
// passes), and back; code 0 is the empty plan.
int radix_code(const std::vector<int>& r);
std::vector<int> radix_from_code(int code);

}  // namespace nr
