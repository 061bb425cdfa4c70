"""ctypes binding of include/nr_strobo.h (stroboscopic-resampling baseline)
and the baseline's spectrum: the library's nearest-neighbour fold followed by
the vendor FFT (rocFFT through torch) -- a comparison method, not part of the
NUFFT path.
"""
from __future__ import annotations

import ctypes
from ctypes import c_char_p, c_double, c_int32, c_int64, c_void_p

from . import nufft_resample as _nr

SIGNATURES = {
    "nr_strobo_points": (c_int32, [c_double, c_int64, c_double, c_double, ctypes.POINTER(c_int64)]),
    "nr_strobo_fold": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_double, c_double, c_double, c_int64,
                                 c_void_p, c_void_p]),
    "nr_strobo_last_error": (c_char_p, []),
}
_bound = False


def lib():
    global _bound
    L = _nr.load()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _check(code):
    if code != 0:
        msg = lib().nr_strobo_last_error()
        raise _nr.NrError(code, msg.decode() if msg else "")


def nr_strobo_points(fs_o, n_samples, mc, f0):
    m = c_int64()
    _check(lib().nr_strobo_points(float(fs_o), int(n_samples), float(mc), float(f0), ctypes.byref(m)))
    return m.value


def nr_strobo_fold(x, n_samples, fs_o, mc, f0, fold, n_seg=1, out=None, stream=None):
    """Folds of the tau-uniform nearest-neighbour series of n_seg segments
    stored one after another (complex64 tensor [n_seg][fold])."""
    import torch
    cplx = x.dtype == torch.complex64
    if not (x.is_cuda and x.is_contiguous() and (cplx or x.dtype == torch.float32)):
        raise ValueError("x must be a contiguous float32 or complex64 CUDA tensor")
    if x.numel() < n_samples * n_seg:
        raise ValueError("x is shorter than n_seg * n_samples")
    if out is None:
        out = torch.empty(int(n_seg), int(fold), dtype=torch.complex64, device=x.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().nr_strobo_fold(c_void_p(x.data_ptr()), int(cplx), int(n_samples), int(n_seg), float(fs_o),
                                float(mc), float(f0), int(fold), c_void_p(out.data_ptr()),
                                c_void_p(stream.cuda_stream)))
    return out


def spectrum(x_o, fs_o, oversample, mc, f0, f_lo, df, K, n_seg=1):
    """Stroboscopic spectra [n_seg][K] at f_lo + k df, k < K (f_lo / df and
    fs_o / df integers) of n_seg segments stored one after another."""
    import torch
    N = int(round(fs_o / df))
    k0 = int(round(f_lo / df))
    if abs(N * df - fs_o) > 1e-9 * fs_o or abs(k0 * df - f_lo) > 1e-9 * max(1.0, abs(f_lo)):
        raise ValueError("fs_o / df and f_lo / df must be integers")
    y = nr_strobo_fold(x_o, x_o.numel() // n_seg, fs_o, mc, f0, N, n_seg=n_seg)
    Y = torch.fft.fft(y, dim=1)
    idx = (k0 + torch.arange(K, device=x_o.device)) % N
    return Y[:, idx] / oversample
