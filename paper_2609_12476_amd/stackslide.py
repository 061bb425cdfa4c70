"""ctypes binding of include/nr_stackslide.h (weighted stack-slide along 0PN
tracks through stored per-segment power spectra).

Argument marshalling only; the computation runs in libnufft_resample.so.
"""
from __future__ import annotations

import ctypes
from ctypes import c_char_p, c_double, c_int32, c_void_p

import numpy as np

from . import nufft_resample as _nr


class NrSsGeometry(ctypes.Structure):
    _fields_ = [("n_seg", c_int32), ("n_beta", c_int32), ("n_bins", c_int32), ("layout", c_int32),
                ("t_coh", c_double), ("f_lo", c_double), ("df", c_double), ("f_start", c_double),
                ("f_max", c_double), ("norm", c_double), ("mu", c_double), ("sigma", c_double)]


SIGNATURES = {
    "nr_ss_create": (c_int32, [ctypes.POINTER(c_void_p), ctypes.POINTER(NrSsGeometry), c_void_p, c_void_p,
                               c_int32, c_int32, c_void_p]),
    "nr_ss_execute": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "nr_ss_execute_range": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "nr_ss_tables": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nr_ss_transpose": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "nr_ss_last_error": (c_char_p, [c_void_p]),
    "nr_ss_destroy": (None, [c_void_p]),
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


def _check(code, h=None):
    if code != 0:
        msg = lib().nr_ss_last_error(h)
        raise _nr.NrError(code, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def geometry(n_seg, n_beta, n_bins, t_coh, f_lo, df, f_start, f_max, norm, mu=2.0, sigma=2.0, layout=0):
    g = NrSsGeometry()
    g.n_seg, g.n_beta, g.n_bins, g.layout = int(n_seg), int(n_beta), int(n_bins), int(layout)
    g.t_coh, g.f_lo, g.df, g.f_start, g.f_max = float(t_coh), float(f_lo), float(df), float(f_start), float(f_max)
    g.norm, g.mu, g.sigma = float(norm), float(mu), float(sigma)
    return g


def nr_ss_create(g, beta_bank, mc, t0_steps, stream=None):
    bank = np.ascontiguousarray(beta_bank, dtype=np.float64)
    m = np.ascontiguousarray(mc, dtype=np.float64)
    h = c_void_p()
    _check(lib().nr_ss_create(ctypes.byref(h), ctypes.byref(g), bank.ctypes.data, m.ctypes.data, len(m),
                              int(t0_steps), stream))
    return h


def nr_ss_transpose(power_kij, n_beta, n_seg, n_bins, power_kji=None, stream=None):
    """power[k][i][j] -> power[k][j][i] on the device (float32 tensors)."""
    import torch
    if power_kji is None:
        power_kji = torch.empty_like(power_kij)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().nr_ss_transpose(_ptr(power_kij), int(n_beta), int(n_seg), int(n_bins), _ptr(power_kji),
                                 c_void_p(stream.cuda_stream)))
    return power_kji


class StackSlide:
    """Stack-slide plan: track tables for n_mc chirp masses x n_seg * t0_steps
    start times over a beta bank (see nr_stackslide.h)."""

    def __init__(self, g, beta_bank, mc, t0_steps, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.g = g
        self.n_mc = len(mc)
        self.t0_steps = int(t0_steps)
        self.handle = nr_ss_create(g, beta_bank, mc, t0_steps, c_void_p(stream.cuda_stream))

    @property
    def n_tracks(self):
        return self.n_mc * self.g.n_seg * self.t0_steps

    def execute(self, power, n_sigma=None, n_used=None, want_used=True):
        import torch
        n = self.g.n_beta * self.g.n_seg * self.g.n_bins
        if not (isinstance(power, torch.Tensor) and power.is_cuda and power.dtype == torch.float32
                and power.is_contiguous() and power.numel() >= n):
            raise ValueError(f"power must be a contiguous float32 CUDA tensor of {n} values")
        shape = (self.n_mc, self.g.n_seg * self.t0_steps)
        if n_sigma is None:
            n_sigma = torch.empty(shape, dtype=torch.float32, device=power.device)
        if n_used is None and want_used:
            n_used = torch.empty(shape, dtype=torch.int32, device=power.device)
        _check(lib().nr_ss_execute(self.handle, _ptr(power), _ptr(n_sigma), _ptr(n_used)), self.handle)
        return n_sigma, n_used

    def execute_range(self, power, seg_begin, seg_count, n_sigma, n_used=None):
        """Add the contribution of segments [seg_begin, seg_begin + seg_count) to
        n_sigma (and n_used); power holds just those segments in the plan's layout."""
        import torch
        n = self.g.n_beta * seg_count * self.g.n_bins
        if not (isinstance(power, torch.Tensor) and power.is_cuda and power.dtype == torch.float32
                and power.is_contiguous() and power.numel() >= n):
            raise ValueError(f"power must be a contiguous float32 CUDA tensor of {n} values")
        m = self.n_mc * self.g.n_seg * self.t0_steps
        if not (n_sigma.is_cuda and n_sigma.dtype == torch.float32 and n_sigma.numel() >= m):
            raise ValueError("n_sigma must be a float32 CUDA tensor of the plan's track grid")
        if n_used is not None and not (n_used.is_cuda and n_used.dtype == torch.int32 and n_used.numel() >= m):
            raise ValueError("n_used must be an int32 CUDA tensor of the plan's track grid")
        _check(lib().nr_ss_execute_range(self.handle, _ptr(power), int(seg_begin), int(seg_count), _ptr(n_sigma),
                                         _ptr(n_used)), self.handle)
        return n_sigma, n_used

    def tables(self):
        """(k, j, w2sum, len) as numpy arrays [n_mc][t0_steps][n_seg] (len: [n_mc][t0_steps])."""
        fam = self.n_mc * self.t0_steps
        n = fam * self.g.n_seg
        k = np.empty(n, np.int32)
        j = np.empty(n, np.int32)
        w2 = np.empty(n, np.float64)
        ln = np.empty(fam, np.int32)
        _check(lib().nr_ss_tables(self.handle, k.ctypes.data, j.ctypes.data, w2.ctypes.data, ln.ctypes.data),
               self.handle)
        s = (self.n_mc, self.t0_steps, self.g.n_seg)
        return k.reshape(s), j.reshape(s), w2.reshape(s), ln.reshape(self.n_mc, self.t0_steps)

    def close(self):
        if getattr(self, "handle", None):
            lib().nr_ss_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
