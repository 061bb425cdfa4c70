"""Oracle for semicoherent NUFFT resampling -- TEST INFRASTRUCTURE ONLY.

Plain, slow, high-precision CPU reference (``nr_oracle.c``: __float128 tau
differences, long-double direct non-uniform DFT and segment sum).  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (IEEE arithmetic, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", _SRC,
           "-o", _LIB + ".tmp", "-lquadmath", "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.nro_beta.restype = ctypes.c_double
        L.nro_beta.argtypes = [ctypes.c_double, ctypes.c_double]
        L.nro_t_sun.restype = ctypes.c_double
        L.nro_num_threads.restype = ctypes.c_int
        L.nro_dtau.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int64, P]
        L.nro_valid.restype = ctypes.c_int
        L.nro_valid.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int64]
        L.nro_spectrum.restype = ctypes.c_int
        L.nro_spectrum.argtypes = [P, ctypes.c_int, ctypes.c_int64] + [ctypes.c_double] * 7 + \
            [ctypes.c_int32, P, P, P]
        L.nro_spectra.argtypes = [P, ctypes.c_int] + [P] * 10 + [ctypes.c_int64] + [P] * 6
        L.nro_semicoherent.argtypes = [P, ctypes.c_int, ctypes.c_int32] + [P] * 4 + \
            [ctypes.c_int32] + [P] * 10
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _strain(x):
    if np.iscomplexobj(x):
        return np.ascontiguousarray(x, dtype=np.complex128).view(np.float64), 1
    return np.ascontiguousarray(x, dtype=np.float64), 0


def beta(mc_msun, f0):
    return lib().nro_beta(float(mc_msun), float(f0))


def num_threads():
    return lib().nro_num_threads()


def t_sun():
    return lib().nro_t_sun()


def dtau(mc_msun, f0, t_start, fs, L):
    out = np.empty(int(L), np.float64)
    lib().nro_dtau(float(mc_msun), float(f0), float(t_start), float(fs), int(L), _p(out))
    return out


def valid(mc_msun, f0, f_max, t_start, fs, L):
    return bool(lib().nro_valid(float(mc_msun), float(f0), float(f_max), float(t_start),
                                float(fs), int(L)))


def spectrum(x, fs, t_start, mc_msun, f0, f_lo, df, K, f_max=0.0, kidx=None):
    """Direct spectrum of one segment x (bins kidx, default 0..K-1). Returns (X, valid)."""
    xs, cplx = _strain(x)
    L = len(x)
    if kidx is not None:
        kidx = np.ascontiguousarray(kidx, np.int32)
        nk = len(kidx)
    else:
        nk = int(K)
    re = np.empty(nk); im = np.empty(nk)
    ok = lib().nro_spectrum(_p(xs), cplx, L, float(fs), float(t_start), float(mc_msun), float(f0),
                            float(f_lo), float(df), float(f_max), nk,
                            _p(kidx) if kidx is not None else None, _p(re), _p(im))
    return re + 1j * im, bool(ok)


def _wl_arrays(w):
    return dict(
        seg_off=np.ascontiguousarray(w.seg_offset, np.int64),
        seg_len=np.ascontiguousarray(w.seg_len, np.int64),
        seg_fs=np.ascontiguousarray(w.seg_fs, np.float64),
        seg_t=np.ascontiguousarray(w.seg_t, np.float64),
        mc=np.ascontiguousarray(w.mc, np.float64), f0=np.ascontiguousarray(w.f0, np.float64),
        f_lo=np.ascontiguousarray(w.f_lo, np.float64), df=np.ascontiguousarray(w.df, np.float64),
        K=np.ascontiguousarray(w.n_bins, np.int32), f_max=np.ascontiguousarray(w.f_max, np.float64))


def spectra(w, inst_idx=None):
    """Spectra of a workload's instances (all, or the listed instance indices).

    Returns (X complex128 packed by instance, offsets int64 [n+1], valid uint8 [n])."""
    a = _wl_arrays(w)
    s, m = w.instances()
    if inst_idx is not None:
        inst_idx = np.asarray(inst_idx, np.int64)
        s, m = s[inst_idx], m[inst_idx]
    s = np.ascontiguousarray(s, np.int32); m = np.ascontiguousarray(m, np.int32)
    K = a["K"][m].astype(np.int64)
    off = np.zeros(len(K) + 1, np.int64)
    np.cumsum(K, out=off[1:])
    re = np.zeros(off[-1]); im = np.zeros(off[-1]); ok = np.zeros(len(s), np.uint8)
    xs, cplx = _strain(w.strain)
    lib().nro_spectra(_p(xs), cplx, _p(a["seg_off"]), _p(a["seg_len"]), _p(a["seg_fs"]),
                      _p(a["seg_t"]), _p(a["mc"]), _p(a["f0"]), _p(a["f_lo"]), _p(a["df"]),
                      _p(a["K"]), _p(a["f_max"]), len(s), _p(s), _p(m), _p(off),
                      _p(re), _p(im), _p(ok))
    return re + 1j * im, off, ok


def semicoherent(w, seg_weight=None):
    """Segment sums for every template over all segments: (stat packed [sum K], offsets, n_used)."""
    a = _wl_arrays(w)
    K = a["K"].astype(np.int64)
    off = np.zeros(len(K) + 1, np.int64)
    np.cumsum(K, out=off[1:])
    stat = np.zeros(off[-1]); used = np.zeros(w.n_tmpl, np.int32)
    xs, cplx = _strain(w.strain)
    sw = None if seg_weight is None else np.ascontiguousarray(seg_weight, np.float64)
    lib().nro_semicoherent(_p(xs), cplx, w.n_seg, _p(a["seg_off"]), _p(a["seg_len"]),
                           _p(a["seg_fs"]), _p(a["seg_t"]), w.n_tmpl, _p(a["mc"]), _p(a["f0"]),
                           _p(a["f_lo"]), _p(a["df"]), _p(a["K"]), _p(a["f_max"]),
                           _p(sw) if sw is not None else None, _p(off), _p(stat), _p(used))
    return stat, off, used
