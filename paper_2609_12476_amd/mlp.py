"""ctypes binding of include/nr_mlp.h (the learned proposal's network).

Argument marshalling only; the computation runs in libnufft_resample.so.
"""
from __future__ import annotations

import ctypes
from ctypes import c_char_p, c_double, c_float, c_int32, c_int64, c_void_p

import numpy as np

from . import nufft_resample as _nr

N_PARAMS = 82689
N_IN = 64

SIGNATURES = {
    "nr_mlp_create": (c_int32, [ctypes.POINTER(c_void_p), c_int64, c_void_p]),
    "nr_mlp_set_params": (c_int32, [c_void_p, c_void_p]),
    "nr_mlp_get_params": (c_int32, [c_void_p, c_void_p]),
    "nr_mlp_get_state": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_int64)]),
    "nr_mlp_set_state": (c_int32, [c_void_p, c_void_p, c_int64]),
    "nr_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "nr_mlp_gradient": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "nr_mlp_adam_step": (c_int32, [c_void_p, c_void_p, c_float]),
    "nr_mlp_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_float, c_void_p]),
    "nr_mlp_region_features": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_double,
                                         c_void_p, c_void_p]),
    "nr_mlp_last_error": (c_char_p, [c_void_p]),
    "nr_mlp_destroy": (None, [c_void_p]),
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
        msg = lib().nr_mlp_last_error(h)
        raise _nr.NrError(code, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _dev_f32(t, n, what):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous float32 CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"{what} needs {n} values")


def nr_mlp_region_features(stat, n_used, n_mc, n_sub, K, norm, features=None, stream=None):
    """Region features [n_mc * n_sub][64] from a coarse segment-sum grid (device tensors)."""
    import torch
    _dev_f32(stat, n_mc * n_sub * K, "stat")
    if not (n_used.is_cuda and n_used.dtype == torch.int32 and n_used.numel() >= n_mc * n_sub):
        raise ValueError("n_used must be an int32 CUDA tensor with one count per template")
    if features is None:
        features = torch.empty(n_mc * n_sub, N_IN, dtype=torch.float32, device=stat.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().nr_mlp_region_features(_ptr(stat), _ptr(n_used), n_mc, n_sub, K, float(norm),
                                        _ptr(features), c_void_p(stream.cuda_stream)))
    return features


class Mlp:
    """The 64-256-256-1 network with device state for batches up to max_batch."""

    def __init__(self, max_batch=4096, params=None, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        _check(lib().nr_mlp_create(ctypes.byref(h), int(max_batch), c_void_p(stream.cuda_stream)))
        self.handle = h
        self.max_batch = int(max_batch)
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} parameters")
        _check(lib().nr_mlp_set_params(self.handle, p.ctypes.data), self.handle)

    def get_params(self):
        p = np.empty(N_PARAMS, np.float32)
        _check(lib().nr_mlp_get_params(self.handle, p.ctypes.data), self.handle)
        return p

    def get_state(self):
        """(state float32 [3 * N_PARAMS]: masters, Adam first and second moments; step)."""
        st = np.empty(3 * N_PARAMS, np.float32)
        step = c_int64()
        _check(lib().nr_mlp_get_state(self.handle, st.ctypes.data, ctypes.byref(step)), self.handle)
        return st, int(step.value)

    def set_state(self, state, step):
        st = np.ascontiguousarray(state, dtype=np.float32)
        if st.size != 3 * N_PARAMS:
            raise ValueError(f"expected {3 * N_PARAMS} state values")
        _check(lib().nr_mlp_set_state(self.handle, st.ctypes.data, int(step)), self.handle)

    def loss(self, x, y, out=None):
        """Mean binary cross-entropy of x [N][64] against y [N] (device), over batches of at
        most max_batch rows, as a device float64 scalar (no parameter changes)."""
        import torch
        N = x.shape[0]
        _dev_f32(x, N * N_IN, "x")
        _dev_f32(y, N, "y")
        part = torch.empty(1, dtype=torch.float32, device=x.device)
        tot = torch.zeros((), dtype=torch.float64, device=x.device) if out is None else out
        for i0 in range(0, N, self.max_batch):
            B = min(self.max_batch, N - i0)
            _check(lib().nr_mlp_gradient(self.handle, _ptr(x[i0:i0 + B]), _ptr(y[i0:i0 + B]), B, None,
                                         _ptr(part)), self.handle)
            tot += part.double()[0] * (B / N)
        return tot

    def forward(self, x, logits=None):
        import torch
        B = x.shape[0]
        _dev_f32(x, B * N_IN, "x")
        if logits is None:
            logits = torch.empty(B, dtype=torch.float32, device=x.device)
        _check(lib().nr_mlp_forward(self.handle, _ptr(x), B, _ptr(logits)), self.handle)
        return logits

    def gradient(self, x, y):
        import torch
        B = x.shape[0]
        _dev_f32(x, B * N_IN, "x")
        _dev_f32(y, B, "y")
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().nr_mlp_gradient(self.handle, _ptr(x), _ptr(y), B, _ptr(g), _ptr(loss)), self.handle)
        return g, loss

    def adam_step(self, grad, lr):
        _dev_f32(grad, N_PARAMS, "grad")
        _check(lib().nr_mlp_adam_step(self.handle, _ptr(grad), float(lr)), self.handle)

    def train_step(self, x, y, lr, loss=None):
        B = x.shape[0]
        _dev_f32(x, B * N_IN, "x")
        _dev_f32(y, B, "y")
        _check(lib().nr_mlp_train_step(self.handle, _ptr(x), _ptr(y), B, float(lr), _ptr(loss)),
               self.handle)
        return loss

    def close(self):
        if getattr(self, "handle", None):
            lib().nr_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
