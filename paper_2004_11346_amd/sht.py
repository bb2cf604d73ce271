"""Python front end: a plan object wrapping the C-ABI, operating on torch
tensors that live on the GPU.  Every transform runs in the native HIP
library; this module only checks shapes/dtypes and passes pointers and the
current stream.

Tensor conventions (see ``include/sht.h``):
  beta : complex [batch, 4N^2], m-major (orders 0, 1, -1, 2, -2, ...;
         degrees k = |m| .. 2N-1 inside an order)
  f, g : complex [batch, 2N, 4N-1], rows = Gauss-Legendre nodes ascending in
         x = cos(theta), columns = phi_j = 2 pi (j + 1/2)/(4N - 1)
"""
from __future__ import annotations

import ctypes
import json

import torch

from . import lib as _l

_DT = {torch.complex128: _l.SHT_F64, torch.complex64: _l.SHT_F32}
_METHOD = {"dense": _l.SHT_DENSE, "idbf": _l.SHT_IDBF}


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def check_tensor(t: torch.Tensor, dtype, shape, name: str, require_cuda: bool = True):
    """Reject what the C ABI cannot take as a plain pointer: host tensors, a
    wrong dtype or shape, non-contiguous storage, and lazy conjugate or
    negative views (their memory holds the unconjugated / unnegated values)."""
    if not isinstance(t, torch.Tensor) or (require_cuda and not t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.is_conj() or t.is_neg():
        raise ValueError(f"{name} is a lazy conjugate/negative view; call .resolve_conj().resolve_neg() first")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def materialize(t: torch.Tensor) -> torch.Tensor:
    """Contiguous tensor whose memory holds its values (lazy conj/neg resolved)."""
    return t.resolve_conj().resolve_neg().contiguous()


class Plan:
    """A transform plan of degree N for ``batch`` fields.

    method: "dense" (plain form) or "idbf" (fast form).
    dtype:  torch.complex128 (FP64) or torch.complex64 (FP32).
    Extra keyword arguments set ``sht_plan_opts`` fields (eps, n0, leaf, rk,
    oversample, rsvd_r, rsvd_q, sampling, seed, threads, f32_mode, min_idbf,
    dense_gen, m_lo, m_hi, dft_schedule, cache_dir).
    """

    def __init__(self, N: int, batch: int = 1, dtype=torch.complex128, method: str = "dense", **opts):
        self._lib = _l.load()
        self.N = int(N)
        self.batch = int(batch)
        self.dtype = dtype
        self.method = method
        self.M = 4 * self.N - 1
        o = _l.default_opts(**opts)
        h = ctypes.c_void_p()
        _l.check(self._lib.sht_plan_create(self.N, self.batch, _DT[dtype], _METHOD[method],
                                           ctypes.byref(o), ctypes.byref(h)), "sht_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ shapes
    @property
    def coef_shape(self):
        return (self.batch, 4 * self.N * self.N)

    @property
    def grid_shape(self):
        return (self.batch, 2 * self.N, self.M)

    def _check(self, t: torch.Tensor, shape, name):
        check_tensor(t, self.dtype, shape, name)

    def empty_coefs(self, device="cuda"):
        return torch.empty(self.coef_shape, dtype=self.dtype, device=device)

    def empty_grid(self, device="cuda"):
        return torch.empty(self.grid_shape, dtype=self.dtype, device=device)

    # ------------------------------------------------------------- transforms
    def forward(self, beta: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Forward SHT: coefficients -> grid values."""
        self._check(beta, self.coef_shape, "beta")
        out = self.empty_grid(beta.device) if out is None else out
        self._check(out, self.grid_shape, "out")
        _l.check(self._lib.sht_forward(self._h, beta.data_ptr(), out.data_ptr(),
                                       ctypes.c_void_p(_stream_ptr(stream))), "sht_forward")
        return out

    def inverse(self, f: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Inverse SHT: grid values -> coefficients."""
        self._check(f, self.grid_shape, "f")
        out = self.empty_coefs(f.device) if out is None else out
        self._check(out, self.coef_shape, "out")
        _l.check(self._lib.sht_inverse(self._h, f.data_ptr(), out.data_ptr(),
                                       ctypes.c_void_p(_stream_ptr(stream))), "sht_inverse")
        return out

    # ------------------------------------------------------------ real fields
    @property
    def half_coef_count(self):
        return self.N * (2 * self.N + 1)

    @property
    def real_dtype(self):
        return torch.float64 if self.dtype == torch.complex128 else torch.float32

    def forward_real(self, beta_half: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Forward SHT of real fields: beta_half [nreal, N(2N+1)] complex (orders
        m >= 0) -> real grid values [nreal, 2N, 4N-1]."""
        nreal = beta_half.shape[0] if beta_half.dim() == 2 else -1
        self._check(beta_half, (nreal, self.half_coef_count), "beta_half")
        out = torch.empty((nreal, 2 * self.N, self.M), dtype=self.real_dtype, device=beta_half.device) \
            if out is None else out
        check_tensor(out, self.real_dtype, (nreal, 2 * self.N, self.M), "out")
        _l.check(self._lib.sht_forward_real(self._h, nreal, beta_half.data_ptr(), out.data_ptr(),
                                            ctypes.c_void_p(_stream_ptr(stream))), "sht_forward_real")
        return out

    def inverse_real(self, f: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Inverse SHT of real fields: real grid [nreal, 2N, 4N-1] -> beta_half."""
        nreal = f.shape[0] if f.dim() == 3 else -1
        check_tensor(f, self.real_dtype, (nreal, 2 * self.N, self.M), "f")
        out = torch.empty((nreal, self.half_coef_count), dtype=self.dtype, device=f.device) if out is None else out
        self._check(out, (nreal, self.half_coef_count), "out")
        _l.check(self._lib.sht_inverse_real(self._h, nreal, f.data_ptr(), out.data_ptr(),
                                            ctypes.c_void_p(_stream_ptr(stream))), "sht_inverse_real")
        return out

    def set_graph_capture(self, enable: bool = True):
        """Graph mode: forward / inverse / backward calls replay a hipGraph per
        (direction, input, output) after their first call."""
        _l.check(self._lib.sht_set_graph_capture(self._h, int(bool(enable))), "sht_set_graph_capture")

    def inverse_noalloc(self, f: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """Inverse SHT that allocates nothing: the phi-analysed grid is staged in
        the library's fixed per-GPU scratch (at most 128 MiB) instead of the
        plan's workspace.  `out` must be given."""
        self._check(f, self.grid_shape, "f")
        self._check(out, self.coef_shape, "out")
        _l.check(self._lib.sht_inverse_noalloc(self._h, f.data_ptr(), out.data_ptr(),
                                               ctypes.c_void_p(_stream_ptr(stream))), "sht_inverse_noalloc")
        return out

    def backward(self, grad_f: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Adjoint of forward (conjugate transpose): grad_f -> grad_beta."""
        self._check(grad_f, self.grid_shape, "grad_f")
        out = self.empty_coefs(grad_f.device) if out is None else out
        self._check(out, self.coef_shape, "out")
        _l.check(self._lib.sht_backward(self._h, grad_f.data_ptr(), out.data_ptr(),
                                        ctypes.c_void_p(_stream_ptr(stream))), "sht_backward")
        return out

    def alt(self, m_lo: int, m_hi: int, direction: str, inp: torch.Tensor, out: torch.Tensor, stream=None):
        """ALT only for orders m_lo <= |m| <= m_hi.  direction: "fwd" (beta -> g),
        "inv" (g -> beta, A^T W) or "adj" (g -> beta, A^T)."""
        d = {"fwd": _l.SHT_FWD, "inv": _l.SHT_INV, "adj": _l.SHT_ADJ}[direction]
        if d == _l.SHT_FWD:
            self._check(inp, self.coef_shape, "beta")
            self._check(out, self.grid_shape, "g")
        else:
            self._check(inp, self.grid_shape, "g")
            self._check(out, self.coef_shape, "beta")
        _l.check(self._lib.sht_alt_apply(self._h, int(m_lo), int(m_hi), d, inp.data_ptr(), out.data_ptr(),
                                         ctypes.c_void_p(_stream_ptr(stream))), "sht_alt_apply")
        return out

    # ------------------------------------------------------------------ info
    def stats(self) -> dict:
        n = _l.check(self._lib.sht_plan_stats(self._h, None, 0), "sht_plan_stats")
        buf = ctypes.create_string_buffer(n)
        _l.check(self._lib.sht_plan_stats(self._h, buf, n), "sht_plan_stats")
        return json.loads(buf.value.decode())

    def profile(self, enable: bool = True):
        """Start (clearing earlier records) or stop per-kernel event timing."""
        _l.check(self._lib.sht_profile(self._h, 1 if enable else 0), "sht_profile")

    def profile_report(self) -> dict:
        """{kernel: {"launches", "total_ms", "avg_ms"}} of the recorded calls."""
        n = _l.check(self._lib.sht_profile_report(self._h, None, 0), "sht_profile_report")
        buf = ctypes.create_string_buffer(n)
        _l.check(self._lib.sht_profile_report(self._h, buf, n), "sht_profile_report")
        return json.loads(buf.value.decode())

    def nodes(self):
        import numpy as np
        x = np.empty(2 * self.N)
        w = np.empty(2 * self.N)
        _l.check(self._lib.sht_plan_nodes(self._h, x.ctypes.data, w.ctypes.data), "sht_plan_nodes")
        return x, w


def host_gauss_legendre(n: int):
    """The library's own Gauss-Legendre rule (host code, no GPU needed)."""
    import numpy as np
    x = np.empty(n)
    w = np.empty(n)
    _l.check(_l.load().sht_host_gauss_legendre(n, x.ctypes.data, w.ctypes.data), "sht_host_gauss_legendre")
    return x, w


class Group:
    """Many independent transforms of different degrees (``Ns[i]``) and field
    counts (``fields[i]``) applied together.  mode "persistent": persistent
    kernels over a longest-first queue (N <= 1024, 1-4 fields); mode
    "batched": one tuned plan per distinct degree over all its fields.  Bind
    the per-transform tensors once, then call ``forward`` / ``inverse`` (or
    capture them into a hipGraph and ``replay``)."""

    def __init__(self, Ns, fields, dtype=torch.complex128, mode: str = "persistent", tune_file=None,
                 plan_cache_dir=None):
        self._lib = _l.load()
        self.Ns = [int(n) for n in Ns]
        self.fields = [int(f) for f in fields]
        if len(self.Ns) != len(self.fields):
            raise ValueError("Ns and fields must have the same length")
        self.dtype = dtype
        n = len(self.Ns)
        arr = ctypes.c_int * n
        h = ctypes.c_void_p()
        o = _l.GroupOpts()
        self._lib.sht_group_opts_default(ctypes.byref(o))
        o.mode = {"persistent": _l.SHT_GROUP_PERSISTENT, "batched": _l.SHT_GROUP_BATCHED}[mode]
        self._keep = [s.encode() if isinstance(s, str) else s for s in (tune_file, plan_cache_dir)]
        o.tune_file, o.plan_cache_dir = self._keep
        _l.check(self._lib.sht_group_create_ex(n, arr(*self.Ns), arr(*self.fields), _DT[dtype], ctypes.byref(o),
                                               ctypes.byref(h)), "sht_group_create")
        self._h = h
        self._bound = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sht_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def coef_shape(self, i):
        return (self.fields[i], 4 * self.Ns[i] ** 2)

    def grid_shape(self, i):
        return (self.fields[i], 2 * self.Ns[i], 4 * self.Ns[i] - 1)

    def bind(self, betas, fs):
        """betas[i]: [fields_i, 4 N_i^2], fs[i]: [fields_i, 2 N_i, 4 N_i - 1]
        (complex, contiguous, on the GPU).  The tensors must stay alive."""
        n = len(self.Ns)
        if len(betas) != n or len(fs) != n:
            raise ValueError("one beta and one f tensor per transform")
        for i in range(n):
            check_tensor(betas[i], self.dtype, self.coef_shape(i), f"beta[{i}]")
            check_tensor(fs[i], self.dtype, self.grid_shape(i), f"f[{i}]")
        arr = ctypes.c_void_p * n
        _l.check(self._lib.sht_group_bind(self._h, arr(*[b.data_ptr() for b in betas]),
                                          arr(*[f.data_ptr() for f in fs])), "sht_group_bind")
        self._bound = (list(betas), list(fs))

    def forward(self, stream=None):
        _l.check(self._lib.sht_group_forward(self._h, ctypes.c_void_p(_stream_ptr(stream))), "sht_group_forward")

    def inverse(self, stream=None):
        _l.check(self._lib.sht_group_inverse(self._h, ctypes.c_void_p(_stream_ptr(stream))), "sht_group_inverse")

    def tune(self, stream=None):
        _l.check(self._lib.sht_group_tune(self._h, ctypes.c_void_p(_stream_ptr(stream))), "sht_group_tune")

    def capture(self, direction: str, stream):
        d = {"fwd": _l.SHT_FWD, "inv": _l.SHT_INV}[direction]
        _l.check(self._lib.sht_group_capture(self._h, d, ctypes.c_void_p(_stream_ptr(stream))), "sht_group_capture")

    def replay(self, direction: str, stream=None):
        d = {"fwd": _l.SHT_FWD, "inv": _l.SHT_INV}[direction]
        _l.check(self._lib.sht_group_replay(self._h, d, ctypes.c_void_p(_stream_ptr(stream))), "sht_group_replay")

    def stats(self) -> dict:
        n = _l.check(self._lib.sht_group_stats(self._h, None, 0), "sht_group_stats")
        buf = ctypes.create_string_buffer(n)
        _l.check(self._lib.sht_group_stats(self._h, buf, n), "sht_group_stats")
        return json.loads(buf.value.decode())
