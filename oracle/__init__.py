"""Plain CPU FP64 oracle for the SHT / associated Legendre transform.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``, never by the product package.
It shares no code with the HIP library.  The C source (``sht_oracle.c``) is
compiled with gcc on first use (or by ``__graft_entry__.build``).

Every function cites the passage of Bremer, Chen & Yang (arXiv 2004.11346) it
writes out:

* ``gauss_legendre``  -- Section 1 (the 2N-point Gauss-Legendre rule in
  x = cos(theta), nodes ascending).
* ``plm``             -- Section 1 / Section 3.1.1 (L2-normalised associated
  Legendre functions; orthonormal basis).  No Condon-Shortley phase.
* ``alt_forward``     -- Section 1, ALT definition; Section 3.1.1 (the
  2N x (2N-|m|) matrix of Pbar_j^{|m|}(cos theta_i) applied to beta).
* ``alt_transpose``   -- Section 3.1.1 (B = A^T W; ``weights=False`` gives A^T).
* ``dft_synthesis`` / ``dft_analysis`` -- Section 1 (f = sum_m g e^{i m phi},
  phi_j = 2 pi (j + 1/2)/(4N - 1)).
* ``sht_forward`` / ``sht_inverse`` / ``sht_adjoint`` -- compositions of the
  above (Section 1; Section 3.1.1).
* ``real_to_full`` / ``full_to_real`` / ``sht_forward_real`` /
  ``sht_inverse_real`` -- real fields: in the expansion of f (Section 1) the
  same Pbar_k^{|m|} multiplies e^{i m phi} and e^{-i m phi}, so f is real
  exactly when beta_{k,-m} = conj(beta_{k,m}) (and beta_{k,0} is real); the
  real transforms are the complex ones on coefficients extended that way.

Parity status of each function is recorded in the tests that pin it
(``tests/test_oracle_pins.py``); every function above is pinned there against
closed forms, library routines, identities or brute-force integration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sht_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            lib.oracle_num_threads.restype = I
            lib.oracle_coef_offset.restype = ctypes.c_longlong
            lib.oracle_coef_offset.argtypes = [I, I]
            lib.oracle_gauss_legendre.argtypes = [I, P, P]
            lib.oracle_plm.argtypes = [I, I, D, P]
            lib.oracle_alt_forward_grid.argtypes = [I, P, P, P]
            lib.oracle_alt_forward_orders.argtypes = [I, P, P, I, P, P]
            lib.oracle_alt_forward_rows.argtypes = [I, P, P, I, P, P]
            lib.oracle_alt_transpose_grid.argtypes = [I, P, P, P, P]
            lib.oracle_alt_transpose_orders.argtypes = [I, P, P, I, P, P, P]
            lib.oracle_dft_synthesis.argtypes = [I, P, I, P, P]
            lib.oracle_dft_analysis.argtypes = [I, P, I, D, P]
            for name in ("oracle_gauss_legendre", "oracle_plm", "oracle_alt_forward_grid",
                         "oracle_alt_forward_orders", "oracle_alt_forward_rows", "oracle_alt_transpose_grid",
                         "oracle_alt_transpose_orders", "oracle_dft_synthesis",
                         "oracle_dft_analysis"):
                getattr(lib, name).restype = I
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _chk(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def coef_offset(N: int, m: int) -> int:
    return int(_load().oracle_coef_offset(N, m))


def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes (ascending) and weights (Section 1)."""
    x = np.empty(n)
    w = np.empty(n)
    _chk(_load().oracle_gauss_legendre(n, _ptr(x), _ptr(w)), "gauss_legendre")
    return x, w


def plm(m: int, kmax: int, t: float) -> np.ndarray:
    """Pbar_k^m(t) for k = m..kmax (L2-normalised, no Condon-Shortley phase)."""
    out = np.empty(kmax - m + 1)
    _chk(_load().oracle_plm(m, kmax, float(t), _ptr(out)), "plm")
    return out


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def alt_forward(N: int, beta: np.ndarray, x: np.ndarray | None = None) -> np.ndarray:
    """Forward ALT for all orders: g[2N, M] (column = m mod M), complex128."""
    if x is None:
        x, _ = gauss_legendre(2 * N)
    beta = _c128(beta)
    assert beta.shape == (4 * N * N,)
    g = np.zeros((2 * N, 4 * N - 1), dtype=np.complex128)
    _chk(_load().oracle_alt_forward_grid(N, _ptr(np.ascontiguousarray(x)), _ptr(beta), _ptr(g)),
         "alt_forward_grid")
    return g


def alt_forward_orders(N: int, beta: np.ndarray, absm, x: np.ndarray | None = None) -> np.ndarray:
    """Forward ALT for listed |m|: out[i, s, l], s=0 -> +|m|, s=1 -> -|m|."""
    if x is None:
        x, _ = gauss_legendre(2 * N)
    beta = _c128(beta)
    absm = np.ascontiguousarray(absm, dtype=np.int32)
    out = np.zeros((len(absm), 2, 2 * N), dtype=np.complex128)
    _chk(_load().oracle_alt_forward_orders(N, _ptr(np.ascontiguousarray(x)), _ptr(beta),
                                           len(absm), _ptr(absm), _ptr(out)), "alt_forward_orders")
    return out


def alt_forward_rows(N: int, beta: np.ndarray, rows, x: np.ndarray | None = None) -> np.ndarray:
    """Forward ALT for all orders at the listed nodes: g_rows[len(rows), M]."""
    if x is None:
        x, _ = gauss_legendre(2 * N)
    beta = _c128(beta)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((len(rows), 4 * N - 1), dtype=np.complex128)
    _chk(_load().oracle_alt_forward_rows(N, _ptr(np.ascontiguousarray(x)), _ptr(beta), len(rows), _ptr(rows),
                                         _ptr(out)), "alt_forward_rows")
    return out


def alt_transpose(N: int, g: np.ndarray, weights: bool = True, x=None, w=None) -> np.ndarray:
    """beta = A^T W g (weights=True, the inverse ALT) or A^T g (weights=False)."""
    if x is None or w is None:
        x, w = gauss_legendre(2 * N)
    g = _c128(g)
    assert g.shape == (2 * N, 4 * N - 1)
    beta = np.zeros(4 * N * N, dtype=np.complex128)
    wp = _ptr(np.ascontiguousarray(w)) if weights else None
    _chk(_load().oracle_alt_transpose_grid(N, _ptr(np.ascontiguousarray(x)), wp, _ptr(g), _ptr(beta)),
         "alt_transpose_grid")
    return beta


def alt_transpose_orders(N: int, gin: np.ndarray, absm, weights: bool = True, x=None, w=None) -> np.ndarray:
    """Transposed ALT for listed |m|; gin[i, s, l] -> out[i, s, k-|m|] (stride 2N)."""
    if x is None or w is None:
        x, w = gauss_legendre(2 * N)
    gin = _c128(gin)
    absm = np.ascontiguousarray(absm, dtype=np.int32)
    assert gin.shape == (len(absm), 2, 2 * N)
    out = np.zeros((len(absm), 2, 2 * N), dtype=np.complex128)
    wp = _ptr(np.ascontiguousarray(w)) if weights else None
    _chk(_load().oracle_alt_transpose_orders(N, _ptr(np.ascontiguousarray(x)), wp, len(absm),
                                             _ptr(absm), _ptr(gin), _ptr(out)), "alt_transpose_orders")
    return out


def dft_synthesis(N: int, g: np.ndarray, rows=None) -> np.ndarray:
    """f[l, j] = sum_m g[l, m mod M] exp(i m phi_j) for the listed rows."""
    g = _c128(g)
    assert g.shape == (2 * N, 4 * N - 1)
    if rows is None:
        out = np.zeros_like(g)
        _chk(_load().oracle_dft_synthesis(N, _ptr(g), 0, None, _ptr(out)), "dft_synthesis")
        return out
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((len(rows), 4 * N - 1), dtype=np.complex128)
    _chk(_load().oracle_dft_synthesis(N, _ptr(g), len(rows), _ptr(rows), _ptr(out)), "dft_synthesis")
    return out


def dft_analysis(N: int, f_rows: np.ndarray, scale: float | None = None) -> np.ndarray:
    """g[l, m mod M] = scale * sum_j f[l, j] exp(-i m phi_j); default scale 1/M."""
    f_rows = _c128(f_rows)
    M = 4 * N - 1
    assert f_rows.ndim == 2 and f_rows.shape[1] == M
    if scale is None:
        scale = 1.0 / M
    out = np.zeros_like(f_rows)
    _chk(_load().oracle_dft_analysis(N, _ptr(f_rows), f_rows.shape[0], float(scale), _ptr(out)),
         "dft_analysis")
    return out


def real_to_full(N: int, beta_half: np.ndarray) -> np.ndarray:
    """Coefficients of orders m >= 0 (orders 0..2N-1, degrees k = m..2N-1 inside
    each) -> the full m-major coefficients of the real field they describe:
    beta_{k,-m} = conj(beta_{k,m}), beta_{k,0} real (its imaginary part
    dropped)."""
    n = 2 * N
    beta_half = _c128(beta_half)
    assert beta_half.shape == (N * (2 * N + 1),)
    full = np.zeros(4 * N * N, dtype=np.complex128)
    h = 0
    for m in range(n):
        seg = beta_half[h:h + n - m]
        h += n - m
        o = coef_offset(N, m)
        if m == 0:
            full[o:o + n] = seg.real
        else:
            full[o:o + n - m] = seg
            o2 = coef_offset(N, -m)
            full[o2:o2 + n - m] = np.conj(seg)
    return full


def full_to_real(N: int, beta: np.ndarray) -> np.ndarray:
    """The orders m >= 0 of full m-major coefficients, in the half layout."""
    n = 2 * N
    beta = _c128(beta)
    out = []
    for m in range(n):
        o = coef_offset(N, m)
        out.append(beta[o:o + n - m])
    return np.concatenate(out)


def sht_forward_real(N: int, beta_half: np.ndarray) -> np.ndarray:
    """Forward SHT of a real field given by its orders m >= 0: real f[2N, M]
    (the real part; the imaginary part of the complex transform is rounding)."""
    return sht_forward(N, real_to_full(N, beta_half)).real


def sht_inverse_real(N: int, f: np.ndarray) -> np.ndarray:
    """Inverse SHT of a real grid f[2N, M]: its coefficients of orders m >= 0."""
    return full_to_real(N, sht_inverse(N, np.asarray(f, dtype=np.float64).astype(np.complex128)))


def sht_forward(N: int, beta: np.ndarray) -> np.ndarray:
    """Forward SHT: coefficients (m-major) -> grid values f[2N, M] (Section 1)."""
    return dft_synthesis(N, alt_forward(N, beta))


def sht_inverse(N: int, f: np.ndarray) -> np.ndarray:
    """Inverse SHT: f[2N, M] -> coefficients; g = (1/M) DFT^H f, beta = A^T W g."""
    return alt_transpose(N, dft_analysis(N, f), weights=True)


def sht_adjoint(N: int, f: np.ndarray) -> np.ndarray:
    """Conjugate transpose of the forward SHT: beta = A^T DFT^H f (no 1/M, no W)."""
    return alt_transpose(N, dft_analysis(N, f, scale=1.0), weights=False)
