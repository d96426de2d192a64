"""ctypes wrapper around the FP64 oracle (``ols_oracle.c``).

Test infrastructure only.  Arrays cross the boundary as complex128 numpy arrays
(interleaved re, im doubles); nothing here does any of the method's arithmetic
beyond marshalling.

Paper: Moryakova & Johansson, arXiv 2406.14116.  The functions follow Sec. II
(overlap-save steps 1-5) and Sec. III-B, eqs. (5)-(7) (HFSO coefficients).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64


def load(path: str):
    """Load an oracle build from ``path`` (the default build unless a test swaps it)."""
    L = ctypes.CDLL(path)
    L.oracle_dft.argtypes = [_I, _P, _P]
    L.oracle_idft.argtypes = [_I, _P, _P]
    L.oracle_hfso_magnitude.argtypes = [_I, _I, _I, _P, _P]
    L.oracle_hfso_coeffs.argtypes = [_I, _I, _I, _I, _P, _P]
    L.oracle_blocks_generic.argtypes = [_P, _I64, _I, _I, _P, _P, _I64, _P]
    L.oracle_blocks_hfso.argtypes = [_P, _I64, _I, _I, _I, _P, _I, _P, _P, _P, _I64, _P]
    L.oracle_channel_hfso.argtypes = [_P, _I64, _I, _I, _I, _P, _I, _P, _P, _P]
    L.oracle_set_threads.argtypes = [_I]
    L.oracle_max_threads.restype = _I
    for name in ("oracle_dft", "oracle_idft", "oracle_hfso_magnitude",
                 "oracle_hfso_coeffs", "oracle_blocks_generic",
                 "oracle_blocks_hfso", "oracle_channel_hfso"):
        getattr(L, name).restype = _I
    return L


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _LIB = load(_build.LIB)
    return _LIB


class use_library:
    """Context manager that points this module at another build of the oracle
    source (used to check that the pins reject planted mistakes)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _LIB
        self.saved = lib()
        _LIB = load(self.path)
        return self

    def __exit__(self, *exc):
        global _LIB
        _LIB = self.saved
        return False


class OracleError(ValueError):
    pass


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P) if a is not None and a.size else None


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what}: invalid arguments (rc={rc})")


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def dft(s) -> np.ndarray:
    """Direct N-point DFT, X(k) = sum_i s(i) exp(-j 2 pi i k / N)."""
    s = _c128(s)
    X = np.empty_like(s)
    _check(lib().oracle_dft(s.size, _ptr(s), _ptr(X)), "dft")
    return X


def idft(Y) -> np.ndarray:
    """Direct N-point IDFT with +j and 1/N (eq. (4))."""
    Y = _c128(Y)
    z = np.empty_like(Y)
    _check(lib().oracle_idft(Y.size, _ptr(Y), _ptr(z)), "idft")
    return z


def hfso_magnitude(n: int, k1: int, v) -> np.ndarray:
    """H_R(k), k in [0, n), per eq. (6) with the mirrored transition band."""
    v = _f64(v)
    hr = np.empty(n, dtype=np.float64)
    _check(lib().oracle_hfso_magnitude(n, k1, v.size, _ptr(v), _ptr(hr)), "hfso_magnitude")
    return hr


def hfso_coeffs(n: int, hop: int, k1: int, v) -> np.ndarray:
    """H(k) = H_R(k) exp(-j 2 pi k D / n), D = (n - hop)/2 (eq. (5))."""
    v = _f64(v)
    H = np.empty(n, dtype=np.complex128)
    _check(lib().oracle_hfso_coeffs(n, hop, k1, v.size, _ptr(v), _ptr(H)), "hfso_coeffs")
    return H


def n_blocks(length: int, hop: int) -> int:
    return 0 if length <= 0 else (length + hop - 1) // hop


def _block_list(length, hop, blocks):
    if blocks is None:
        return None, n_blocks(length, hop)
    b = np.ascontiguousarray(np.asarray(blocks, dtype=np.int64))
    return b, b.size


def blocks_generic(x, n: int, hop: int, H, blocks=None) -> np.ndarray:
    """OLS with one arbitrary coefficient vector H; returns (n_sel, hop)."""
    x = _c128(x)
    H = _c128(H)
    if H.size != n:
        raise OracleError("H must have n entries")
    b, n_sel = _block_list(x.size, hop, blocks)
    out = np.empty((n_sel, hop), dtype=np.complex128)
    _check(lib().oracle_blocks_generic(_ptr(x), x.size, n, hop, _ptr(H), _ptr(b),
                                       n_sel, _ptr(out)), "blocks_generic")
    return out


def _schedule(schedule):
    sched = sorted((int(f), int(k)) for f, k in schedule)
    frm = np.ascontiguousarray([f for f, _ in sched], dtype=np.int64)
    k1s = np.ascontiguousarray([k for _, k in sched], dtype=np.int32)
    return frm, k1s


def blocks_hfso(x, n: int, hop: int, v, schedule, blocks=None) -> np.ndarray:
    """HFSO OLS output of the listed blocks, shape (n_sel, hop).

    ``schedule`` is a list of (from_block, k1); block m uses the pair with the
    largest from_block <= m.
    """
    x = _c128(x)
    v = _f64(v)
    frm, k1s = _schedule(schedule)
    b, n_sel = _block_list(x.size, hop, blocks)
    out = np.empty((n_sel, hop), dtype=np.complex128)
    _check(lib().oracle_blocks_hfso(_ptr(x), x.size, n, hop, v.size, _ptr(v), frm.size,
                                    _ptr(frm), _ptr(k1s), _ptr(b), n_sel, _ptr(out)),
           "blocks_hfso")
    return out


def channel_hfso(x, n: int, hop: int, v, schedule) -> np.ndarray:
    """Whole-channel HFSO OLS output, same length as x."""
    x = _c128(x)
    v = _f64(v)
    frm, k1s = _schedule(schedule)
    y = np.empty_like(x)
    _check(lib().oracle_channel_hfso(_ptr(x), x.size, n, hop, v.size, _ptr(v), frm.size,
                                     _ptr(frm), _ptr(k1s), _ptr(y)), "channel_hfso")
    return y


def error_db(y, y_ref) -> float:
    """Normalized RMS error in dB: 10 log10(sum|y - y_ref|^2 / sum|y_ref|^2)."""
    y = np.asarray(y, dtype=np.complex128)
    y_ref = np.asarray(y_ref, dtype=np.complex128)
    num = float(np.sum(np.abs(y - y_ref) ** 2))
    den = float(np.sum(np.abs(y_ref) ** 2))
    if num == 0.0:
        return -np.inf
    return 10.0 * np.log10(num / den)
