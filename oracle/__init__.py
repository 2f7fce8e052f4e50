"""CPU oracle for the dense Pauli decomposition (T. Jones, 2024).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke`` and the
CPU-baseline leg of ``bench.py`` may use this module; the GPU library never
does.  The arithmetic lives in ``pauli_oracle.c`` (plain C, binary64,
single-threaded); this file only builds it with gcc and marshals numpy arrays.

Functions follow the paper:
  coefficient  -- one coefficient by the Gray-code algorithm (section 3)
  coefficient_natural -- the natural-order variant with lambda in full (section 3)
  operator_at, flip_mask -- the operator of a qubit and the X/Y mask (section 2)
  decompose    -- all 4^N coefficients, Eq. (1); optional thread fan-out over
                  disjoint ranges of n (coefficients are independent, section 3)
  decompose_qgray -- all 4^N coefficients with n in quaternary Gray order and
                  the recurrence of lambda_0 across n (section 2), serial
  quaternary_gray -- the k-th string of that order
  recompose    -- sum_n c_n P_n, Eq. (1), from Eq. (pauli_tensor_elems_bitwise)
  grad_entries -- adjoint of the decomposition at chosen entries of G
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pauli_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile pauli_oracle.c with gcc (binary64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(path: str) -> str:
    """The same source built with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts), for a test run with PAULI_ORACLE_LIB=path and gcc's
    libasan preloaded."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-fPIC", "-shared", "-Wall", "-Wextra",
                           "-o", path, _SRC])
    return path


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = os.environ.get("PAULI_ORACLE_LIB")   # a separately built copy (sanitizer runs)
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        u64, i64, ci = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        lib.oracle_operator_at.argtypes = [u64, ci]
        lib.oracle_operator_at.restype = ci
        lib.oracle_flip_mask.argtypes = [u64, ci]
        lib.oracle_flip_mask.restype = u64
        for name in ("oracle_coefficient", "oracle_coefficient_natural"):
            getattr(lib, name).argtypes = [dp, ci, u64, dp]
            getattr(lib, name).restype = None
        lib.oracle_decompose_range.argtypes = [dp, ci, u64, u64, dp]
        lib.oracle_decompose_range.restype = None
        lib.oracle_decompose.argtypes = [dp, ci, dp]
        lib.oracle_decompose.restype = None
        lib.oracle_decompose_qgray.argtypes = [dp, ci, dp]
        lib.oracle_decompose_qgray.restype = None
        lib.oracle_quaternary_gray.argtypes = [u64, ci]
        lib.oracle_quaternary_gray.restype = u64
        lib.oracle_coeffs_at.argtypes = [dp, ci, up, i64, dp]
        lib.oracle_coeffs_at.restype = None
        lib.oracle_pauli_element.argtypes = [u64, ci, u64, u64, dp]
        lib.oracle_pauli_element.restype = None
        lib.oracle_recompose_entries.argtypes = [dp, ci, up, up, i64, ctypes.c_double, dp]
        lib.oracle_recompose_entries.restype = None
        lib.oracle_recompose.argtypes = [dp, ci, dp]
        lib.oracle_recompose.restype = None
        lib.oracle_grad_entries.argtypes = [dp, ci, up, up, i64, dp]
        lib.oracle_grad_entries.restype = None
        _lib = lib
        return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _uptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _as_c128(G: np.ndarray) -> np.ndarray:
    # complex64 widens to complex128 exactly
    return np.ascontiguousarray(G, dtype=np.complex128)


def _check_square(G: np.ndarray) -> int:
    D = G.shape[-1]
    if G.ndim != 2 or G.shape[0] != D or D & (D - 1):
        raise ValueError("G must be a square 2^N x 2^N matrix")
    return D.bit_length() - 1


def operator_at(n: int, t: int) -> int:
    """Operator of string n on qubit t: 0 = identity, 1 = X, 2 = Y, 3 = Z."""
    return int(_load().oracle_operator_at(n, t))


def flip_mask(n: int, N: int) -> int:
    """Bit t set where string n has X or Y on qubit t."""
    return int(_load().oracle_flip_mask(n, N))


def coefficient(G: np.ndarray, n: int) -> complex:
    G = _as_c128(G)
    N = _check_square(G)
    out = np.zeros(2)
    _load().oracle_coefficient(_dptr(G), N, n, _dptr(out))
    return complex(out[0], out[1])


def coefficient_natural(G: np.ndarray, n: int) -> complex:
    G = _as_c128(G)
    N = _check_square(G)
    out = np.zeros(2)
    _load().oracle_coefficient_natural(_dptr(G), N, n, _dptr(out))
    return complex(out[0], out[1])


def decompose(G: np.ndarray, threads: int = 1) -> np.ndarray:
    """All 4^N coefficients (complex128).  threads > 1 splits n into disjoint
    contiguous ranges evaluated concurrently (ctypes releases the GIL)."""
    G = _as_c128(G)
    N = _check_square(G)
    total = 1 << (2 * N)
    out = np.zeros(total, dtype=np.complex128)
    lib = _load()
    if threads <= 1 or total < 64:
        lib.oracle_decompose(_dptr(G), N, _dptr(out))
        return out
    bounds = np.linspace(0, total, threads + 1).astype(np.int64)
    views = []
    ths = []
    for q in range(threads):
        a, b = int(bounds[q]), int(bounds[q + 1])
        if a == b:
            continue
        v = out[a:b]
        views.append(v)
        th = threading.Thread(target=lib.oracle_decompose_range, args=(_dptr(G), N, a, b, _dptr(v)))
        th.start()
        ths.append(th)
    for th in ths:
        th.join()
    return out


def decompose_qgray(G: np.ndarray) -> np.ndarray:
    """All 4^N coefficients, strings walked in quaternary Gray order with the
    across-n recurrence of lambda_0 (serial; equal to decompose bit for bit)."""
    G = _as_c128(G)
    N = _check_square(G)
    out = np.zeros(1 << (2 * N), dtype=np.complex128)
    _load().oracle_decompose_qgray(_dptr(G), N, _dptr(out))
    return out


def quaternary_gray(k: int, N: int) -> int:
    return int(_load().oracle_quaternary_gray(k, N))


def coeffs_at(G: np.ndarray, ns, threads: int = 1) -> np.ndarray:
    G = _as_c128(G)
    N = _check_square(G)
    ns = np.ascontiguousarray(ns, dtype=np.uint64)
    out = np.zeros(ns.shape[0], dtype=np.complex128)
    lib = _load()
    if threads <= 1 or ns.shape[0] < 2 * threads:
        lib.oracle_coeffs_at(_dptr(G), N, _uptr(ns), ns.shape[0], _dptr(out))
        return out
    bounds = np.linspace(0, ns.shape[0], threads + 1).astype(np.int64)
    ths = []
    keep = []
    for q in range(threads):
        a, b = int(bounds[q]), int(bounds[q + 1])
        if a == b:
            continue
        nv = np.ascontiguousarray(ns[a:b])
        ov = out[a:b]
        keep.append(nv)
        th = threading.Thread(target=lib.oracle_coeffs_at, args=(_dptr(G), N, _uptr(nv), b - a, _dptr(ov)))
        th.start()
        ths.append(th)
    for th in ths:
        th.join()
    return out


def pauli_element(n: int, N: int, i: int, j: int) -> complex:
    out = np.zeros(2)
    _load().oracle_pauli_element(n, N, i, j, _dptr(out))
    return complex(out[0], out[1])


def recompose(c: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.complex128)
    N = (c.shape[0].bit_length() - 1) // 2
    if c.ndim != 1 or c.shape[0] != 1 << (2 * N):
        raise ValueError("c must hold 4^N coefficients")
    D = 1 << N
    G = np.zeros((D, D), dtype=np.complex128)
    _load().oracle_recompose(_dptr(c), N, _dptr(G))
    return G


def recompose_entries(c: np.ndarray, rows, cols, scale: float = 1.0) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.complex128)
    N = (c.shape[0].bit_length() - 1) // 2
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    cols = np.ascontiguousarray(cols, dtype=np.uint64)
    out = np.zeros(rows.shape[0], dtype=np.complex128)
    _load().oracle_recompose_entries(_dptr(c), N, _uptr(rows), _uptr(cols), rows.shape[0], scale,
                                     _dptr(out))
    return out


def grad_entries(gc: np.ndarray, rows, cols) -> np.ndarray:
    """dL/dRe G + i dL/dIm G at (rows, cols), given gc = dL/dRe c + i dL/dIm c."""
    gc = np.ascontiguousarray(gc, dtype=np.complex128)
    N = (gc.shape[0].bit_length() - 1) // 2
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    cols = np.ascontiguousarray(cols, dtype=np.uint64)
    out = np.zeros(rows.shape[0], dtype=np.complex128)
    _load().oracle_grad_entries(_dptr(gc), N, _uptr(rows), _uptr(cols), rows.shape[0], _dptr(out))
    return out
