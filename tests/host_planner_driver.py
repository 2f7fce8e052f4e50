"""Drives the host-side code of libpauli that runs before any device call --
argument validation, the uneven-batch layout, the Pauli-string plan and the
tune-file parser -- with seeded random and damaged inputs, through the C ABI
with fake (never dereferenced) device pointers.  Every call must fail with
the documented status before touching a device.  Run by
tests/test_sanitizers.py against a copy of the library whose host code is
built with AddressSanitizer and UndefinedBehaviorSanitizer; imports no torch.

    python tests/host_planner_driver.py LIBPATH TUNEFILE
"""
import ctypes
import os
import re
import sys

import numpy as np

EINVAL, ENOMEM = 1, 4


class Opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("in_dtype", ctypes.c_int), ("out_dtype", ctypes.c_int),
                ("tile", ctypes.c_int), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


def main(path, tune):
    with open(tune, "w") as f:
        f.write("2 10 3\n1 9 99\n\n" + "x" * 5000 + "\n"
                "B 3 1 999999999 5 5 5 5 5 5 5 5 5 5 5\n"      # a count no batch can have
                "B 3 2 1048576 1048576 0 0 0 0 0 0 0 0 0 0\n"  # too many in all
                "B 1 2 -1 2\nB\nB 3\nB 3 4 1 2 3\n"            # negative, short, truncated
                "B 3 4 0 0 1 1 2 1 0 0 0 0 0 0\n")             # one good line
    os.environ["PAULI_TUNE_CACHE"] = tune
    L = ctypes.CDLL(path)
    vp, ci, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.pauli_last_error.restype = ctypes.c_char_p
    L.pauli_batched_workspace_bytes.argtypes = [ci, ctypes.POINTER(ci), ci]
    L.pauli_batched_workspace_bytes.restype = sz
    L.pauli_decompose_batched.argtypes = [ci, ctypes.POINTER(vp), ctypes.POINTER(ci), ctypes.POINTER(vp),
                                          ctypes.POINTER(Opts)]
    L.pauli_batched_tile_selected.argtypes = [ci, ctypes.POINTER(ci), ci]
    L.pauli_tile_selected.argtypes = [ci, ci]
    for name in ("pauli_coeffs_at", "pauli_coeffs_at_backward"):
        getattr(L, name).argtypes = [vp, ci, ctypes.POINTER(ctypes.c_uint), ci, vp, ctypes.POINTER(Opts)]
    L.pauli_coeffs_at_workspace_bytes.argtypes = [ci, ci]
    L.pauli_coeffs_at_workspace_bytes.restype = sz
    L.pauli_decompose.argtypes = [vp, ci, ci, vp, ctypes.POINTER(Opts)]
    L.pauli_decompose_noalloc.argtypes = [vp, ci, ci, vp, ctypes.POINTER(Opts)]
    rng = np.random.default_rng(9100)

    # tune file: damaged lines ignored, the good ones used
    assert L.pauli_tile_selected(2, 10) == 3
    Na = (ci * 5)(5, 3, 6, 4, 5)
    assert L.pauli_batched_tile_selected(5, Na, 2) == 4

    def opts(algo=2, ws=None, wsb=0):
        o = Opts()
        o.algo, o.in_dtype, o.out_dtype, o.tile = algo, 0, 0, 0
        o.workspace, o.workspace_bytes = ws, wsb
        return o

    # uneven batch: layout of random N lists, then a refusal for a small workspace
    for trial in range(60):
        count = int(rng.integers(1, 700))
        Ns = rng.integers(1, 13, count)
        algo = int(rng.choice([1, 2]))
        N = (ci * count)(*[int(n) for n in Ns])
        need = L.pauli_batched_workspace_bytes(count, N, algo)
        packed = sum((max(32, 1 << int(n)) ** 2) * (12 if algo == 2 else 8) for n in Ns)
        assert need >= packed, (need, packed)
        G = (vp * count)(*[0x100000000 + (k << 28) for k in range(count)])
        O = (vp * count)(*[0x100000000 + (1 << 40) + (k << 28) for k in range(count)])
        o = opts(algo, ws=0x7000000000000, wsb=need - 1)
        assert L.pauli_decompose_batched(count, G, N, O, ctypes.byref(o)) == ENOMEM
    bad = (ci * 2)(3, 13)
    assert L.pauli_batched_workspace_bytes(2, bad, 2) == 0

    # string lists: the plan's workspace stays within the published bound
    pat = re.compile(rb"workspace of (\d+) bytes needed")
    for trial in range(80):
        N = int(rng.integers(0, 17))
        count = int(rng.integers(1, 3000 if N < 12 else 20000))
        strings = rng.integers(0, 4 ** N, count, dtype=np.uint64).astype(np.uint32)
        if trial % 5 == 0:      # many strings of one line group
            strings[:] = strings[0]
        sp = strings.ctypes.data_as(ctypes.POINTER(ctypes.c_uint))
        bound = L.pauli_coeffs_at_workspace_bytes(N, count)
        for fn in (L.pauli_coeffs_at, L.pauli_coeffs_at_backward):
            o = opts(ws=0x7000000000000, wsb=256)
            st = fn(0x100000000, N, sp, count, 0x300000000000, ctypes.byref(o))
            msg = L.pauli_last_error()
            if st == ENOMEM:
                need = int(pat.search(msg).group(1))
                assert need <= bound, (N, count, need, bound)
            else:
                assert st == 0 and bound >= 256, (st, msg)   # cannot happen: the plan needs more
        bad_s = strings.copy()
        bad_s[-1] = 0xFFFFFFFF if N < 16 else 0
        if N < 16:
            assert L.pauli_coeffs_at(0x100000000, N, bad_s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint)), count,
                                     0x300000000000, ctypes.byref(opts())) == EINVAL

    # single-matrix entry points: refusals before any launch
    for N, batch, want in ((-1, 1, EINVAL), (17, 1, EINVAL), (3, 0, EINVAL), (12, 1, ENOMEM)):
        assert L.pauli_decompose_noalloc(0x100000000, N, batch, 0x300000000000, ctypes.byref(opts())) == want
    o = opts(ws=0x7000000000000, wsb=16)
    assert L.pauli_decompose(0x100000000, 10, 1, 0x300000000000, ctypes.byref(o)) == ENOMEM
    print("host planner driver: ok")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
