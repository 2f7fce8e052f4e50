"""GPU behaviour of the C ABI beyond parity: the two-pass entry points equal
the one-call entry points bit for bit, caller workspace and library pool give
identical results, repeated runs are bitwise deterministic, complex128 input
and output, non-finite inputs propagate to the outputs that read them."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_two_pass_equals_one_call(algo, mode):
    p = lib()
    L = p.load_library()
    N = 9
    if mode == 0:
        x = torch.from_numpy(workloads.iid_complex(N, 5, np.complex64)).cuda()
    else:
        x = torch.from_numpy(workloads.iid_complex(N, 6, np.complex64).reshape(-1)).cuda()
    shape = (4 ** N,) if mode == 0 else (1 << N, 1 << N)
    a = torch.empty(shape, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    ws = torch.empty(L.pauli_workspace_bytes(p.ALGOS[algo], N, 1), dtype=torch.uint8, device="cuda")
    o = p._opts(algo, 0, 0, 0, stream(), ws)
    one = [L.pauli_decompose, L.pauli_reconstruct, L.pauli_decompose_backward][mode]
    assert one(x.data_ptr(), N, 1, a.data_ptr(), ctypes.byref(o)) == 0
    assert L.pauli_pack(x.data_ptr(), N, 1, mode, ctypes.byref(o)) == 0
    assert L.pauli_contract(N, 1, mode, b.data_ptr(), ctypes.byref(o)) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_library_pool_vs_caller_workspace_and_determinism():
    p = lib()
    L = p.load_library()
    N = 10
    G = torch.from_numpy(workloads.iid_complex(N, 7, np.complex64)).cuda()
    outs = []
    for use_ws in (True, False, False, True):
        out = torch.empty(4 ** N, dtype=torch.complex64, device="cuda")
        ws = torch.empty(L.pauli_workspace_bytes(2, N, 1), dtype=torch.uint8, device="cuda") if use_ws else None
        o = p._opts("split_bf16", 0, 0, 0, stream(), ws)
        assert L.pauli_decompose(G.data_ptr(), N, 1, out.data_ptr(), ctypes.byref(o)) == 0
        outs.append(out)
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "fp64_gray"])
def test_complex128_in_and_out(algo):
    p = lib()
    N = 8
    G = workloads.iid_complex(N, 8)   # complex128
    c = p.decompose(torch.from_numpy(G).cuda(), algo=algo).cpu().numpy()
    assert c.dtype == np.complex128
    ref = oracle.decompose(G, threads=8)
    tol = {"split_bf16": 1e-6, "split_fp16": 1e-6, "fp32": 1e-5, "fp64_gray": 1e-12}[algo]
    assert np.abs(c - ref).max() / np.abs(ref).max() <= tol


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "fp64_gray"])
def test_nonfinite_input_propagates(algo):
    """A NaN on one XOR diagonal reaches exactly the coefficients of that flip
    mask; every other coefficient stays finite."""
    p = lib()
    N = 7
    G = workloads.iid_complex(N, 9, np.complex64)
    r, c = 5, 70
    G[r, c] = np.nan
    out = p.decompose(torch.from_numpy(G).cuda(), algo=algo).cpu().numpy()
    x_bad = r ^ c
    from tests import pauli_ref as pr
    bad = np.zeros(4 ** N, dtype=bool)
    for z in range(1 << N):
        bad[pr.n_of_xz(x_bad, z, N)] = True
    assert np.all(np.isfinite(out[~bad]))
    assert not np.any(np.isfinite(out[bad]))


@pytest.mark.parametrize("algo", ["split_bf16", "fwht"])
def test_concurrent_streams_do_not_share_scratch(algo):
    """Decompositions enqueued on two streams at once, with no ordering
    between them, each use their own cached scratch buffer: both results
    equal the eager ones."""
    import paper_2401_16378_amd as p
    p.load_library()
    N = 11
    A = torch.from_numpy(workloads.iid_complex(N, 1600, np.complex64)).cuda()
    B = torch.from_numpy(workloads.iid_complex(N, 1601, np.complex64)).cuda()
    want_a, want_b = p.decompose(A, algo=algo), p.decompose(B, algo=algo)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs_a, outs_b = [], []
    for _ in range(4):
        with torch.cuda.stream(s1):
            outs_a.append(p.decompose(A, algo=algo))
        with torch.cuda.stream(s2):
            outs_b.append(p.decompose(B, algo=algo))
    torch.cuda.synchronize()
    for a, b in zip(outs_a, outs_b):
        assert torch.equal(a, want_a) and torch.equal(b, want_b)


@pytest.mark.parametrize("algo", ["split_fp16", "fp64_gray", "fwht"])
def test_misaligned_complex64_view(algo):
    """A complex64 view that starts at an odd element (8 mod 16 bytes) is
    refused by the C ABI and realigned by the binding: the result equals the
    one for an aligned copy of the same values, bit for bit."""
    p = lib()
    L = p.load_library()
    N = 9
    G = torch.from_numpy(workloads.iid_complex(N, 31, np.complex64)).cuda()
    buf = torch.empty(4 ** N + 1, dtype=torch.complex64, device="cuda")
    buf[1:] = G.reshape(-1)
    view = buf[1:].view(1 << N, 1 << N)
    assert view.data_ptr() % 16 == 8
    out = torch.empty(4 ** N, dtype=torch.complex64, device="cuda")
    o = p._opts(algo, 0, 0, 0, stream(), p.workspace(algo, N, 1, G.device))
    assert L.pauli_decompose(view.data_ptr(), N, 1, out.data_ptr(), ctypes.byref(o)) == 1   # EINVAL
    a = p.decompose(view, algo=algo)
    b = p.decompose(G, algo=algo)
    assert torch.equal(a, b)
    assert view.data_ptr() % 16 == 8 and torch.equal(view, G)   # the caller's tensor is untouched
