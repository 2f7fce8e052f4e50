"""pauli_decompose_noalloc (the entry point for callers that cannot allocate
device memory) against pauli_decompose, through the C ABI: the same kernels
run on the library's fixed per-GPU scratch instead of a workspace, so the
results must agree bit for bit.  Two calls in a row per algorithm, the second
with a smaller matrix (the scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

ALGOS = {"split_bf16": 2, "split_fp16": 4, "fp32": 1, "fwht": 3, "fwht_f32": 5, "fp64_gray": 0, "split_i8": 6}


def lib():
    import paper_2401_16378_amd as p
    return p, p.load_library()


def call(fn, G, N, batch, algo, out_dtype):
    p, L = lib()
    out = torch.empty(batch * (1 << (2 * N)), dtype=out_dtype, device=G.device)
    o = p._Opts()
    L.pauli_opts_default(ctypes.byref(o))
    o.algo = ALGOS[algo]
    o.in_dtype = 0 if G.dtype == torch.complex64 else 1
    o.out_dtype = 0 if out_dtype == torch.complex64 else 1
    o.stream = torch.cuda.current_stream().cuda_stream
    if fn == "pauli_decompose":
        need = L.pauli_workspace_bytes(o.algo, N, batch)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=G.device)
        o.workspace = ws.data_ptr()
        o.workspace_bytes = need
    st = getattr(L, fn)(G.data_ptr(), N, batch, out.data_ptr(), ctypes.byref(o))
    assert st == 0, (fn, algo, N, p.last_error())
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("algo", list(ALGOS))
def test_noalloc_matches_decompose(algo):
    p, L = lib()
    assert L.pauli_noalloc_scratch_bytes() == 64 << 20
    in_dt = torch.complex128 if algo in ("fp64_gray", "fwht") else torch.complex64
    for N, batch, seed in ((11, 1, 7100), (9, 2, 7101)):   # second call smaller
        need = L.pauli_workspace_bytes(ALGOS[algo], N, batch)
        assert need <= L.pauli_noalloc_scratch_bytes()
        G = workloads.iid_complex_batch(N, batch, seed, np.complex64)
        Gd = torch.from_numpy(G).to("cuda").to(in_dt)
        ref = call("pauli_decompose", Gd, N, batch, algo, in_dt)
        got = call("pauli_decompose_noalloc", Gd, N, batch, algo, in_dt)
        assert torch.equal(got, ref), (algo, N, batch)


def test_noalloc_refuses_oversized_requests():
    p, L = lib()
    G = torch.zeros(1 << 12, 1 << 12, dtype=torch.complex64, device="cuda")
    out = torch.empty(1 << 24, dtype=torch.complex64, device="cuda")
    o = p._Opts()
    L.pauli_opts_default(ctypes.byref(o))   # split-bf16: 12 bytes per element, 192 MiB at N = 12
    assert L.pauli_decompose_noalloc(G.data_ptr(), 12, 1, out.data_ptr(), ctypes.byref(o)) == 4
    assert "fixed scratch" in p.last_error()
