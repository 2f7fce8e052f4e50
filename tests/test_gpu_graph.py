"""Capturing the library's calls in a HIP graph (torch.cuda.graph): decompose
and reconstruct enqueue only kernels on the caller's stream (the packed
operand lives in a caller-provided workspace), so a captured graph must
reproduce the eager result bit for bit on every replay, also with unrelated
eager work, synchronisations and new input values in between."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "fp64_gray", "fwht", "split_i8"])
def test_capture_and_replay(algo):
    p = lib()
    adjoint = algo != "split_i8"   # the int8 path is forward only
    N = 10
    G = torch.from_numpy(workloads.iid_complex(N, 1500, np.complex64)).cuda()
    G2 = torch.from_numpy(workloads.iid_complex(N, 1501, np.complex64)).cuda()
    eager = p.decompose(G, algo=algo)
    eager2 = p.decompose(G2, algo=algo)
    back = p.reconstruct(eager, algo=algo) if adjoint else None
    torch.cuda.synchronize()

    src = G.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                   # warm-up on the capture stream (workspace cached)
        p.decompose(src, algo=algo)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c = p.decompose(src, algo=algo)
        r = p.reconstruct(c, algo=algo) if adjoint else None
    for rep in range(4):
        junk = torch.randn(1 << 18, device="cuda").sum()   # eager work between replays
        src.copy_(G if rep % 2 == 0 else G2)
        g.replay()
        torch.cuda.synchronize()
        want = eager if rep % 2 == 0 else eager2
        assert torch.equal(c, want), (algo, rep)
        if adjoint and rep % 2 == 0:
            assert torch.equal(r, back), (algo, rep)
        del junk
    del g


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "split_i8"])
def test_capture_and_replay_hermitian(algo):
    """The Hermitian entry point enqueues the same two kernels (pack, then
    the Hermitian contraction): captured, it must match the eager result on
    every replay."""
    p = lib()
    N = 10
    H = torch.from_numpy(workloads.hermitian(N, 1502)).cuda()
    H2 = torch.from_numpy(workloads.hermitian(N, 1503)).cuda()
    eager = p.decompose_hermitian(H, algo=algo)
    eager2 = p.decompose_hermitian(H2, algo=algo)
    torch.cuda.synchronize()
    src = H.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.decompose_hermitian(src, algo=algo)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c = p.decompose_hermitian(src, algo=algo)
    for rep in range(4):
        junk = torch.randn(1 << 18, device="cuda").sum()
        src.copy_(H if rep % 2 == 0 else H2)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(c, eager if rep % 2 == 0 else eager2), (algo, rep)
        del junk
    del g
