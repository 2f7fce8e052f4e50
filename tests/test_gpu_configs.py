"""GPU parity at the named workload sizes, in the launch configuration the
benchmark times (default tile, complex64 in and out for the MFMA paths).

Full-size outputs are checked element by element against the oracle on a
seeded sample of coefficients (the oracle computes them one by one), and over
all coefficients through properties that hold at any size: Parseval
(sum |c|^2 = 2^-N ||G||_F^2, globally and for every flip mask x), Hermitian
input => real coefficients, and agreement with the binary64 Gray kernel.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64_gray": 1e-12, "fp32": 1e-5, "split_bf16": 1e-6, "split_fp16": 1e-6}


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def flip_of_index(n: torch.Tensor) -> torch.Tensor:
    """x with bit t = bit(2t) ^ bit(2t+1) of n (test-side copy of the mapping)."""
    x = torch.zeros_like(n)
    for t in range(16):
        x |= (((n >> (2 * t)) ^ (n >> (2 * t + 1))) & 1) << t
    return x


def check_parseval(Gd: torch.Tensor, cd: torch.Tensor, tol: float):
    """Global and per-flip-mask Parseval identities, evaluated on the GPU in
    binary64 (test-side reductions only)."""
    N = Gd.shape[0].bit_length() - 1
    D = 1 << N
    a2 = cd.to(torch.complex128).abs() ** 2
    g2 = Gd.to(torch.complex128).abs() ** 2
    lhs, rhs = a2.sum().item(), g2.sum().item() / D
    assert abs(lhs - rhs) <= tol * rhs, (lhs, rhs)
    x_of_n = flip_of_index(torch.arange(D * D, device=cd.device, dtype=torch.int64))
    per_x = torch.zeros(D, dtype=torch.float64, device=cd.device).index_add_(0, x_of_n, a2)
    del x_of_n
    i = torch.arange(D, device=cd.device)
    ref = torch.empty(D, dtype=torch.float64, device=cd.device)
    for x in range(D):
        ref[x] = g2[i ^ x, i].sum()
    ref /= D
    assert (per_x - ref).abs().max().item() <= tol * ref.max().item()


@pytest.mark.parametrize("N", [12, 14])
def test_precision_configs(N):
    """Hermitian complex64, N=12 (4096^2) and N=14 (16384^2): every path on the
    same input; the full oracle at N=12, 65,536 seeded sampled coefficients at
    N=14; Parseval, real coefficients and cross-path agreement over all
    coefficients."""
    p = lib()
    seed = workloads.SEED_N12 if N == 12 else workloads.SEED_N14
    G = workloads.hermitian(N, seed)
    Gd = torch.from_numpy(G).to("cuda")
    outs = {}
    for algo in ("split_bf16", "split_fp16", "fp32"):
        outs[algo] = p.decompose(Gd, algo=algo).cpu().numpy()
    c64d = p.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128)
    outs["fp64_gray"] = c64d.cpu().numpy()
    check_parseval(Gd, c64d, 1e-10)
    del c64d
    check_parseval(Gd, torch.from_numpy(outs["split_bf16"]).to("cuda"), 1e-6)
    check_parseval(Gd, torch.from_numpy(outs["split_fp16"]).to("cuda"), 1e-6)
    del Gd
    torch.cuda.empty_cache()
    if N == 12:
        # every coefficient against the full oracle
        ref = oracle.decompose(G.astype(np.complex128), threads=threads())
        idx = np.arange(4 ** N, dtype=np.int64)
    else:
        # a seeded sample of 65,536 coefficients, computed one by one
        ns = workloads.sample_indices(4 ** N, 65536, seed=workloads.SEED_SAMPLE + N)
        ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=threads())
        idx = ns.astype(np.int64)
    mx = np.abs(ref).max()
    for algo, c in outs.items():
        err = np.abs(c[idx].astype(np.complex128) - ref).max() / mx
        assert err <= TOL[algo], (algo, err)
    # the binary64 kernel adds the same terms in the same order as the oracle
    assert np.array_equal(outs["fp64_gray"][idx], ref)
    # all coefficients against the binary64 kernel
    c64 = outs["fp64_gray"]
    m64 = np.abs(c64).max()
    for algo in ("split_bf16", "split_fp16", "fp32"):
        err = np.abs(outs[algo].astype(np.complex128) - c64).max() / m64
        assert err <= TOL[algo], (algo, err)
    # Hermitian => real coefficients
    assert np.abs(c64.imag).max() <= 1e-12 * m64
    assert np.abs(outs["split_bf16"].imag).max() <= 1e-6 * m64
    assert np.abs(outs["split_fp16"].imag).max() <= 1e-6 * m64


def test_n6_config():
    """N=6 complex128 iid (4096 coefficients): full oracle, every path; N=4
    cross-checked against brute force in the CPU suite."""
    p = lib()
    G = workloads.iid_complex(6, workloads.SEED_N6)
    ref = oracle.decompose(G)
    Gd = torch.from_numpy(G).to("cuda")
    for algo in TOL:
        c = p.decompose(Gd, algo=algo, out_dtype=torch.complex128).cpu().numpy()
        assert np.abs(c - ref).max() / np.abs(ref).max() <= TOL[algo], algo
        if algo == "fp64_gray":
            assert np.array_equal(c, ref)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16"])
def test_kronecker_full_size_n14(algo):
    """G = A (x) B at N=14 (A: N=7, B: N=7): c(G)[nA*4^7 + nB] = c(A)[nA] c(B)[nB]
    checked over all 2.7e8 coefficients of the output."""
    p = lib()
    A = workloads.iid_complex(7, 77, np.complex64)
    B = workloads.iid_complex(7, 78, np.complex64)
    G = torch.kron(torch.from_numpy(A).to("cuda"), torch.from_numpy(B).to("cuda"))
    c = p.decompose(G, algo=algo)
    cA = torch.from_numpy(oracle.decompose(A)).to("cuda")
    cB = torch.from_numpy(oracle.decompose(B)).to("cuda")
    ref = (cA[:, None] * cB[None, :]).reshape(-1)
    err = ((c.to(torch.complex128) - ref).abs().max() / ref.abs().max()).item()
    assert err <= 1e-6, err


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16"])
def test_one_hot_full_size_n14(algo):
    """G = P_m at N=14 for a few m: the output is exactly e_m (ordering, phase)."""
    p = lib()
    from tests import pauli_ref as pr
    rng = np.random.default_rng(14)
    for m in rng.integers(0, 4 ** 14, size=2):
        m = int(m)
        A = torch.from_numpy(pr.pauli_string(m & 0x3FFF, 7).astype(np.complex64)).to("cuda")
        B = torch.from_numpy(pr.pauli_string(m >> 14, 7).astype(np.complex64)).to("cuda")
        P = torch.kron(B, A)  # qubits 7..13 from m's high digits
        c = p.decompose(P, algo=algo)
        nz = torch.nonzero(c).flatten().cpu().numpy()
        assert list(nz) == [m]
        assert c[m].item() == 1
