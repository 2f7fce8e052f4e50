"""Fast Walsh-Hadamard algorithm (PAULI_ALGO_FWHT): all 4^N coefficients in
O(N 4^N) through a binary64 intermediate, and its adjoint (reconstruction,
gradient).  It is not the paper's evaluation
order, so it is held to the binary64 tolerance against the oracle (1e-12 of
max|c|), plus the exact one-hots, the Hermitian and Parseval invariants at
N = 14 and agreement with the binary64 Gray-code kernel.

PAULI_ALGO_FWHT_F32 rounds the intermediate to binary32: each coefficient is
held to its rounding bound (2^-24 times the 2-norm of the coefficients whose
partial transform the intermediate vector holds, per rounding) against the
oracle or the binary64 kernel; results that are exact in binary32 (one-hots,
small-integer Kronecker products) must stay exact."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests import pauli_ref as pr

pytestmark = pytest.mark.gpu


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def rel_err(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


def compact_even(v):
    v = v & 0x55555555
    v = (v | (v >> 1)) & 0x33333333
    v = (v | (v >> 2)) & 0x0F0F0F0F
    v = (v | (v >> 4)) & 0x00FF00FF
    return (v | (v >> 8)) & 0x0000FFFF


def rounding_bound(ref, N, roundings):
    """Per coefficient n = (x, z): roundings * 2^-24 * the 2-norm of the
    coefficients c(x, 32 k + (z & 31)) over k, the vector whose partial
    transform one binary32 intermediate row holds (test-side copy of the
    index mapping)."""
    xp = torch if isinstance(ref, torch.Tensor) else np
    if xp is torch:
        n = torch.arange(4 ** N, dtype=torch.int64, device=ref.device)
    else:
        n = np.arange(4 ** N, dtype=np.int64)
    z = compact_even(n >> 1)
    x = compact_even(n) ^ z
    key = (x << 5) | (z & 31)
    del n, x, z
    a2 = xp.abs(ref) ** 2
    if xp is torch:
        nrm = torch.zeros((1 << N) * 32, dtype=torch.float64, device=ref.device).index_add_(0, key, a2).sqrt()
    else:
        nrm = np.sqrt(np.bincount(key, weights=a2, minlength=(1 << N) * 32))
    return roundings * 2.0 ** -24 * nrm[key]


def check_f32_bound(got, ref, N):
    xp = torch if isinstance(ref, torch.Tensor) else np
    roundings = 1 if N <= 14 else 2   # N = 15, 16: one more rounding after the top pass
    bound = rounding_bound(ref, N, roundings)
    mx = xp.abs(ref).max()
    excess = xp.abs(got - ref) - (bound * (1 + 1e-6) + 1e-13 * mx)
    assert excess.max() <= 0, float(excess.max())


@pytest.mark.parametrize("N", [9, 10, 11, 12])
@pytest.mark.parametrize("in_dt", [np.complex64, np.complex128])
def test_full_vs_oracle(N, in_dt):
    p = lib()
    G = workloads.iid_complex(N, 1100 + N, in_dt)
    c = p.decompose(torch.from_numpy(G).cuda(), algo="fwht", out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.decompose(G, threads=threads())
    assert rel_err(c, ref) <= 1e-12


@pytest.mark.parametrize("N", [9, 10, 11, 12])
@pytest.mark.parametrize("in_dt", [np.complex64, np.complex128])
def test_f32_full_vs_oracle(N, in_dt):
    """The binary32 intermediate within its rounding bound, every
    coefficient, complex128 output (no output rounding)."""
    p = lib()
    G = workloads.iid_complex(N, 1100 + N, in_dt)
    c = p.decompose(torch.from_numpy(G).cuda(), algo="fwht_f32", out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.decompose(G, threads=threads())
    check_f32_bound(c, ref, N)
    assert rel_err(c, ref) <= 1e-6


@pytest.mark.parametrize("algo", ["fwht", "fwht_f32"])
def test_one_hot_exact(algo):
    p = lib()
    N = 9
    rng = np.random.default_rng(12)
    for m in list(rng.integers(0, 4 ** N, 6)) + [0, 4 ** N - 1]:
        P = torch.from_numpy(pr.pauli_string(int(m), N).astype(np.complex64)).cuda()
        c = p.decompose(P, algo=algo).cpu().numpy()
        e = np.zeros(4 ** N, np.complex64)
        e[int(m)] = 1
        assert np.array_equal(c, e), int(m)


def test_batch_and_complex64_out():
    p = lib()
    N = 10
    Gs = np.stack([workloads.iid_complex(N, 1200 + k, np.complex64) for k in range(3)])
    c = p.decompose(torch.from_numpy(Gs).cuda(), algo="fwht").cpu().numpy()
    assert c.shape == (3, 4 ** N) and c.dtype == np.complex64
    for k in range(3):
        assert rel_err(c[k], oracle.decompose(Gs[k])) <= 1e-6    # complex64 output rounding


def test_n14_vs_gray_and_invariants():
    """Precision workload at N = 14: against the binary64 Gray-code kernel in
    full, against the oracle on 8,192 sampled coefficients, Hermitian => real,
    Parseval sum |c|^2 = 2^-N ||G||_F^2."""
    p = lib()
    N = 14
    G = workloads.hermitian(N, workloads.SEED_N14)
    Gd = torch.from_numpy(G).cuda()
    c = p.decompose(Gd, algo="fwht", out_dtype=torch.complex128)
    g = p.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128)
    assert ((c - g).abs().max() / g.abs().max()).item() <= 1e-12
    ns = workloads.sample_indices(4 ** N, 8192, seed=workloads.SEED_SAMPLE)
    cs = c[torch.from_numpy(ns.astype(np.int64)).cuda()].cpu().numpy()
    assert rel_err(cs, oracle.coeffs_at(G, ns, threads=threads())) <= 1e-12
    assert (c.imag.abs().max() / c.abs().max()).item() <= 1e-12
    lhs = (c.abs() ** 2).sum().item()
    rhs = (Gd.to(torch.complex128).abs() ** 2).sum().item() / 2 ** N
    assert abs(lhs - rhs) <= 1e-12 * rhs


def test_f32_n14_vs_gray():
    """Precision workload at N = 14 with the binary32 intermediate: every
    coefficient within its rounding bound of the binary64 Gray-code kernel,
    Hermitian => real to binary32 rounding, and the complex64 result within
    1e-6 of max|c| (the split paths' bar)."""
    p = lib()
    N = 14
    Gd = torch.from_numpy(workloads.hermitian(N, workloads.SEED_N14)).cuda()
    g = p.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128)
    c = p.decompose(Gd, algo="fwht_f32", out_dtype=torch.complex128)
    check_f32_bound(c, g, N)
    mx = g.abs().max()
    assert ((c - g).abs().max() / mx).item() <= 1e-7
    del c
    c64 = p.decompose(Gd, algo="fwht_f32")
    assert ((c64.to(torch.complex128) - g).abs().max() / mx).item() <= 1e-6
    p.release_workspace()


def test_f32_n15_vs_binary64():
    """N = 15, random data: the binary32 intermediate is rounded twice (after
    pass 1 and after the top pass); every coefficient within twice its
    rounding bound of the binary64-intermediate result (itself held to the
    oracle by the exact Kronecker case and the sampled checks)."""
    p = lib()
    N = 15
    gen = torch.Generator(device="cuda").manual_seed(1515)
    G = torch.randn((1 << N, 1 << N), dtype=torch.complex64, device="cuda", generator=gen)
    ref = p.decompose(G, algo="fwht", out_dtype=torch.complex128)
    p.release_workspace()
    got = p.decompose(G, algo="fwht_f32", out_dtype=torch.complex128)
    del G
    p.release_workspace()
    check_f32_bound(got, ref, N)
    assert ((got - ref).abs().max() / ref.abs().max()).item() <= 2e-7
    del got, ref
    torch.cuda.empty_cache()


def test_reconstruct_vs_oracle_full_n9():
    p = lib()
    N = 9
    c = workloads.iid_complex(N, 1309, np.complex128).reshape(-1)
    G = p.reconstruct(torch.from_numpy(c).cuda(), algo="fwht").cpu().numpy()
    assert rel_err(G, oracle.recompose(c)) <= 1e-12


@pytest.mark.parametrize("which", ["reconstruct", "decompose_backward"])
@pytest.mark.parametrize("N", [9, 11])
def test_f32_adjoint_vs_oracle(which, N):
    """The adjoint through a binary32 intermediate: each entry y(x, i) =
    G[i ^ x][i] is within 2^-24 of the 2-norm of its 32 neighbours y(x, 32 i_h
    + l) per rounding, so within 2^-24 sqrt(32) max|G|."""
    p = lib()
    c = workloads.iid_complex(N, 1500 + N, np.complex128).reshape(-1)
    got = getattr(p, which)(torch.from_numpy(c).cuda(), algo="fwht_f32").cpu().numpy()
    rows, cols = workloads.sample_entries(1 << N, 1024, seed=1550 + N)
    r, q = rows.astype(np.int64), cols.astype(np.int64)
    ref = (oracle.recompose_entries if which == "reconstruct" else oracle.grad_entries)(c, rows, cols)
    full = (p.reconstruct if which == "reconstruct" else p.decompose_backward)(
        torch.from_numpy(c).cuda(), algo="fwht").cpu().numpy()
    bound = 2.0 ** -24 * np.sqrt(32) * np.abs(full).max()
    assert np.abs(got[r, q] - ref).max() <= bound * (1 + 1e-6)


@pytest.mark.parametrize("N", [10, 11, 12])
def test_reconstruct_vs_oracle_sampled(N):
    """Full recomposition by the oracle costs 8^N; 1,024 sampled entries
    (O(2^N) each) stand in at larger N."""
    p = lib()
    c = workloads.iid_complex(N, 1300 + N, np.complex128).reshape(-1)
    G = p.reconstruct(torch.from_numpy(c).cuda(), algo="fwht")
    rows, cols = workloads.sample_entries(1 << N, 1024, seed=1350 + N)
    r, q = torch.from_numpy(rows.astype(np.int64)).cuda(), torch.from_numpy(cols.astype(np.int64)).cuda()
    got = G[r, q].cpu().numpy()
    ref = oracle.recompose_entries(c, rows, cols)
    assert rel_err(got, ref) <= 1e-12


def test_backward_vs_oracle_entries():
    p = lib()
    N = 10
    g = workloads.iid_complex(N, 1400, np.complex128).reshape(-1)
    got = p.decompose_backward(torch.from_numpy(g).cuda(), algo="fwht").cpu().numpy()
    rows, cols = workloads.sample_entries(1 << N, 512, seed=1401)
    ref = oracle.grad_entries(g, rows, cols)
    assert rel_err(got[rows.astype(np.int64), cols.astype(np.int64)], ref) <= 1e-12


def test_round_trip_n14():
    """decompose then reconstruct at N = 14 returns G to binary64 rounding."""
    p = lib()
    N = 14
    Gd = torch.from_numpy(workloads.hermitian(N, workloads.SEED_N14)).cuda().to(torch.complex128)
    c = p.decompose(Gd, algo="fwht")
    G2 = p.reconstruct(c, algo="fwht")
    assert ((G2 - Gd).abs().max() / Gd.abs().max()).item() <= 1e-12


@pytest.mark.parametrize("N", [0, 5, 8])
def test_small_orders_same_for_f32(N):
    """Up to N = 8 there is no intermediate: both FWHT algorithms run the same
    binary64 kernel."""
    p = lib()
    G = torch.from_numpy(workloads.iid_complex(N, 1680 + N, np.complex128)).cuda()
    assert torch.equal(p.decompose(G, algo="fwht_f32"), p.decompose(G, algo="fwht"))
    c = G.reshape(-1)
    assert torch.equal(p.reconstruct(c, algo="fwht_f32"), p.reconstruct(c, algo="fwht"))


@pytest.mark.parametrize("N", list(range(0, 9)))
def test_small_orders_vs_oracle(N):
    """Up to N = 8 a single kernel works in LDS: forward and adjoint."""
    p = lib()
    G = workloads.iid_complex(N, 1600 + N, np.complex128)
    c = p.decompose(torch.from_numpy(G).cuda(), algo="fwht").cpu().numpy()
    assert rel_err(c, oracle.decompose(G)) <= 1e-12
    cc = workloads.iid_complex(N, 1650 + N, np.complex128).reshape(-1)
    R = p.reconstruct(torch.from_numpy(cc).cuda(), algo="fwht").cpu().numpy()
    if N <= 7:
        assert rel_err(R, oracle.recompose(cc)) <= 1e-12
    else:
        rows, cols = workloads.sample_entries(1 << N, 1024, seed=1660)
        ref = oracle.recompose_entries(cc, rows, cols)
        assert rel_err(R[rows.astype(np.int64), cols.astype(np.int64)], ref) <= 1e-12


@pytest.mark.parametrize("algo", ["fwht", "fwht_f32"])
def test_n15_exact_kronecker(algo):
    """N = 15 adds a pass over the top bit of i_h (N = 16, two bits, is in the
    maximum-size tests).  G = A (x) B with small integer parts (A 128 x 128,
    B 256 x 256) is exact in complex64 and its coefficients c(A) c(B) are
    dyadic, so binary64 butterflies must reproduce them exactly, and
    reconstruct must return G exactly; every partial sum is an integer below
    2^24, so the binary32 intermediate is exact too."""
    p = lib()
    rng = np.random.default_rng(1715)
    A = (rng.integers(-2, 3, (128, 128)) + 1j * rng.integers(-2, 3, (128, 128))).astype(np.complex64)
    B = (rng.integers(-2, 3, (256, 256)) + 1j * rng.integers(-2, 3, (256, 256))).astype(np.complex64)
    cA, cB = oracle.decompose(A), oracle.decompose(B)
    Gd = torch.kron(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    c = p.decompose(Gd, algo=algo, out_dtype=torch.complex128)
    ns = rng.integers(0, 4 ** 15, 65536, dtype=np.uint64)
    ns[:2] = [0, 4 ** 15 - 1]
    ref = cA[(ns >> 16).astype(np.int64)] * cB[(ns & 0xFFFF).astype(np.int64)]
    got = c[torch.from_numpy(ns.astype(np.int64)).cuda()].cpu().numpy()
    assert np.array_equal(got, ref)
    G2 = p.reconstruct(c, algo=algo, out_dtype=torch.complex128)
    assert torch.equal(G2, Gd.to(torch.complex128))
    del c, G2, Gd
    p.release_workspace()


@pytest.mark.parametrize("N", [6, 9, 10])
@pytest.mark.parametrize("which", ["reconstruct", "decompose_backward"])
def test_adjoint_dtype_combinations(N, which):
    """complex64 coefficients are widened exactly and every sum is binary64,
    so each input/output dtype pair equals the complex128 result (rounded
    once to binary32 for complex64 output) bit for bit; N = 6 takes the
    one-kernel path, N >= 9 the two passes."""
    p = lib()
    fn = getattr(p, which)
    c64 = workloads.iid_complex(N, 1700 + N, np.complex64).reshape(-1)
    c128 = c64.astype(np.complex128)
    ref = fn(torch.from_numpy(c128).cuda(), algo="fwht", out_dtype=torch.complex128)
    assert torch.equal(fn(torch.from_numpy(c64).cuda(), algo="fwht", out_dtype=torch.complex128), ref)
    ref64 = ref.to(torch.complex64)
    assert torch.equal(fn(torch.from_numpy(c64).cuda(), algo="fwht", out_dtype=torch.complex64), ref64)
    assert torch.equal(fn(torch.from_numpy(c128).cuda(), algo="fwht", out_dtype=torch.complex64), ref64)
