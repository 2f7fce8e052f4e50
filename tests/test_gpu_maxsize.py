"""Largest order the library accepts, N = 16 (65536 x 65536, 2^32
coefficients, 32 GiB per complex64 operand): every offset into G, the packed
operand and the output passes 2^32 here.

G = A (x) B for two seeded 256 x 256 matrices with small integer parts, so
G is exact in complex64, c(G)_n = c(A)_{n >> 16} c(B)_{n & 0xFFFF} exactly
(the oracle's Kronecker pin), and every path computes these dyadic values
without rounding: split-bf16 (the integers sit on the hi grid, FP32 sums
stay below 2^24), binary32, the binary64 string list and the binary64 fast
Walsh-Hadamard path (whose 64 GiB intermediate replaces split-bf16's 48 GiB
workspace), and the Hermitian entry point on (A + A^H) (x) (B + B^H).
Sampled outputs are therefore compared for equality.  Needs about 180 GiB
of device memory.  The int8 path's largest exact sums are checked first, on
an all-equal matrix.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

N = 16


def small_int_matrix(seed):
    rng = np.random.default_rng(seed)
    re = rng.integers(-2, 3, (256, 256))
    im = rng.integers(-2, 3, (256, 256))
    return (re + 1j * im).astype(np.complex64)


def test_n16_int8_largest_sums():
    """The int8 path's extreme at N = 16: every component equal (G = (1 + i)
    J), so every q is the largest L and the phase mask z = 0 sums 2^16 equal
    digits, the largest |256 A2 + A1| the int32 fold can meet (2^16 x 32639 <
    2^31).  c = 1 + i for the 2^16 strings with z = 0 (any flip mask), 0 for
    all others.  Runs before the Kronecker fixture takes its memory."""
    import paper_2401_16378_amd as p
    p.load_library()
    print("N=16 int8 all-equal matrix", flush=True)
    G = torch.full((1 << N, 1 << N), 1 + 1j, dtype=torch.complex64, device="cuda")
    c = p.decompose(G, algo="split_i8")
    del G
    p.release_workspace()
    torch.cuda.synchronize()
    assert int((c != 0).sum().item()) == 1 << N
    # the strings with z = 0: n = spread_even(x), x < 2^16 (index them directly:
    # boolean-mask indexing of 2^32 elements is not usable in torch)
    x = np.arange(1 << N, dtype=np.int64)
    n = np.zeros_like(x)
    for t in range(N):
        n |= ((x >> t) & 1) << (2 * t)
    picked = c[torch.from_numpy(n).cuda()]
    assert bool(torch.all(picked == (1 + 1j)).item())
    del c, picked
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def kron_case():
    import paper_2401_16378_amd as p
    p.load_library()
    A, B = small_int_matrix(16001), small_int_matrix(16002)
    cA, cB = oracle.decompose(A), oracle.decompose(B)
    rng = np.random.default_rng(16003)
    ns = rng.integers(0, 4 ** N, 65536, dtype=np.uint64)
    ns[:4] = [0, 4 ** N - 1, 4 ** 8 - 1, (4 ** N - 1) ^ 0x5555]
    ref = cA[(ns >> 16).astype(np.int64)] * cB[(ns & 0xFFFF).astype(np.int64)]
    print("N=16 case: building G = A (x) B on the device", flush=True)
    G = torch.kron(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    assert G.shape == (1 << N, 1 << N) and G.dtype == torch.complex64
    yield p, G, ns, ref
    del G
    p.release_workspace()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "fwht", "fwht_f32"])
def test_n16_decompose_exact(kron_case, algo):
    p, G, ns, ref = kron_case
    print("N=16 decompose", algo, flush=True)
    c = p.decompose(G, algo=algo)
    assert c.shape == (4 ** N,)
    got = c[torch.from_numpy(ns.astype(np.int64)).cuda()].cpu().numpy()
    assert np.array_equal(got, ref.astype(np.complex64)), np.abs(got - ref).max()
    del c
    p.release_workspace()


def test_n16_coeffs_at_exact(kron_case):
    p, G, ns, ref = kron_case
    print("N=16 coeffs_at", flush=True)
    got = p.coeffs_at(G, ns.astype(np.uint32), out_dtype=torch.complex128).cpu().numpy()
    assert np.array_equal(got, ref)


def test_n16_reconstruct(kron_case):
    """The adjoint at full size: reconstruct from the exact coefficients and
    compare sampled entries of G (mid/lo planes carry the low bits, so this
    one is checked to the split-bf16 tolerance, not bit for bit)."""
    p, G, ns, ref = kron_case
    print("N=16 reconstruct", flush=True)
    c = p.decompose(G, algo="split_bf16")
    G2 = p.reconstruct(c, algo="split_bf16")
    del c
    rng = np.random.default_rng(16004)
    rows = torch.from_numpy(rng.integers(0, 1 << N, 4096)).cuda()
    cols = torch.from_numpy(rng.integers(0, 1 << N, 4096)).cuda()
    a, b = G[rows, cols], G2[rows, cols]
    err = ((a - b).abs().max() / G.abs().max()).item()
    assert err <= 1e-6, err
    assert torch.equal(G2[0, :64], G[0, :64]) or ((G2[0, :64] - G[0, :64]).abs().max() / G.abs().max()).item() <= 1e-6
    del G2
    p.release_workspace()


def test_n16_hermitian_exact(kron_case):
    """The Hermitian entry point at N = 16: H = (A + A^H) (x) (B + B^H) is
    Hermitian with integer entries of modulus <= 32, so the half walk's sums
    stay exact and c(H)_n = c(A_h)_{n >> 16} c(B_h)_{n & 0xFFFF} exactly
    (real), including the flip-mask blocks with the highest skipped bits."""
    p, _, ns, _ = kron_case
    print("N=16 Hermitian decompose", flush=True)
    A, B = small_int_matrix(16001), small_int_matrix(16002)
    Ah = (A + A.conj().T).astype(np.complex64)
    Bh = (B + B.conj().T).astype(np.complex64)
    cA, cB = oracle.decompose(Ah), oracle.decompose(Bh)
    ref = cA[(ns >> 16).astype(np.int64)] * cB[(ns & 0xFFFF).astype(np.int64)]
    H = torch.kron(torch.from_numpy(Ah).cuda(), torch.from_numpy(Bh).cuda())
    c = p.decompose_hermitian(H)
    del H
    got = c[torch.from_numpy(ns.astype(np.int64)).cuda()].cpu().numpy()
    assert np.array_equal(got, ref.astype(np.complex64)), np.abs(got - ref).max()
    assert torch.all(c.imag == 0)
    del c
    p.release_workspace()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", ["split_fp16", "split_bf16", "split_i8"])
def test_n15_random_vs_binary64(algo):
    """N = 15 on dense random data (no structure that keeps sums exact): every
    one of the 2^30 coefficients of the matrix-core path within 1e-6 of
    max|c| of the binary64 fast transform (itself held to the oracle to 1e-12
    elsewhere), and 256 seeded coefficients within 1e-6 of the oracle's own
    binary64 Gray-order sums."""
    import os
    import paper_2401_16378_amd as p
    p.load_library()
    n = 15
    gen = torch.Generator(device="cuda").manual_seed(1515 + len(algo))
    G = torch.randn((1 << n, 1 << n), dtype=torch.complex64, device="cuda", generator=gen)
    print("N=15 random: binary64 reference", flush=True)
    ref = p.decompose(G, algo="fwht", out_dtype=torch.complex128)
    p.release_workspace()
    print("N=15 random:", algo, flush=True)
    c = p.decompose(G, algo=algo)
    p.release_workspace()
    mx = ref.abs().max()
    err = ((c.to(torch.complex128) - ref).abs().max() / mx).item()
    assert err <= 1e-6, err
    ns = np.random.default_rng(1516).integers(0, 4 ** n, 256, dtype=np.uint64)
    Gh = G.cpu().numpy().astype(np.complex128)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    want = oracle.coeffs_at(Gh, ns, threads=threads)
    got = c[torch.from_numpy(ns.astype(np.int64)).cuda()].cpu().numpy()
    assert np.abs(got - want).max() / mx.item() <= 1e-6
    del G, ref, c, Gh
    torch.cuda.empty_cache()
