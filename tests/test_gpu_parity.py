"""GPU parity of every algorithm against the CPU oracle, through the C ABI.

Tolerances (error = max_n |c_n - oracle_n| / max_n |oracle_n|): binary64 Gray
kernel 1e-12 (and expected bit-identical: it adds the same terms in the same
Gray order), binary32 MFMA 1e-5, split-bf16 MFMA 1e-6.  Coefficient ordering
is checked bit-exactly with one-hot Pauli strings, whose coefficients are
exact small integers in every precision.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests import pauli_ref as pr

pytestmark = pytest.mark.gpu

TOL = {"fp64_gray": 1e-12, "fp32": 1e-5, "split_bf16": 1e-6, "split_fp16": 1e-6}
ALGOS = list(TOL)


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("N", list(range(0, 9)))
def test_gray_bitexact_small(N):
    G = workloads.iid_complex(N, 500 + N)
    c = lib().decompose(dev(G), algo="fp64_gray").cpu().numpy()
    ref = oracle.decompose(G, threads=8)
    assert rel_err(c, ref) <= TOL["fp64_gray"]
    assert np.array_equal(c, ref), "binary64 Gray kernel differs from the Gray-order oracle sum"


def test_gray_n10_config():
    """N=10, complex128 iid: full oracle, <= 1e-12 and bit-identical."""
    G = workloads.iid_complex(10, workloads.SEED_N10)
    c = lib().decompose(dev(G), algo="fp64_gray").cpu().numpy()
    ref = oracle.decompose(G, threads=16)
    assert rel_err(c, ref) <= 1e-12
    assert np.array_equal(c, ref)


@pytest.mark.parametrize("algo", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("N", list(range(0, 10)))
def test_mfma_small(algo, N):
    G = workloads.iid_complex(N, 600 + N, np.complex64)
    c = lib().decompose(dev(G), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.decompose(G, threads=8)
    assert rel_err(c, ref) <= TOL[algo]


@pytest.mark.parametrize("algo", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("tile", list(range(1, 16)))
def test_mfma_every_tile_n9(algo, tile):
    p = lib()
    N = 9
    if not p.tile_valid(tile, N, algo):
        assert algo == "fp32" and tile in (1, 2, 7, 10, 11)
        with pytest.raises(p.PauliError):
            p.decompose(dev(workloads.iid_complex(N, 700, np.complex64)), algo=algo, tile=tile)
        return
    G = workloads.iid_complex(N, 700 + tile, np.complex64)
    c = p.decompose(dev(G), algo=algo, tile=tile).cpu().numpy()
    ref = oracle.decompose(G, threads=8)
    assert rel_err(c, ref) <= TOL[algo]


@pytest.mark.parametrize("algo", ["fp32", "split_bf16", "split_fp16"])
def test_tiles_bitexact_n10(algo):
    """Every tile shape sums the K slices of an output element in the same
    order, so all of them (register-ring and LDS-staged alike) must agree bit
    for bit, in both directions."""
    p = lib()
    N = 10
    assert p.tile_count(algo) == 15
    G = dev(workloads.iid_complex(N, 710, np.complex64))
    c = dev(workloads.iid_complex(N, 711, np.complex64).reshape(-1))
    tiles = [t for t in range(1, 16) if p.tile_valid(t, N, algo)]
    assert len(tiles) == (10 if algo == "fp32" else 15)
    ref_f = p.decompose(G, algo=algo, tile=tiles[0])
    ref_a = p.reconstruct(c, algo=algo, tile=tiles[0])
    for tile in tiles[1:]:
        assert torch.equal(p.decompose(G, algo=algo, tile=tile), ref_f), tile
        assert torch.equal(p.reconstruct(c, algo=algo, tile=tile), ref_a), tile


@pytest.mark.parametrize("algo", ALGOS)
def test_one_hot_ordering(algo):
    p = lib()
    for N in (1, 2, 3):
        for m in range(4 ** N):
            P = pr.pauli_string(m, N).astype(np.complex64)
            c = p.decompose(dev(P), algo=algo).cpu().numpy()
            e = np.zeros(4 ** N, dtype=np.complex64)
            e[m] = 1
            assert np.array_equal(c, e), (algo, N, m)
    rng = np.random.default_rng(5)
    for N in (6, 9):
        for m in rng.integers(0, 4 ** N, size=4):
            P = pr.pauli_string(int(m), N).astype(np.complex64)
            c = p.decompose(dev(P), algo=algo).cpu().numpy()
            e = np.zeros(4 ** N, dtype=np.complex64)
            e[int(m)] = 1
            assert np.array_equal(c, e), (algo, N, int(m))


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("N", [1, 3, 6, 9])
def test_reconstruct_roundtrip(algo, N):
    p = lib()
    c = workloads.iid_complex(N, 800 + N).reshape(-1).astype(np.complex64)
    G = p.reconstruct(dev(c), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.recompose(c) if N <= 6 else None
    if ref is not None:
        assert rel_err(G, ref) <= TOL[algo]
    # decompose(reconstruct(c)) == c
    c2 = p.decompose(dev(G.astype(np.complex128)), algo="fp64_gray").cpu().numpy()
    assert rel_err(c2, c) <= max(TOL[algo], 1e-12) * 4


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("N", [2, 5, 8])
def test_backward_vs_oracle_grad(algo, N):
    p = lib()
    gc = workloads.iid_complex(N, 900 + N).reshape(-1).astype(np.complex64)
    g = p.decompose_backward(dev(gc), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    D = 1 << N
    rows, cols = workloads.sample_entries(D, min(D * D, 256), seed=N)
    ref = oracle.grad_entries(gc, rows, cols)
    got = g[rows.astype(np.int64), cols.astype(np.int64)]
    assert np.abs(got - ref).max() <= TOL[algo] * 4 * np.abs(ref).max()


@pytest.mark.parametrize("algo", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("N", [2, 5, 6, 9])
def test_adjoint_complex128_coefficients(algo, N):
    """The matrix-core adjoint reads complex128 coefficients rounded to
    binary32: reconstruction and gradient equal those of the complex64 copy
    bit for bit, and the reconstruction matches the oracle's recomposition.
    N = 2 is padded; N = 5 and 6 fill one and two waves of a pack tile."""
    p = lib()
    c128 = workloads.iid_complex(N, 950 + N).reshape(-1)
    c64 = c128.astype(np.complex64)
    for fn in (p.reconstruct, p.decompose_backward):
        a = fn(dev(c128), algo=algo, out_dtype=torch.complex128)
        b = fn(dev(c64), algo=algo, out_dtype=torch.complex128)
        assert torch.equal(a, b), fn.__name__
    G = p.reconstruct(dev(c128), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.recompose(c64)
    assert rel_err(G, ref) <= TOL[algo]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("which", ["decompose", "reconstruct", "decompose_backward"])
def test_dtype_combinations(algo, which):
    """Every input/output dtype pair of every entry point.  Each path forms a
    result in binary64 and rounds it once for complex64 output; complex64
    input is widened exactly.  So for values representable in binary32 all
    four pairs follow from one result bit for bit.  The matrix-core
    algorithms read complex128 input rounded to binary32, so a general
    complex128 input gives the result of its complex64 rounding."""
    p = lib()
    fn = getattr(p, which)
    N = 7
    x64 = workloads.iid_complex(N, 1800 + N, np.complex64)
    if which != "decompose":
        x64 = x64.reshape(-1)
    x128 = x64.astype(np.complex128)
    ref = fn(dev(x64), algo=algo, out_dtype=torch.complex128)
    assert torch.equal(fn(dev(x128), algo=algo, out_dtype=torch.complex128), ref)
    ref64 = ref.to(torch.complex64)
    assert torch.equal(fn(dev(x64), algo=algo, out_dtype=torch.complex64), ref64)
    assert torch.equal(fn(dev(x128), algo=algo, out_dtype=torch.complex64), ref64)
    if algo != "fp64_gray":
        y128 = workloads.iid_complex(N, 1850 + N)
        if which != "decompose":
            y128 = y128.reshape(-1)
        assert torch.equal(fn(dev(y128), algo=algo, out_dtype=torch.complex128),
                           fn(dev(y128.astype(np.complex64)), algo=algo, out_dtype=torch.complex128))


@pytest.mark.parametrize("algo", ALGOS)
def test_batch_dimension(algo):
    p = lib()
    N = 6
    Gs = workloads.iid_complex_batch(N, 3, 1234)
    c = p.decompose(dev(Gs), algo=algo).cpu().numpy()
    for b in range(3):
        c1 = p.decompose(dev(Gs[b]), algo=algo).cpu().numpy()
        assert np.array_equal(c[b], c1)
