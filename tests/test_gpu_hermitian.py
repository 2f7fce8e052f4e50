"""Hermitian variant of the matrix-core decomposition (pauli_decompose_hermitian).

For Hermitian G every coefficient is real, and for a flip mask x the gathered
diagonal satisfies v_x[i ^ x] = conj(v_x[i]) (Eq. (c_def_in_terms_of_fn)), so
half of the i, doubled, carry the whole sum.  The result must match the
oracle to the tolerance of the general path (split-bf16 1e-6, binary32 1e-5
of max|c|), and every imaginary part must be exactly zero.  Flip-mask tiles
that walk half of K need 32*xb >= (unrolled step) * (K per slice); N = 11 and
above also exercise the longest unrolled step on half of K.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-6, "split_fp16": 1e-6}


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def rel_err(a, b):
    return float(np.abs(np.asarray(a) - b).max() / np.abs(b).max())


def herm_int(D, rng):
    """Hermitian matrix with small integer entries: exact in complex64."""
    A = rng.integers(-3, 4, (D, D)) + 1j * rng.integers(-3, 4, (D, D))
    H = A + A.conj().T
    return H.astype(np.complex64)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
@pytest.mark.parametrize("N", list(range(0, 11)))
def test_small_vs_oracle(algo, N):
    G = workloads.hermitian(N, 700 + N)
    c = lib().decompose_hermitian(torch.from_numpy(G).cuda(), algo=algo).cpu().numpy()
    ref = oracle.decompose(G.astype(np.complex128), threads=16)
    assert rel_err(c, ref) <= TOL[algo], rel_err(c, ref)
    assert np.all(c.imag == 0)


_REF10 = {}


def ref10():
    if "G" not in _REF10:
        G = workloads.hermitian(10, 710)
        _REF10["G"] = G
        _REF10["c"] = oracle.decompose(G.astype(np.complex128), threads=16)
    return _REF10["G"], _REF10["c"]


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
@pytest.mark.parametrize("tile", list(range(1, 16)))
def test_every_tile_n10(algo, tile):
    p = lib()
    G, ref = ref10()
    Gd = torch.from_numpy(G).cuda()
    if not p.tile_valid_hermitian(tile, 10, algo):
        with pytest.raises(p.PauliError):
            p.decompose_hermitian(Gd, algo=algo, tile=tile)
        return
    c = p.decompose_hermitian(Gd, algo=algo, tile=tile).cpu().numpy()
    assert rel_err(c, ref) <= TOL[algo]
    assert np.all(c.imag == 0)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
@pytest.mark.parametrize("N", [11, 12, 13])
def test_vs_binary64_and_sampled_oracle(algo, N):
    """All coefficients against the binary64 fast-transform path (itself
    pinned to the oracle), and a seeded sample against the oracle."""
    p = lib()
    G = workloads.hermitian(N, 720 + N)
    Gd = torch.from_numpy(G).cuda()
    c = p.decompose_hermitian(Gd, algo=algo).cpu().numpy()
    c64 = p.decompose(Gd, algo="fwht", out_dtype=torch.complex128).cpu().numpy()
    assert rel_err(c, c64) <= TOL[algo]
    assert np.all(c.imag == 0)
    ns = workloads.sample_indices(4 ** N, 2048, seed=workloads.SEED_SAMPLE + 50 + N)
    ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=16)
    idx = ns.astype(np.int64)
    assert np.abs(c[idx] - ref).max() <= TOL[algo] * np.abs(c64).max()


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
def test_kronecker_exact_n11(algo):
    """G = A (x) B with small-integer Hermitian parts: every partial sum is an
    exact small integer, so the coefficients must equal c(A) (x) c(B)
    exactly, the product of the oracle's (exact, dyadic) coefficients."""
    rng = np.random.default_rng(911)
    A, B = herm_int(64, rng), herm_int(32, rng)
    cA = oracle.decompose(A.astype(np.complex128))
    cB = oracle.decompose(B.astype(np.complex128))
    G = np.kron(A, B)
    c = lib().decompose_hermitian(torch.from_numpy(G).cuda(), algo=algo).cpu().numpy()
    n = np.arange(4 ** 11, dtype=np.int64)
    ref = cA[n >> 10] * cB[n & 1023]
    assert np.array_equal(c.astype(np.complex128), ref)


def test_batch_and_complex128_out():
    p = lib()
    Gs = np.stack([workloads.hermitian(8, 730 + k) for k in range(3)])
    c = p.decompose_hermitian(torch.from_numpy(Gs).cuda(), out_dtype=torch.complex128).cpu().numpy()
    assert c.shape == (3, 4 ** 8) and c.dtype == np.complex128
    for k in range(3):
        ref = oracle.decompose(Gs[k].astype(np.complex128), threads=16)
        assert rel_err(c[k], ref) <= 1e-6
        assert np.all(c[k].imag == 0)


def test_n14_config():
    """The N = 14 Hermitian workload: all coefficients against the binary64
    fast transform, a sample against the oracle, Parseval, agreement with the
    general split-bf16 path."""
    p = lib()
    N = 14
    G = workloads.hermitian(N, workloads.SEED_N14)
    Gd = torch.from_numpy(G).cuda()
    ch = p.decompose_hermitian(Gd)
    assert torch.all(ch.imag == 0)
    c64 = p.decompose(Gd, algo="fwht", out_dtype=torch.complex128)
    m = c64.abs().max().item()
    assert (ch.to(torch.complex128) - c64).abs().max().item() <= 1e-6 * m
    cg = p.decompose(Gd)
    assert (ch - cg).abs().max().item() <= 2e-6 * m
    # Parseval: sum |c|^2 = 2^-N ||G||_F^2
    lhs = (ch.to(torch.complex128).abs() ** 2).sum().item()
    rhs = (Gd.to(torch.complex128).abs() ** 2).sum().item() / 2 ** N
    assert abs(lhs - rhs) <= 1e-6 * rhs
    del cg, c64, Gd
    hc = ch.cpu().numpy()
    del ch
    p.release_workspace()
    torch.cuda.empty_cache()
    ns = workloads.sample_indices(4 ** N, 4096, seed=workloads.SEED_SAMPLE + 77)
    ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=16)
    assert np.abs(hc[ns.astype(np.int64)] - ref).max() <= 1e-6 * m


def test_requires_grad_refused():
    p = lib()
    G = torch.from_numpy(workloads.hermitian(4, 5)).cuda().requires_grad_()
    with pytest.raises(ValueError):
        p.decompose_hermitian(G)


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
def test_complex128_input(algo):
    """complex128 input is read rounded to binary32 (as for every matrix-core
    path): the same coefficients as the complex64 copy of the matrix."""
    p = lib()
    G64 = workloads.hermitian(9, 740)
    G128 = torch.from_numpy(G64.astype(np.complex128)).cuda()
    a = p.decompose_hermitian(G128, algo=algo, out_dtype=torch.complex128)
    b = p.decompose_hermitian(torch.from_numpy(G64).cuda(), algo=algo, out_dtype=torch.complex128)
    assert torch.equal(a, b)
    ref = oracle.decompose(G64.astype(np.complex128), threads=16)
    assert rel_err(a.cpu().numpy(), ref) <= TOL[algo]


def test_explicit_workspace_and_stream():
    """The C entry point with a caller workspace on a side stream."""
    import ctypes
    p = lib()
    N = 9
    G = torch.from_numpy(workloads.hermitian(N, 741)).cuda()
    want = p.decompose_hermitian(G)
    need = p.load_library().pauli_workspace_bytes(p.ALGOS["split_bf16"], N, 1)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = torch.empty(4 ** N, dtype=torch.complex64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    o = p._opts("split_bf16", 0, 0, 0, ctypes.c_void_p(s.cuda_stream), ws)
    assert p.load_library().pauli_decompose_hermitian(G.data_ptr(), N, 1, out.data_ptr(), ctypes.byref(o)) == 0
    s.synchronize()
    assert torch.equal(out, want)


def _nan_workspace(p, algo, N, batch=1):
    need = p.load_library().pauli_workspace_bytes(p.ALGOS[algo], N, batch)
    return torch.full((need,), 0xFF, dtype=torch.uint8, device="cuda")   # NaN in bf16 and binary32


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
@pytest.mark.parametrize("N", [9, 10, 12])
def test_pack_skips_only_unread_parts(algo, N):
    """The Hermitian pack leaves the K ranges that no tile's half walk reads
    unwritten: on a workspace of NaN bytes every tile must still give the
    oracle's coefficients (a read of an unpacked part would show as NaN)."""
    import ctypes
    p = lib()
    G = workloads.hermitian(N, 750 + N)
    Gd = torch.from_numpy(G).cuda()
    ns = workloads.sample_indices(4 ** N, 2048, seed=workloads.SEED_SAMPLE + 90 + N)
    ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=16)
    idx = torch.from_numpy(ns.astype(np.int64)).cuda()
    for tile in range(1, 13):
        if not p.tile_valid_hermitian(tile, N, algo):
            continue
        ws = _nan_workspace(p, algo, N)
        out = torch.empty(4 ** N, dtype=torch.complex64, device="cuda")
        o = p._opts(algo, 0, 0, tile, p._stream(Gd), ws)
        assert p.load_library().pauli_decompose_hermitian(Gd.data_ptr(), N, 1, out.data_ptr(), ctypes.byref(o)) == 0
        c = out.cpu().numpy()
        assert np.all(np.isfinite(c)), (algo, N, tile)
        assert np.abs(c[ns.astype(np.int64)] - ref).max() <= TOL[algo] * np.abs(ref).max(), (algo, N, tile)
        del ws


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32"])
def test_split_passes_any_contraction_tile(algo):
    """pauli_pack mode 3 does not depend on the tile: a contraction with any
    register-ring tile after it equals the one-call Hermitian entry point."""
    import ctypes
    p = lib()
    N = 11
    G = torch.from_numpy(workloads.hermitian(N, 760)).cuda()
    lib_ = p.load_library()
    for tile in (1, 3, 6, 9, 12):
        if not p.tile_valid_hermitian(tile, N, algo):
            continue
        want = p.decompose_hermitian(G, algo=algo, tile=tile)
        ws = _nan_workspace(p, algo, N)
        out = torch.empty(4 ** N, dtype=torch.complex64, device="cuda")
        pack_o = p._opts(algo, 0, 0, 0, p._stream(G), ws)            # default tile for the pack
        cont_o = p._opts(algo, 0, 0, tile, p._stream(G), ws)
        assert lib_.pauli_pack(G.data_ptr(), N, 1, 3, ctypes.byref(pack_o)) == 0
        assert lib_.pauli_contract(N, 1, 3, out.data_ptr(), ctypes.byref(cont_o)) == 0
        assert torch.equal(out, want), (algo, tile)


@pytest.mark.parametrize("algo", ["split_fp16", "split_bf16"])
def test_row_pairs_complex128_every_tile_n11(algo):
    """The row-halved tiles (2^b >= the tile's rows) with complex128 output,
    whose second output stage doubles a larger LDS area (and the 8-wave tile,
    where two stages of 16-byte values do not fit and no rows are paired):
    every register-ring tile at N = 11 gives complex64 output equal to its
    complex128 output rounded, and the complex128 output within the split
    tolerance of the binary64 fast transform, with zero imaginary parts."""
    p = lib()
    N = 11
    Gd = torch.from_numpy(workloads.hermitian(N, 1111)).cuda()
    ref = p.decompose(Gd, algo="fwht", out_dtype=torch.complex128)
    m = ref.abs().max().item()
    for tile in range(1, 13):
        if not p.tile_valid_hermitian(tile, N, algo):
            continue
        c128 = p.decompose_hermitian(Gd, algo=algo, tile=tile, out_dtype=torch.complex128)
        c64 = p.decompose_hermitian(Gd, algo=algo, tile=tile)
        assert torch.equal(c64, c128.to(torch.complex64)), tile
        assert torch.all(c128.imag == 0), tile
        assert (c128 - ref).abs().max().item() <= TOL[algo] * m, tile
