"""The fixed-point int8 path (split_i8) through the C ABI: decomposition,
its Hermitian variant, reconstruction and the backward (adjoint).

Against the oracle: every coefficient at N = 0..10 (ragged N < 5 padded to
32, the one-slice-at-a-time kernel below N = 8) and at the N = 12 Hermitian
workload, a seeded 65,536-coefficient sample at N = 14 plus all coefficients
against the binary64 Gray kernel.  The bar is the decomposition's 1e-6 of
max|c| and, for every input, the path's own bound: the quantisation moves
each component of G by at most m / (2L) (m the largest |Re|, |Im| of the
matrix, L = 8355711), so each coefficient is off by at most sqrt(2) m / (2L)
in modulus, plus the output's rounding.

Exact properties: the int8 sums are exact integers, so wherever the
quantisation itself is exact the result is the oracle's up to the final
scaling, and the conjugate, transpose and power-of-two scaling identities
hold bit for bit (the quantised matrix transforms the same way).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

L8 = 8355711.0


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def dec(G, out_dtype=None):
    return lib().decompose(dev(G), algo="split_i8", out_dtype=out_dtype).cpu().numpy()


def bound(G, ref, out_dtype):
    """The path's error bound in modulus: quantisation + output rounding."""
    m = max(np.abs(G.real).max(), np.abs(G.imag).max())
    rnd = (2.0 ** -24 if out_dtype == torch.complex64 else 2.0 ** -52) * np.abs(ref).max()
    return np.sqrt(2.0) * (m / (2 * L8) + rnd) * (1 + 1e-9)


def check(G, c, ref, out_dtype):
    err = np.abs(c.astype(np.complex128) - ref).max()
    assert err <= bound(G, ref, out_dtype), (err, bound(G, ref, out_dtype))
    return err / np.abs(ref).max()


@pytest.mark.parametrize("N", list(range(0, 11)))
def test_vs_oracle(N):
    G = workloads.iid_complex(N, 8800 + N, np.complex64)
    ref = oracle.decompose(G.astype(np.complex128), threads=threads())
    rel = check(G, dec(G), ref, torch.complex64)
    assert rel <= 1e-6, rel


@pytest.mark.parametrize("N", [3, 7, 10])
def test_complex128_in_and_out(N):
    """Binary64 input is quantised from its binary64 values (the scale is
    taken in binary64 too), binary64 output keeps the exact sums' scaling."""
    G = workloads.iid_complex(N, 8850 + N, np.complex128)
    ref = oracle.decompose(G, threads=threads())
    rel = check(G, dec(G, torch.complex128), ref, torch.complex128)
    assert rel <= 1e-6, rel


def test_n12_hermitian_full():
    """The N = 12 Hermitian workload, every coefficient; Hermitian input gives
    exactly real coefficients (each pair i, i ^ x sums to a real or an
    imaginary integer before the phase)."""
    G = workloads.hermitian(12, workloads.SEED_N12)
    c = dec(G)
    ref = oracle.decompose(G.astype(np.complex128), threads=threads())
    rel = check(G, c, ref, torch.complex64)
    assert rel <= 1e-6, rel
    assert np.all(c.imag == 0)


def test_n14_hermitian_sample_and_gray():
    """The N = 14 Hermitian workload in the benchmark's launch configuration:
    65,536 seeded coefficients against the oracle, all coefficients against
    the binary64 Gray kernel, exactly real, Parseval."""
    p = lib()
    N = 14
    G = workloads.hermitian(N, workloads.SEED_N14)
    Gd = dev(G)
    c = p.decompose(Gd, algo="split_i8").cpu().numpy()
    c64 = p.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128).cpu().numpy()
    g2 = float((Gd.to(torch.complex128).abs() ** 2).sum().item()) / (1 << N)
    del Gd
    torch.cuda.empty_cache()
    ns = workloads.sample_indices(4 ** N, 65536, seed=workloads.SEED_SAMPLE + N)
    ref = oracle.coeffs_at(G.astype(np.complex128), ns, threads=threads())
    idx = ns.astype(np.int64)
    err = np.abs(c[idx].astype(np.complex128) - ref).max()
    assert err <= bound(G, ref, torch.complex64)
    assert err / np.abs(ref).max() <= 1e-6
    rel = check(G, c, c64, torch.complex64)
    assert rel <= 1e-6, rel
    assert np.all(c.imag == 0)
    s = float((np.abs(c.astype(np.complex128)) ** 2).sum())
    assert abs(s - g2) <= 1e-6 * g2
    # the Hermitian entry point (a quarter of the walks) gives the same exact sums
    ch = p.decompose_hermitian(dev(G), algo="split_i8").cpu().numpy()
    assert np.array_equal(ch, c)


def test_exact_when_quantisation_is():
    """Components in {0, +-1} 2^5 (the largest a power of two, so every q is 0
    or +-L): the sums are exact and only the last scaling rounds."""
    N = 9
    rng = np.random.default_rng(8900)
    G = (rng.integers(-1, 2, (1 << N, 1 << N)) + 1j * rng.integers(-1, 2, (1 << N, 1 << N))) * 32.0
    G[0, 0] = 32.0
    ref = oracle.decompose(G, threads=threads())
    c = dec(G, torch.complex128)
    assert np.abs(c - ref).max() <= 4e-16 * np.abs(ref).max()


@pytest.mark.parametrize("N", [1, 3])
def test_one_hot_strings_exact(N):
    """G = P_m gives c = e_m exactly (complex64 output), for every m."""
    D = 1 << N
    for m in range(4 ** N):
        P = np.array([[oracle.pauli_element(m, N, i, j) for j in range(D)] for i in range(D)], np.complex64)
        c = dec(P)
        want = np.zeros(4 ** N, np.complex64)
        want[m] = 1
        assert np.array_equal(c, want), m


def test_conjugate_transpose_and_scaling_bit_exact():
    """c(G^H) = conj c(G) and c(G^T)_n = (-1)^{#Y(n)} c(G)_n bit for bit, and
    c(2^k G) = 2^k c(G) bit for bit (the quantised integers are the same)."""
    N = 9
    G = workloads.iid_complex(N, 8910, np.complex128)
    c = dec(G, torch.complex128)
    n = np.arange(4 ** N)
    ny = np.zeros_like(n)                      # number of Y operators in string n
    for t in range(N):
        b0, b1 = (n >> (2 * t)) & 1, (n >> (2 * t + 1)) & 1
        ny += (b0 ^ b1) & b1                   # Y on qubit t: x_t = z_t = 1
    sign = np.where(ny & 1, -1.0, 1.0)
    assert np.array_equal(dec(G.conj().T, torch.complex128), c.conj())
    assert np.array_equal(dec(G.T, torch.complex128), sign * c)
    for k in (-40, 40):
        assert np.array_equal(dec(np.ldexp(G.real, k) + 1j * np.ldexp(G.imag, k), torch.complex128),
                              np.ldexp(c.real, k) + 1j * np.ldexp(c.imag, k))


def test_batch_scales_are_per_matrix():
    """A batch of matrices 2^40 apart in size: each member equals its own
    single call bit for bit (one scale record per matrix)."""
    p = lib()
    N = 8
    mats = [workloads.iid_complex(N, 8920 + k, np.complex128) * 2.0 ** (40 * (k - 1)) for k in range(3)]
    B = dev(np.stack(mats))
    cb = p.decompose(B, algo="split_i8").cpu().numpy()
    for k, G in enumerate(mats):
        assert np.array_equal(cb[k], dec(G)), k


def test_zero_and_non_finite():
    """An all-zero matrix gives zeros; an infinite or NaN component makes every
    coefficient of its matrix NaN and leaves the other batch members alone."""
    p = lib()
    N = 6
    D = 1 << N
    assert np.array_equal(dec(np.zeros((D, D), np.complex64)), np.zeros(D * D, np.complex64))
    G = workloads.iid_complex(N, 8930, np.complex64)
    good = dec(G)
    for bad in (np.inf, -np.inf, np.nan):
        H = G.copy()
        H[3, 5] = complex(1.0, bad)
        cb = p.decompose(dev(np.stack([H, G])), algo="split_i8").cpu().numpy()
        assert np.all(np.isnan(cb[0].real)) and np.all(np.isnan(cb[0].imag))
        assert np.array_equal(cb[1], good)


def test_mixed_magnitudes_within_the_fixed_point_bound():
    """Rows scaled by 2^-20 .. 2^20: entries far below the largest one keep
    only the absolute precision m / (2L), so the error relative to max|c| can
    exceed the floating-point splits' while staying within the stated bound."""
    N = 9
    D = 1 << N
    G = workloads.iid_complex(N, 8940, np.complex128)
    G *= np.ldexp(1.0, np.random.default_rng(8941).integers(-20, 21, D))[:, None]
    ref = oracle.decompose(G, threads=threads())
    check(G, dec(G, torch.complex128), ref, torch.complex128)


def test_batched_refused():
    """The uneven-batch entry point refuses the algorithm (PAULI_EUNSUPPORTED)
    without launching anything."""
    p = lib()
    G = dev(workloads.iid_complex(6, 8950, np.complex64))
    with pytest.raises(p.PauliError) as e:
        p.decompose_batched([G], algo="split_i8")
    assert e.value.status == 2


def adjoint_bound(c, ref, out_dtype, scale):
    """Each entry of the adjoint sums 2^N quantised terms: at most 2^N m / (2L)
    per component (m the largest component of c), times the scale, plus the
    output's rounding."""
    m = max(np.abs(c.real).max(), np.abs(c.imag).max())
    n = c.shape[-1]
    D = int(round(np.sqrt(n)))
    rnd = (2.0 ** -24 if out_dtype == torch.complex64 else 2.0 ** -52) * np.abs(ref).max()
    return np.sqrt(2.0) * (scale * D * m / (2 * L8) + rnd) * (1 + 1e-9)


@pytest.mark.parametrize("N", [0, 1, 3, 5, 7, 8, 9, 10])
def test_reconstruct_and_backward_vs_oracle(N):
    """pauli_reconstruct (G = sum_n c_n P_n) and pauli_decompose_backward
    (2^-N sum_n g_n P_n) against the oracle's recomposition, within the
    adjoint's bound and 1e-6 of max|G|."""
    p = lib()
    c = workloads.iid_complex(N, 8980 + N, np.complex64).reshape(-1)
    ref = oracle.recompose(c.astype(np.complex128))
    G = p.reconstruct(dev(c), algo="split_i8").cpu().numpy()
    err = np.abs(G.astype(np.complex128) - ref).max()
    assert err <= adjoint_bound(c, ref, torch.complex64, 1.0), err
    assert err <= 1e-6 * np.abs(ref).max()
    gG = p.decompose_backward(dev(c), algo="split_i8").cpu().numpy()
    ref2 = ref / (1 << N)
    err2 = np.abs(gG.astype(np.complex128) - ref2).max()
    assert err2 <= adjoint_bound(c, ref2, torch.complex64, 2.0 ** -N), err2
    assert err2 <= 1e-6 * np.abs(ref2).max()


def test_round_trip_two_pass_and_autograd():
    """reconstruct(decompose(G)) = G within 8e-6 of max|G| (two quantised
    passes); modes 1 and 2 of the two-pass entry points equal the one-call
    adjoints bit for bit; through torch.autograd the gradient is
    pauli_decompose_backward of grad_c."""
    import ctypes
    p = lib()
    L = p.load_library()
    N = 9
    G = workloads.iid_complex(N, 8990, np.complex64)
    Gd = dev(G)
    c = p.decompose(Gd, algo="split_i8")
    G2 = p.reconstruct(c, algo="split_i8").cpu().numpy()
    assert np.abs(G2 - G).max() <= 1e-6 * np.abs(G).max() * 8
    ws = p.workspace("split_i8", N, 1, Gd.device)
    o = p._opts("split_i8", 0, 0, 0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ws)
    for mode, fn, scale in ((1, p.reconstruct, 1.0), (2, p.decompose_backward, None)):
        out = torch.empty(4 ** N, dtype=torch.complex64, device="cuda")
        assert L.pauli_pack(ctypes.c_void_p(c.data_ptr()), N, 1, mode, ctypes.byref(o)) == 0
        assert L.pauli_contract(N, 1, mode, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o)) == 0
        torch.cuda.synchronize()
        assert torch.equal(out.reshape(1 << N, 1 << N), fn(c, algo="split_i8")), mode
    Gg = Gd.clone().requires_grad_(True)
    cg = p.PauliDecompose.apply(Gg, "split_i8")
    w = torch.rand(cg.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    (w * cg.abs() ** 2).sum().backward()
    gc = (2 * w * cg.detach()).contiguous()   # dL/dRe + i dL/dIm, up to autograd's own rounding
    want = p.decompose_backward(gc, algo="split_i8")
    assert (Gg.grad - want).abs().max().item() <= 1e-5 * want.abs().max().item()


@pytest.mark.parametrize("N", [0, 3, 5, 8, 9, 10, 11, 12])
def test_hermitian_variant_bit_identical(N):
    """decompose_hermitian walks half of K and half of the rows for flip masks
    from 512 on (N >= 10); its integer sums are exact, so on Hermitian input it
    equals the general int8 decomposition bit for bit (complex64 and
    complex128), and both match the oracle within the path's bound."""
    p = lib()
    G = workloads.hermitian(N, 8960 + N)
    Gd = dev(G)
    c = p.decompose(Gd, algo="split_i8").cpu().numpy()
    ch = p.decompose_hermitian(Gd, algo="split_i8").cpu().numpy()
    assert np.array_equal(ch, c)
    assert np.all(ch.imag == 0)
    if N <= 11:
        ref = oracle.decompose(G.astype(np.complex128), threads=threads())
        assert check(G, ch, ref, torch.complex64) <= 1e-6
    if N in (10, 11):
        G2 = dev(G.astype(np.complex128))
        c2 = p.decompose(G2, algo="split_i8").cpu().numpy()
        assert np.array_equal(p.decompose_hermitian(G2, algo="split_i8").cpu().numpy(), c2)


def test_hermitian_variant_batch_and_two_pass():
    """A batch of Hermitian matrices 2^30 apart in size, and the same call split
    into pauli_pack / pauli_contract mode 3, equal the general path bit for bit."""
    import ctypes
    p = lib()
    L = p.load_library()
    N = 11
    mats = [workloads.hermitian(N, 8970 + k) * np.float32(2.0 ** (30 * k - 30)) for k in range(3)]
    B = dev(np.stack(mats))
    cb = p.decompose_hermitian(B, algo="split_i8").cpu().numpy()
    for k, G in enumerate(mats):
        assert np.array_equal(cb[k], dec(G)), k
    ws = p.workspace("split_i8", N, 3, B.device)
    o = p._opts("split_i8", 0, 0, 0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ws)
    out = torch.empty(3 * 4 ** N, dtype=torch.complex64, device="cuda")
    assert L.pauli_pack(ctypes.c_void_p(B.data_ptr()), N, 3, 3, ctypes.byref(o)) == 0
    assert L.pauli_contract(N, 3, 3, ctypes.c_void_p(out.data_ptr()), ctypes.byref(o)) == 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(3, -1), cb)


@pytest.mark.parametrize("N", [0, 2, 4, 7])
def test_batches_equal_single_calls(N):
    """Equal-order batches (including the orders below 5, padded to 32 x 32)
    through the decomposition, its Hermitian variant and both adjoints:
    every member equals its own single call bit for bit."""
    p = lib()
    count = 3
    mats = [workloads.iid_complex(N, 9000 + 10 * N + k, np.complex64) for k in range(count)]
    herm = [((m + m.conj().T) / 2).astype(np.complex64) for m in mats]
    B, H = dev(np.stack(mats)), dev(np.stack(herm))
    cb = p.decompose(B, algo="split_i8").cpu().numpy()
    hb = p.decompose_hermitian(H, algo="split_i8").cpu().numpy()
    vecs = dev(np.stack([m.reshape(-1) for m in mats]))
    rb = p.reconstruct(vecs, algo="split_i8").cpu().numpy()
    gb = p.decompose_backward(vecs, algo="split_i8").cpu().numpy()
    for k in range(count):
        assert np.array_equal(cb[k], dec(mats[k])), ("decompose", k)
        assert np.array_equal(hb[k], p.decompose_hermitian(dev(herm[k]), algo="split_i8").cpu().numpy()), ("herm", k)
        v = dev(mats[k].reshape(-1))
        assert np.array_equal(rb[k], p.reconstruct(v, algo="split_i8").cpu().numpy()), ("reconstruct", k)
        assert np.array_equal(gb[k], p.decompose_backward(v, algo="split_i8").cpu().numpy()), ("backward", k)


@pytest.mark.parametrize("which", ["decompose", "reconstruct", "decompose_backward"])
def test_dtype_pairs(which):
    """Every input/output dtype pair of the three entry points: complex64
    input widens exactly (the same quantised integers), and complex64 output
    is the binary64 result rounded once, so all four pairs follow from one
    result bit for bit.  (Unlike the floating-point splits, a general
    complex128 input is quantised from its binary64 values, not from its
    complex64 rounding.)"""
    p = lib()
    fn = getattr(p, which)
    N = 7
    x64 = workloads.iid_complex(N, 9100 + N, np.complex64)
    if which != "decompose":
        x64 = x64.reshape(-1)
    x128 = x64.astype(np.complex128)
    ref = fn(dev(x64), algo="split_i8", out_dtype=torch.complex128)
    assert torch.equal(fn(dev(x128), algo="split_i8", out_dtype=torch.complex128), ref)
    ref64 = ref.to(torch.complex64)
    assert torch.equal(fn(dev(x64), algo="split_i8", out_dtype=torch.complex64), ref64)
    assert torch.equal(fn(dev(x128), algo="split_i8", out_dtype=torch.complex64), ref64)
