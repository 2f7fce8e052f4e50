"""Coefficients of a list of Pauli strings (pauli_coeffs_at): every result is
one binary64 signed sum over an XOR diagonal, so it must match the oracle's
per-string coefficient to 1e-12 of the largest magnitude in the list, keep
the caller's order (repeats included) and give exact one-hots."""
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


@pytest.mark.parametrize("N", list(range(0, 7)))
@pytest.mark.parametrize("in_dt", [np.complex64, np.complex128])
def test_all_strings_small(N, in_dt):
    p = lib()
    G = workloads.iid_complex(N, 900 + N, in_dt)
    ns = np.arange(4 ** N, dtype=np.uint32)
    got = p.coeffs_at(torch.from_numpy(G).cuda(), ns, out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.decompose(G)
    assert rel_err(got, ref) <= 1e-12


def test_one_hot_exact():
    p = lib()
    for N in (1, 2, 3):
        ns = np.arange(4 ** N, dtype=np.uint32)[::-1].copy()
        for m in range(4 ** N):
            P = torch.from_numpy(pr.pauli_string(m, N).astype(np.complex64)).cuda()
            c = p.coeffs_at(P, ns).cpu().numpy()
            e = (ns == m).astype(np.complex64)
            assert np.array_equal(c, e), (N, m)


def test_random_list_order_and_repeats_n10():
    p = lib()
    N = 10
    G = workloads.iid_complex(N, workloads.SEED_N10, np.complex128)
    rng = np.random.default_rng(77)
    ns = rng.integers(0, 4 ** N, 3000).astype(np.uint32)
    ns[100:110] = ns[5]                         # repeats
    ns[200] = 0                                 # identity
    Gd = torch.from_numpy(G).cuda()
    ref = oracle.coeffs_at(G, ns, threads=threads())
    for out_dt in (torch.complex128, torch.complex64):
        got = p.coeffs_at(Gd, ns, out_dtype=out_dt).cpu().numpy()
        tol = 1e-12 if out_dt == torch.complex128 else 1e-6
        assert rel_err(got, ref) <= tol
        assert np.all(got[100:110] == got[5])
    rev = p.coeffs_at(Gd, ns[::-1].copy()).cpu().numpy()
    fwd = p.coeffs_at(Gd, ns).cpu().numpy()
    assert np.array_equal(rev[::-1], fwd)       # same value whatever the list order


def test_one_line_group_many_chunks():
    """1000 strings with flip masks in 0..15 form one line group cut into
    several 256-string chunks."""
    p = lib()
    N = 10
    G = workloads.iid_complex(N, 910, np.complex64)
    rng = np.random.default_rng(8)
    x = rng.integers(0, 16, 1000)
    z = rng.integers(0, 1 << N, 1000)
    ns = np.array([pr.n_of_xz(int(a), int(b), N) for a, b in zip(x, z)], dtype=np.uint32)
    got = p.coeffs_at(torch.from_numpy(G).cuda(), ns, out_dtype=torch.complex128).cpu().numpy()
    ref = oracle.coeffs_at(G, ns, threads=threads())
    assert rel_err(got, ref) <= 1e-12


def test_n14_sample_vs_binary64_decomposition():
    """Precision workload at N = 14 (complex64 Hermitian): 65,536 sampled
    strings against the binary64 Gray-code decomposition at the same indices
    (itself pinned to the oracle) and 2,048 of them against the oracle."""
    p = lib()
    N = 14
    G = workloads.hermitian(N, workloads.SEED_N14)
    Gd = torch.from_numpy(G).cuda()
    ns = workloads.sample_indices(4 ** N, 65536, seed=workloads.SEED_SAMPLE).astype(np.uint32)
    got = p.coeffs_at(Gd, ns, out_dtype=torch.complex128)
    full = p.decompose(Gd, algo="fp64_gray", out_dtype=torch.complex128)
    ref = full[torch.from_numpy(ns.astype(np.int64)).cuda()]
    err = ((got - ref).abs().max() / ref.abs().max()).item()
    assert err <= 1e-12, err
    g = got.cpu().numpy()
    assert np.abs(g.imag).max() <= 1e-12 * np.abs(g).max()     # Hermitian: real coefficients
    sub = ns[:2048]
    assert rel_err(g[:2048], oracle.coeffs_at(G, sub, threads=threads())) <= 1e-12


def test_workspace_argument():
    p = lib()
    N = 8
    G = torch.from_numpy(workloads.iid_complex(N, 920, np.complex64)).cuda()
    ns = np.arange(0, 4 ** N, 37, dtype=np.uint32)
    need = p.load_library().pauli_coeffs_at_workspace_bytes(N, len(ns))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    a = p.coeffs_at(G, ns, workspace_tensor=ws)
    b = p.coeffs_at(G, ns)
    assert torch.equal(a, b)
    with pytest.raises(p.PauliError):
        p.coeffs_at(G, ns, workspace_tensor=ws[:256])


def dense_list_gradient(N, strings, g):
    """The oracle's 2^-N sum_k g_k P_{n_k} at every entry (repeats add)."""
    gc = np.zeros(4 ** N, np.complex128)
    np.add.at(gc, np.asarray(strings, dtype=np.int64), g)
    D = 1 << N
    rows, cols = np.divmod(np.arange(D * D, dtype=np.uint64), D)
    return oracle.grad_entries(gc, rows, cols).reshape(D, D)


@pytest.mark.parametrize("N", [0, 1, 3, 5, 8])
def test_backward_vs_oracle(N):
    p = lib()
    rng = np.random.default_rng(930 + N)
    L = min(4 ** N, 40) + 3
    ns = rng.integers(0, 4 ** N, L).astype(np.uint32)
    ns[-1] = ns[0]                                   # a repeat adds
    g = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    got = p.coeffs_at_backward(torch.from_numpy(g).cuda(), N, ns).cpu().numpy()
    ref = dense_list_gradient(N, ns, g)
    assert rel_err(got, ref) <= 1e-12


def test_backward_equals_full_adjoint_n10():
    """Scattering the list gradient into a 4^N vector and running the binary64
    full adjoint must give the same matrix."""
    p = lib()
    N = 10
    rng = np.random.default_rng(940)
    ns = rng.integers(0, 4 ** N, 5000).astype(np.uint32)
    g = rng.standard_normal(5000) + 1j * rng.standard_normal(5000)
    got = p.coeffs_at_backward(torch.from_numpy(g).cuda(), N, ns)
    gc = torch.zeros(4 ** N, dtype=torch.complex128, device="cuda")
    gc.index_add_(0, torch.from_numpy(ns.astype(np.int64)).cuda(), torch.from_numpy(g).cuda())
    full = p.decompose_backward(gc, algo="fp64_gray")
    assert ((got - full).abs().max() / full.abs().max()).item() <= 1e-12


def test_backward_dtype_combinations():
    """The list adjoint widens complex64 gradients exactly and sums in
    binary64: every gradient/output dtype pair equals the complex128 result
    (rounded once to binary32 for complex64 output) bit for bit."""
    p = lib()
    N = 8
    rng = np.random.default_rng(945)
    ns = rng.integers(0, 4 ** N, 3000).astype(np.uint32)
    g64 = (rng.standard_normal(3000) + 1j * rng.standard_normal(3000)).astype(np.complex64)
    g128 = g64.astype(np.complex128)
    ref = p.coeffs_at_backward(torch.from_numpy(g128).cuda(), N, ns, out_dtype=torch.complex128)
    assert torch.equal(p.coeffs_at_backward(torch.from_numpy(g64).cuda(), N, ns, out_dtype=torch.complex128), ref)
    ref64 = ref.to(torch.complex64)
    assert torch.equal(p.coeffs_at_backward(torch.from_numpy(g64).cuda(), N, ns, out_dtype=torch.complex64), ref64)
    assert torch.equal(p.coeffs_at_backward(torch.from_numpy(g128).cuda(), N, ns, out_dtype=torch.complex64), ref64)


def test_autograd_list_loss():
    """L = sum_k w_k |c_k - t_k|^2 over a list of strings, through
    PauliCoeffsAt: the gradient equals the oracle's adjoint of 2 w (c - t)."""
    p = lib()
    N = 7
    G = workloads.iid_complex(N, 950, np.complex128)
    rng = np.random.default_rng(951)
    ns = rng.integers(0, 4 ** N, 300).astype(np.uint32)
    t = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    w = rng.uniform(0, 1, 300)
    Gd = torch.from_numpy(G).cuda().requires_grad_(True)
    c = p.PauliCoeffsAt.apply(Gd, ns)
    loss = (torch.from_numpy(w).cuda() * (c - torch.from_numpy(t).cuda()).abs() ** 2).sum()
    loss.backward()
    cref = oracle.coeffs_at(G, ns)
    ref = dense_list_gradient(N, ns, 2.0 * w * (cref - t))
    assert rel_err(Gd.grad.cpu().numpy(), ref) <= 1e-12
