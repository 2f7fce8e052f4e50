"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, index or bit order, a transposed operand, a wrong phase) fails at
least one of them:
  - brute-force Tr(P_n G) with explicitly built Kronecker products, Eq. (cn_compact)
  - the printed ordering of Eq. (2) and the printed Pauli matrices of Eq. (3)
  - agreement of the paper's two algorithms, Fast and Slow (Fig. 1b)
  - one-hot strings, closed forms, Kronecker factorisation, symmetries,
    Parseval, Hermitian => real, recomposition (Eq. (1)), adjoint identities,
    and central finite differences of a quadratic loss.
"""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads
from tests import pauli_ref as pr

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_trace(N, seed):
    G = workloads.iid_complex(N, seed + 100 * N)
    c = oracle.decompose(G)
    ref = np.array([pr.brute_coeff(G, n) for n in range(4 ** N)])
    assert rel_err(c, ref) < 1e-14


def test_bruteforce_trace_seeded_n4_workload():
    G = workloads.iid_complex(4, workloads.SEED_N4_BRUTE)
    c = oracle.decompose(G)
    ref = np.array([pr.brute_coeff(G, n) for n in range(256)])
    assert rel_err(c, ref) < 1e-14


def test_golden_pauli_matrices_eq3():
    mats = {k: np.zeros((2, 2), dtype=np.complex128) for k in "IXYZ"}
    with open(os.path.join(GOLDEN, "eq3_paulis.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, r, c, re, im = line.split()
            mats[name][int(r), int(c)] = float(re) + 1j * float(im)
    for flag, name in enumerate("IXYZ"):
        np.testing.assert_array_equal(mats[name], pr.PAULIS[flag])
        # single-qubit decomposition of each printed matrix is the one-hot e_flag
        c = oracle.decompose(mats[name])
        np.testing.assert_array_equal(c, np.eye(4)[flag])
        for i in range(2):
            for j in range(2):
                assert oracle.pauli_element(flag, 1, i, j) == mats[name][i, j]


def test_golden_ordering_eq2():
    with open(os.path.join(GOLDEN, "eq2_ordering.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for n_str, lab in rows:
        n = int(n_str)
        assert pr.label(n, 2) == lab
        M = np.ones((1, 1), dtype=np.complex128)
        for ch in lab:  # leftmost factor first, as printed
            M = np.kron(M, pr.PAULIS["IXYZ".index(ch)])
        c = oracle.decompose(M)
        expect = np.zeros(16)
        expect[n] = 1.0
        np.testing.assert_array_equal(c, expect)


def test_y_phase():
    # c_Y = 1 for G = Y pins the sign of the (-i) phase and the gather G[i^m][i]
    c = oracle.decompose(pr.Y)
    np.testing.assert_array_equal(c, np.array([0, 0, 1, 0], dtype=np.complex128))
    # the transpose of Y is -Y: a transposed gather would return -1 here
    c = oracle.decompose(pr.Y.T.copy())
    np.testing.assert_array_equal(c, np.array([0, 0, -1, 0], dtype=np.complex128))


def test_flags_and_mask():
    rng = np.random.default_rng(5)
    for _ in range(200):
        N = int(rng.integers(1, 16))
        n = int(rng.integers(0, 4 ** N))
        ds = pr.digits(n, N)
        for t in range(N):
            assert oracle.operator_at(n, t) == ds[t]
        m = sum((1 << t) for t in range(N) if ds[t] in (1, 2))
        assert oracle.flip_mask(n, N) == m


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_fast_vs_slow(N):
    G = workloads.iid_complex(N, 7 + N)
    ns = range(4 ** N) if N <= 5 else workloads.sample_indices(4 ** N, 300, seed=N)
    for n in ns:
        a = oracle.coefficient(G, int(n))
        b = oracle.coefficient_natural(G, int(n))
        assert abs(a - b) <= 1e-13 * max(1.0, abs(b))


@pytest.mark.parametrize("N", [1, 2, 3])
def test_one_hot_all(N):
    for m in range(4 ** N):
        c = oracle.decompose(pr.pauli_string(m, N))
        e = np.zeros(4 ** N, dtype=np.complex128)
        e[m] = 1.0
        np.testing.assert_array_equal(c, e)


def test_one_hot_sampled_n6():
    rng = np.random.default_rng(11)
    for m in rng.integers(0, 4 ** 6, size=6):
        c = oracle.decompose(pr.pauli_string(int(m), 6))
        e = np.zeros(4 ** 6)
        e[int(m)] = 1.0
        np.testing.assert_array_equal(c, e)


@pytest.mark.parametrize("N", [1, 3, 5])
def test_closed_forms(N):
    D = 1 << N
    total = 4 ** N
    # all-ones matrix = (I + X)^{(x)N}: coefficient 1 exactly on {I,X}^N strings
    c = oracle.decompose(np.ones((D, D)))
    e = np.array([1.0 if all(d in (0, 1) for d in pr.digits(n, N)) else 0.0 for n in range(total)])
    np.testing.assert_array_equal(c, e)
    # |0><0| = ((I + Z)/2)^{(x)N}: 2^-N on {I,Z}^N strings
    P0 = np.zeros((D, D))
    P0[0, 0] = 1.0
    c = oracle.decompose(P0)
    e = np.array([2.0 ** -N if all(d in (0, 3) for d in pr.digits(n, N)) else 0.0 for n in range(total)])
    np.testing.assert_array_equal(c, e)
    # diagonal matrix: the {I,Z} coefficients are the Walsh-Hadamard transform / 2^N
    d = np.random.default_rng(N).standard_normal(D)
    c = oracle.decompose(np.diag(d))
    zs = np.arange(D)
    n_of_z = [sum(3 << (2 * t) for t in range(N) if (z >> t) & 1) for z in zs]
    wht = scipy.linalg.hadamard(D) @ d / D
    assert rel_err(c[n_of_z], wht) < 1e-14
    off = np.ones(total, dtype=bool)
    off[n_of_z] = False
    assert np.all(c[off] == 0)


def test_kronecker_factorisation():
    A = workloads.iid_complex(2, 21)
    B = workloads.iid_complex(3, 22)
    cA, cB = oracle.decompose(A), oracle.decompose(B)
    cAB = oracle.decompose(np.kron(A, B))
    expect = np.kron(cA, cB)  # index nA * 4^3 + nB
    assert rel_err(cAB, expect) < 1e-14


def test_symmetries():
    N = 4
    G = workloads.iid_complex(N, 31)
    H = workloads.iid_complex(N, 32)
    c = oracle.decompose(G)
    # Paulis are Hermitian: c(G^H) = conj(c(G))
    assert rel_err(oracle.decompose(G.conj().T.copy()), c.conj()) < 1e-14
    # Y^T = -Y and the others are symmetric: c(G^T)_n = (-1)^{#Y} c(G)_n
    sgn = np.array([(-1.0) ** pr.count_y(n, N) for n in range(4 ** N)])
    assert rel_err(oracle.decompose(G.T.copy()), sgn * c) < 1e-14
    # linearity
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    assert rel_err(oracle.decompose(a * G + b * H), a * c + b * oracle.decompose(H)) < 1e-13


def test_hermitian_real():
    G = workloads.hermitian(5, 41).astype(np.complex128)
    c = oracle.decompose(G)
    assert np.abs(c.imag).max() <= 1e-15 * np.abs(c).max()


@pytest.mark.parametrize("N", [2, 5, 6])
def test_parseval(N):
    G = workloads.iid_complex(N, 51 + N)
    c = oracle.decompose(G)
    lhs = np.sum(np.abs(c) ** 2)
    rhs = np.sum(np.abs(G) ** 2) / (1 << N)
    assert abs(lhs - rhs) <= 1e-13 * rhs


@pytest.mark.parametrize("N", [1, 2, 4])
def test_recompose_roundtrip(N):
    G = workloads.iid_complex(N, 61 + N)
    c = oracle.decompose(G)
    assert rel_err(oracle.recompose(c), G) < 1e-14
    c2 = workloads.iid_complex(N, 71 + N).reshape(-1)[: 4 ** N].copy()
    assert rel_err(oracle.decompose(oracle.recompose(c2)), c2) < 1e-14
    # recomposition against explicit sum of Kronecker products
    Gk = sum(c2[n] * pr.pauli_string(n, N) for n in range(4 ** N))
    assert rel_err(oracle.recompose(c2), Gk) < 1e-14


def test_adjoint_dot_product():
    N = 4
    D = 1 << N
    G = workloads.iid_complex(N, 81)
    g = workloads.iid_complex(N, 82).reshape(-1)[: 4 ** N].copy()
    rows, cols = np.divmod(np.arange(D * D), D)
    DHg = oracle.grad_entries(g, rows, cols).reshape(D, D)
    lhs = np.vdot(g, oracle.decompose(G))  # <g, D(G)>
    rhs = np.vdot(DHg, G)  # <D^H g, G>
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_gradient_central_fd():
    """L = sum_n w_n |c_n - t_n|^2 is quadratic in (Re G, Im G), so central
    differences are exact up to rounding."""
    N = 3
    D = 1 << N
    G = workloads.iid_complex(N, 91)
    T = workloads.iid_complex(N, 92)
    w = np.random.default_rng(93).uniform(0, 1, 4 ** N)
    t = oracle.decompose(T)

    def loss(Gm):
        return float(np.sum(w * np.abs(oracle.decompose(Gm) - t) ** 2))

    gc = 2.0 * w * (oracle.decompose(G) - t)  # dL/dRe c + i dL/dIm c
    rows, cols = workloads.sample_entries(D, 12, seed=94)
    grad = oracle.grad_entries(gc, rows, cols)
    h = 1e-3
    for q in range(len(rows)):
        r, cc = int(rows[q]), int(cols[q])
        E = np.zeros((D, D), dtype=np.complex128)
        E[r, cc] = h
        d_re = (loss(G + E) - loss(G - E)) / (2 * h)
        d_im = (loss(G + 1j * E) - loss(G - 1j * E)) / (2 * h)
        assert abs(grad[q] - (d_re + 1j * d_im)) <= 1e-9 * max(1.0, abs(grad[q]))


def test_threaded_driver_matches_serial():
    G = workloads.iid_complex(5, 101)
    np.testing.assert_array_equal(oracle.decompose(G, threads=4), oracle.decompose(G))
    ns = workloads.sample_indices(4 ** 5, 100, seed=3)
    np.testing.assert_array_equal(oracle.coeffs_at(G, ns, threads=3), oracle.decompose(G)[ns.astype(np.int64)])


def test_n0():
    G = np.array([[2.5 - 1.0j]])
    np.testing.assert_array_equal(oracle.decompose(G), np.array([2.5 - 1.0j]))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_quaternary_gray_order(N):
    """The quaternary Gray enumeration (section 2) visits every string once,
    starts at the identity, and changes exactly one operator per step, to an
    adjacent flag (I-X, X-Y or Y-Z)."""
    seq = [oracle.quaternary_gray(k, N) for k in range(4 ** N)]
    assert seq[0] == 0
    assert sorted(seq) == list(range(4 ** N))
    for a, b in zip(seq, seq[1:]):
        diff = [t for t in range(N) if oracle.operator_at(a, t) != oracle.operator_at(b, t)]
        assert len(diff) == 1
        t = diff[0]
        assert abs(oracle.operator_at(a, t) - oracle.operator_at(b, t)) == 1


def test_quaternary_gray_two_digits():
    """The reflected order for two operators written out: the low digit runs
    up, then down each time the high digit advances."""
    want = [0x0, 0x1, 0x2, 0x3, 0x7, 0x6, 0x5, 0x4, 0x8, 0x9, 0xA, 0xB, 0xF, 0xE, 0xD, 0xC]
    # digits (high, low) -> n = 4 * high + low
    assert [oracle.quaternary_gray(k, 2) for k in range(16)] == [4 * (w >> 2) + (w & 3) for w in want]


@pytest.mark.parametrize("N", [0, 1, 2, 3, 4, 5, 6])
def test_qgray_decomposition_bitexact(N):
    """The across-n recurrence of lambda_0 only changes how lambda_0 is
    formed; lambda stays exactly in {+-1, +-i}, so every coefficient equals
    the per-string evaluation bit for bit (and brute force to rounding)."""
    G = workloads.iid_complex(N, 900 + N)
    c = oracle.decompose_qgray(G)
    np.testing.assert_array_equal(c, oracle.decompose(G))
    if N <= 3:
        ref = np.array([pr.brute_coeff(G, n) for n in range(4 ** N)])
        assert rel_err(c, ref) < 1e-14


def test_qgray_eq2_example():
    """Eq. (2)'s ordering: 1(x)X is string 1, X(x)1 string 4, Y(x)Y string
    10 and Z(x)Z string 15, so G = 2 1(x)X - 3i X(x)1 + Y(x)Y + 0.5 Z(x)Z
    decomposes to exactly those four coefficients and zeros (Eq. (3)
    matrices)."""
    I2 = np.eye(2, dtype=np.complex128)
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    G = 2 * np.kron(I2, X) - 3j * np.kron(X, I2) + np.kron(Y, Y) + 0.5 * np.kron(Z, Z)
    c = oracle.decompose_qgray(G)
    want = np.zeros(16, dtype=np.complex128)
    want[1], want[4], want[10], want[15] = 2.0, -3j, 1.0, 0.5
    np.testing.assert_array_equal(c, want)
