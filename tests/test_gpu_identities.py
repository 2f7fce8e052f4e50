"""Identities of the decomposition checked on every GPU path: closed forms
whose coefficients are known exactly (all-ones matrix, |0><0|, diagonal
matrices), the symmetries c(G^H) = conj c(G) and c(G^T)_n = (-1)^{#Y(n)} c(G)_n,
linearity, and the adjoint relation Re<g, D(G)> = Re<D^H g, G> between the
decomposition D and its backward entry point D^H.

Tolerances are those of the parity tests (error relative to max|c|): 1e-12
for the binary64 paths, 1e-5 for binary32, 1e-6 for the splits and the int8
path, and bit equality where every floating-point path's sums are exact
(small integers, powers of two).
"""
import numpy as np
import pytest
import torch
from scipy.linalg import hadamard

import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp64_gray": 1e-12, "fwht": 1e-12, "fwht_f32": 1e-6, "fp32": 1e-5, "split_bf16": 1e-6,
       "split_fp16": 1e-6, "split_i8": 1e-6}
ALGOS = list(TOL)
# every path whose sums of small dyadic values are exact all the way to the
# output (the int8 path's sums are exact too, but its final scaling by a
# rounded mm / L can leave binary64 outputs one unit in the last place off)
EXACT_ALGOS = [a for a in ALGOS if a != "split_i8"]


def lib():
    import paper_2401_16378_amd as p
    p.load_library()
    return p


def compact_even(v):
    v = v & 0x55555555
    v = (v | (v >> 1)) & 0x33333333
    v = (v | (v >> 2)) & 0x0F0F0F0F
    v = (v | (v >> 4)) & 0x00FF00FF
    return (v | (v >> 8)) & 0x0000FFFF


def masks(N):
    """(x, z) of every coefficient index n (test-side copy of the mapping:
    x_t = bit 2t ^ bit 2t+1, z_t = bit 2t+1)."""
    n = np.arange(4 ** N, dtype=np.int64)
    z = compact_even(n >> 1)
    return compact_even(n) ^ z, z


def popcount(v):
    return np.array([bin(int(a)).count("1") for a in v], dtype=np.int64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("algo", EXACT_ALGOS)
@pytest.mark.parametrize("N", [6, 9])
def test_all_ones_and_ground_projector_exact(algo, N):
    """J (every entry 1): c = 1 exactly on the strings of I and X only (z = 0),
    0 elsewhere; |0><0|: c = 2^-N exactly on the strings of I and Z only
    (x = 0), 0 elsewhere.  Every path sums small dyadic values exactly."""
    p = lib()
    D = 1 << N
    x, z = masks(N)
    J = np.ones((D, D), np.complex64)
    cJ = p.decompose(dev(J), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    assert np.array_equal(cJ, np.where(z == 0, 1.0, 0.0).astype(np.complex128))
    E = np.zeros((D, D), np.complex64)
    E[0, 0] = 1
    cE = p.decompose(dev(E), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    assert np.array_equal(cE, np.where(x == 0, 2.0 ** -N, 0.0).astype(np.complex128))


@pytest.mark.parametrize("algo", ALGOS)
def test_diagonal_is_walsh_hadamard(algo):
    """diag(d): the flip mask x = 0 coefficients are H d / 2^N (H the Sylvester
    Hadamard matrix of scipy), every other coefficient exactly 0."""
    p = lib()
    N = 8
    D = 1 << N
    rng = np.random.default_rng(808)
    d = (rng.standard_normal(D) + 1j * rng.standard_normal(D)).astype(np.complex64)
    c = p.decompose(dev(np.diag(d)), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    x, z = masks(N)
    want = hadamard(D) @ d.astype(np.complex128) / D
    got = np.zeros(D, np.complex128)
    got[z[x == 0]] = c[x == 0]
    assert np.abs(got - want).max() <= TOL[algo] * np.abs(want).max()
    assert np.all(c[x != 0] == 0)


@pytest.mark.parametrize("algo", ALGOS)
def test_adjoint_and_transpose_symmetries(algo):
    """c(G^H) = conj c(G) and c(G^T)_n = (-1)^{#Y(n)} c(G)_n (Y^T = -Y, the
    other Pauli matrices symmetric), #Y(n) = popc(x & z)."""
    p = lib()
    N = 9
    G = workloads.iid_complex(N, 909, np.complex64)
    c = p.decompose(dev(G), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    cH = p.decompose(dev(G.conj().T), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    cT = p.decompose(dev(G.T), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    x, z = masks(N)
    sign = np.where(popcount(x & z) & 1, -1.0, 1.0)
    m = np.abs(c).max()
    assert np.abs(cH - c.conj()).max() <= 2 * TOL[algo] * m
    assert np.abs(cT - sign * c).max() <= 2 * TOL[algo] * m


@pytest.mark.parametrize("algo", ALGOS)
def test_linearity(algo):
    """c(a G + b H) = a c(G) + b c(H) for complex scalars a, b."""
    p = lib()
    N = 9
    G = workloads.iid_complex(N, 910, np.complex128)
    H = workloads.iid_complex(N, 911, np.complex128)
    a, b = 0.75 - 0.5j, -1.25 + 0.25j
    cG = p.decompose(dev(G), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    cH = p.decompose(dev(H), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    cS = p.decompose(dev(a * G + b * H), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    ref = a * cG + b * cH
    assert np.abs(cS - ref).max() <= 3 * TOL[algo] * np.abs(ref).max()


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("N", [7, 10])
def test_adjoint_dot_product(algo, N):
    """Re<g, D(G)> = Re<D^H g, G> with D = decompose and D^H = the backward
    entry point (2^-N sum_n g_n P_n), each evaluated on the GPU path."""
    p = lib()
    G = workloads.iid_complex(N, 1700 + N, np.complex128)
    g = workloads.iid_complex(N, 1750 + N, np.complex128).reshape(-1)
    DG = p.decompose(dev(G), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    DHg = p.decompose_backward(dev(g), algo=algo, out_dtype=torch.complex128).cpu().numpy()
    lhs = np.vdot(g, DG).real
    rhs = np.vdot(DHg, G).real
    scale = np.linalg.norm(g) * np.linalg.norm(DG)
    assert abs(lhs - rhs) <= 10 * TOL[algo] * scale
