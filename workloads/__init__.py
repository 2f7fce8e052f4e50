"""Seeded synthetic inputs for the dense Pauli decomposition workloads.

Shared by the tests, the benchmark, the smoke check and the oracle runs.  This
module draws random numbers and builds matrices; it holds none of the
decomposition's arithmetic.

The paper benchmarks "random, dense, complex" matrices without naming a
distribution (section 4); these generators use iid standard-normal real and
imaginary parts from numpy's PCG64, drawn real part first, C order, in float64
and then cast.  Hermitian inputs are G = (A + A^H)/2 evaluated in complex64,
which is exactly Hermitian (elementwise addition commutes).
"""
from __future__ import annotations

import numpy as np

# seeds of the named workloads
SEED_N6 = 1006
SEED_N4_BRUTE = 1004
SEED_N10 = 1010
SEED_N12 = 1012
SEED_N14 = 1014
SEED_BATCH = 2000
SEED_BWD_G = 3000
SEED_BWD_T = 3001
SEED_BWD_W = 3002
SEED_SAMPLE = 4000


def iid_complex(N: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """2^N x 2^N matrix, re and im iid N(0,1)."""
    rng = np.random.default_rng(seed)
    D = 1 << N
    re = rng.standard_normal((D, D))
    im = rng.standard_normal((D, D))
    G = np.empty((D, D), dtype=np.complex128)
    G.real = re
    G.imag = im
    return G.astype(dtype, copy=False)


def iid_complex_batch(N: int, count: int, seed: int, dtype=np.complex64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    D = 1 << N
    out = np.empty((count, D, D), dtype=dtype)
    for b in range(count):
        re = rng.standard_normal((D, D))
        im = rng.standard_normal((D, D))
        out[b].real = re
        out[b].imag = im
    return out


def hermitian(N: int, seed: int) -> np.ndarray:
    """complex64 Hermitian G = (A + A^H)/2 with A iid complex N(0,1)."""
    A = iid_complex(N, seed, np.complex64)
    return ((A + A.conj().T) * np.float32(0.5)).astype(np.complex64)


def batch_spec(seed: int = SEED_BATCH, count: int = 512, nmin: int = 3, nmax: int = 9,
               hermitian_frac: float = 0.2):
    """The uneven batch: N_k uniform on nmin..nmax, exactly round(frac*count)
    Hermitian members (seeded choice), complex64.  Returns (Ns, matrices)."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(nmin, nmax + 1, size=count)
    n_herm = int(hermitian_frac * count)
    herm = np.zeros(count, dtype=bool)
    herm[rng.choice(count, size=n_herm, replace=False)] = True
    mats = []
    for k in range(count):
        D = 1 << int(Ns[k])
        re = rng.standard_normal((D, D))
        im = rng.standard_normal((D, D))
        A = (re + 1j * im).astype(np.complex64)
        if herm[k]:
            A = ((A + A.conj().T) * np.float32(0.5)).astype(np.complex64)
        mats.append(A)
    return [int(n) for n in Ns], mats, herm


def backward_problem(N: int = 11, count: int = 8):
    """Inputs of the differentiation workload: G (count matrices), a second
    random batch G2 whose coefficients are the targets t, and weights
    w ~ U(0,1) of shape (count, 4^N).  All complex64 / float64 as drawn."""
    G = iid_complex_batch(N, count, SEED_BWD_G)
    G2 = iid_complex_batch(N, count, SEED_BWD_T)
    w = np.random.default_rng(SEED_BWD_W).uniform(0.0, 1.0, size=(count, 1 << (2 * N)))
    return G, G2, w


def sample_indices(total: int, count: int, seed: int = SEED_SAMPLE) -> np.ndarray:
    """count distinct coefficient indices in [0, total), uniform without
    replacement, sorted."""
    rng = np.random.default_rng(seed)
    if count >= total:
        return np.arange(total, dtype=np.uint64)
    return np.sort(rng.choice(total, size=count, replace=False)).astype(np.uint64)


def sample_entries(D: int, count: int, seed: int):
    """count distinct (row, col) positions of a D x D matrix."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(D * D, size=count, replace=False)
    return (flat // D).astype(np.uint64), (flat % D).astype(np.uint64)
