"""Differentiation workload on the CPU: a batch of 8 complex64 matrices at
N = 11 with loss L = sum_n w_n |c_n - t_n|^2 (w ~ U(0,1), t = coefficients of
a second random matrix), 64 seeded entries of G.

Holds the inputs, the oracle's gradient at those entries (2^-N sum_n g_n P_n
with g = 2 w (c - t), c and t evaluated by the oracle) and central finite
differences of L in binary64; shared by the CPU pin of the oracle gradient
and the GPU gradient tests.
"""
import os

import numpy as np

import oracle
import workloads
from tests import pauli_ref as pr

N = 11
D = 1 << N


def threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def make_problem():
    G, G2, w = workloads.backward_problem(N, 8)
    rng = np.random.default_rng(workloads.SEED_BWD_W + 1)
    flat = rng.choice(8 * D * D, size=64, replace=False)
    b, rem = np.divmod(flat, D * D)
    rows, cols = np.divmod(rem, D)
    # oracle coefficients of G and G2 on every string touching a sampled entry
    ref = []
    for q in range(64):
        x = int(rows[q]) ^ int(cols[q])
        ns = np.array([pr.n_of_xz(x, z, N) for z in range(D)], dtype=np.uint64)
        c = oracle.coeffs_at(G[b[q]].astype(np.complex128), ns, threads=threads())
        t = oracle.coeffs_at(G2[b[q]].astype(np.complex128), ns, threads=threads())
        ref.append((ns, c, t))
    return G, G2, w, (b, rows, cols), ref


def make_finite_differences(problem):
    """Central differences of L in binary64 at all 64 entries, real and
    imaginary directions, h = 1e-3; only the 2^N coefficients whose flip mask
    is row ^ col depend on entry (row, col), so only they are re-evaluated."""
    G, G2, w, (b, rows, cols), ref = problem
    h = 1e-3
    fd = np.zeros(64, dtype=np.complex128)
    for q in range(64):
        ns, c, t = ref[q]
        Gq = G[b[q]].astype(np.complex128)
        wq = w[b[q], ns.astype(np.int64)]

        def loss_delta(delta):
            Gp = Gq.copy()
            Gp[rows[q], cols[q]] += delta
            cp = oracle.coeffs_at(Gp, ns, threads=threads())
            return float(np.sum(wq * np.abs(cp - t) ** 2))

        d_re = (loss_delta(h) - loss_delta(-h)) / (2 * h)
        d_im = (loss_delta(1j * h) - loss_delta(-1j * h)) / (2 * h)
        fd[q] = d_re + 1j * d_im
    return fd


def oracle_gradient(problem):
    G, G2, w, (b, rows, cols), ref = problem
    out = np.zeros(64, dtype=np.complex128)
    for q in range(64):
        ns, c, t = ref[q]
        gc = np.zeros(4 ** N, dtype=np.complex128)
        gc[ns.astype(np.int64)] = 2.0 * w[b[q], ns.astype(np.int64)] * (c - t)
        out[q] = oracle.grad_entries(gc, rows[q:q + 1], cols[q:q + 1])[0]
    return out
