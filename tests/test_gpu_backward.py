"""Differentiation workload: a batch of 8 complex64 matrices at N = 11 with
loss L = sum_n w_n |c_n - t_n|^2 (w ~ U(0,1), t = coefficients of a second
random matrix).  The gradient from the hand-written adjoint kernel (through
torch.autograd) is checked on 64 seeded entries against

  * the oracle's gradient, 2^-N sum_n g_n P_n with g = 2 w (c - t) and c, t
    evaluated by the oracle, and
  * central finite differences of L in binary64, with the affected
    coefficients re-evaluated by the oracle (L is quadratic, so central
    differences are exact up to rounding).

Tolerance: 1e-5 max|grad| for the split, int8 and fp32 paths, 1e-10 for binary64.
The oracle gradient itself is pinned to the finite differences on the CPU.
"""
import numpy as np
import pytest
import torch

from tests import backward_workload as bw

pytestmark = pytest.mark.gpu

TOL = {"split_bf16": 1e-5, "split_fp16": 1e-5, "fp32": 1e-5, "split_i8": 1e-5, "fp64_gray": 1e-10, "fwht": 1e-10}


@pytest.fixture(scope="module")
def problem():
    return bw.make_problem()


@pytest.fixture(scope="module")
def finite_differences(problem):
    return bw.make_finite_differences(problem)


def oracle_gradient(problem):
    return bw.oracle_gradient(problem)


def gpu_gradient(problem, algo):
    import paper_2401_16378_amd as pauli
    G, G2, w, (b, rows, cols), ref = problem
    dt = torch.complex128 if algo in ("fp64_gray", "fwht") else torch.complex64   # binary64 algorithms
    Gd = torch.from_numpy(G).to("cuda").to(dt).requires_grad_(True)
    t = pauli.decompose(torch.from_numpy(G2).to("cuda").to(dt), algo=algo).detach()
    c = pauli.PauliDecompose.apply(Gd, algo)
    wd = torch.from_numpy(w).to("cuda")
    loss = (wd * (c.to(torch.complex128) - t.to(torch.complex128)).abs() ** 2).sum()
    loss.backward()
    g = Gd.grad[torch.from_numpy(b).cuda(), torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()]
    return g.to(torch.complex128).cpu().numpy()


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "split_i8", "fp64_gray", "fwht"])
def test_adjoint_gradient_vs_oracle(problem, algo):
    ref = oracle_gradient(problem)
    got = gpu_gradient(problem, algo)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= TOL[algo], err


@pytest.mark.parametrize("algo", ["split_bf16", "split_fp16", "fp32", "split_i8", "fp64_gray", "fwht"])
def test_adjoint_gradient_vs_finite_differences(problem, finite_differences, algo):
    """The GPU gradient (hand-written adjoint through torch.autograd) against
    the central differences directly, all 64 entries.  The differences carry
    a rounding error near 1e-10 of max|grad| (binary64 losses of order one
    divided by 2h), so the binary64 algorithms are held to 1e-8 here; their
    1e-10 bar is met against the oracle's gradient above."""
    fd = finite_differences
    got = gpu_gradient(problem, algo)
    err = np.abs(got - fd).max() / np.abs(fd).max()
    assert err <= max(TOL[algo], 1e-8), err
