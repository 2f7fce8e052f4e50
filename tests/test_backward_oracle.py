"""Pins the oracle's gradient of the differentiation workload (8 complex64
matrices at N = 11, L = sum_n w_n |c_n - t_n|^2, 64 seeded entries) to central
finite differences of L, on the CPU."""
import numpy as np
import pytest

from tests import backward_workload as bw


@pytest.fixture(scope="module")
def problem():
    return bw.make_problem()


@pytest.fixture(scope="module")
def finite_differences(problem):
    return bw.make_finite_differences(problem)


def test_oracle_gradient_vs_finite_differences(problem, finite_differences):
    """Pins the oracle gradient of this workload to central differences at
    every one of the 64 sampled entries (L is quadratic in G, so central
    differences are exact up to rounding)."""
    grad = bw.oracle_gradient(problem)
    fd = finite_differences
    assert np.abs(grad - fd).max() <= 1e-8 * np.abs(grad).max(), np.abs(grad - fd).max()
