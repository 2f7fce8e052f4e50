"""Test-side textbook objects, independent of the oracle and of the GPU path:
Pauli matrices of Eq. (3) and Pauli strings built by explicit Kronecker
products with qubit 0 as the rightmost factor (section 2, notation)."""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = [I2, X, Y, Z]
LETTERS = "IXYZ"


def digits(n: int, N: int):
    """Base-4 digits of n, digit t = operator on qubit t."""
    return [(n >> (2 * t)) & 3 for t in range(N)]


def pauli_string(n: int, N: int) -> np.ndarray:
    M = np.ones((1, 1), dtype=np.complex128)
    for t in range(N):
        M = np.kron(PAULIS[(n >> (2 * t)) & 3], M)
    return M


def label(n: int, N: int) -> str:
    """Kronecker-product label, leftmost factor first (as printed in Eq. (2))."""
    return "".join(LETTERS[d] for d in reversed(digits(n, N)))


def brute_coeff(G: np.ndarray, n: int) -> complex:
    N = G.shape[0].bit_length() - 1
    return complex(np.trace(pauli_string(n, N) @ G) / G.shape[0])


def n_of_labels(s: str) -> int:
    """Inverse of label()."""
    N = len(s)
    n = 0
    for t in range(N):
        n |= LETTERS.index(s[N - 1 - t]) << (2 * t)
    return n


def count_y(n: int, N: int) -> int:
    return sum(1 for d in digits(n, N) if d == 2)


def n_of_xz(x: int, z: int, N: int) -> int:
    """Index of the string with flip mask x (X or Y on qubit t) and phase mask
    z (Y or Z on qubit t): operator flag I=0, X=1, Y=2, Z=3 per qubit."""
    n = 0
    for t in range(N):
        xt, zt = (x >> t) & 1, (z >> t) & 1
        flag = {(0, 0): 0, (1, 0): 1, (1, 1): 2, (0, 1): 3}[(xt, zt)]
        n |= flag << (2 * t)
    return n
