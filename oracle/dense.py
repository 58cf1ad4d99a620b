"""Dense-matrix checks for n <= 6 (numpy/scipy).  Test infrastructure.

Pauli strings are built as Kronecker products of the paper's Pauli matrices
(Sec. 2.1, Eq. pauli_mat).  Qubit 0 is the least significant bit of the basis
index (Sec. 3), so it is the RIGHTMOST Kronecker factor:
P = kron(sigma_{n-1}, ..., sigma_0).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

SIGMA = [
    np.eye(2, dtype=complex),
    np.array([[0, 1], [1, 0]], dtype=complex),
    np.array([[0, -1j], [1j, 0]], dtype=complex),
    np.array([[1, 0], [0, -1]], dtype=complex),
]
H1 = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
S1 = np.array([[1, 0], [0, 1j]], dtype=complex)
GATE1 = {0: H1, 1: S1, 2: S1.conj().T, 3: SIGMA[1], 4: SIGMA[2], 5: SIGMA[3]}


def pauli(letters, phase: int = 0) -> np.ndarray:
    m = np.array([[1]], dtype=complex)
    for l in reversed(list(letters)):
        m = np.kron(m, SIGMA[int(l)])
    return (1j ** phase) * m


def embed1(g: np.ndarray, q: int, n: int) -> np.ndarray:
    m = np.array([[1]], dtype=complex)
    for j in reversed(range(n)):
        m = np.kron(m, g if j == q else np.eye(2))
    return m


def embed2(code: int, q0: int, q1: int, n: int) -> np.ndarray:
    """CNOT (q0 control, q1 target), CZ or SWAP as a permutation/phase matrix."""
    N = 1 << n
    m = np.zeros((N, N), dtype=complex)
    for c in range(N):
        b0, b1 = (c >> q0) & 1, (c >> q1) & 1
        r, ph = c, 1.0
        if code == 6 and b0:
            r = c ^ (1 << q1)
        elif code == 7 and b0 and b1:
            ph = -1.0
        elif code == 8 and b0 != b1:
            r = c ^ (1 << q0) ^ (1 << q1)
        m[r, c] = ph
    return m


def gate(code: int, q0: int, q1: int, n: int) -> np.ndarray:
    if code in GATE1:
        return embed1(GATE1[code], q0, n)
    return embed2(code, q0, q1, n)


def circuit_unitary(gates, n: int) -> np.ndarray:
    U = np.eye(1 << n, dtype=complex)
    for g, q0, q1 in np.asarray(gates).reshape(-1, 3):
        U = gate(int(g), int(q0), int(q1), n) @ U
    return U


def rotation(letters, theta: float, phase: int = 0) -> np.ndarray:
    """exp(-i theta/2 * i^phase P) by scipy's matrix exponential."""
    return expm(-0.5j * theta * pauli(letters, phase))


def match_pauli(M: np.ndarray, n: int):
    """Find (letters, phase) with M = i^phase * P, or None."""
    import itertools
    for letters in itertools.product(range(4), repeat=n):
        P = pauli(letters)
        for k in range(4):
            if np.allclose(M, (1j ** k) * P, atol=1e-12):
                return np.array(letters, dtype=np.uint8), k
    return None
