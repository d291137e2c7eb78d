"""Gate matrices in the computational basis, FP64 (oracle; test-only).

For a gate on qubits (q[0], ..., q[k-1]) the matrix index is
sum_j b_j 2^(k-1-j) with b_j the bit of qubit q[j]: q[0] is the most
significant (the left Kronecker factor, as the CNOT control of Example 2).

Rotation conventions (not fixed by the paper; the reading used throughout):
RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2),
RZZ(t) = exp(-i t Z(x)Z/2), PHASE(l) = diag(1, e^{il}),
CP(l) = diag(1, 1, 1, e^{il}).
"""
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def _expm_pauli(theta, pauli):
    # exp(-i theta/2 P) = cos(theta/2) I - i sin(theta/2) P for P^2 = I
    d = pauli.shape[0]
    return math.cos(theta / 2) * np.eye(d, dtype=np.complex128) - 1j * math.sin(theta / 2) * pauli


def matrix(g):
    k = g["kind"]
    t = g["param"]
    if k == "U":
        return np.asarray(g["matrix"], dtype=np.complex128)
    if k == "H":
        return H.copy()
    if k == "X":
        return X.copy()
    if k == "Y":
        return Y.copy()
    if k == "Z":
        return Z.copy()
    if k == "S":
        return np.diag([1, 1j]).astype(np.complex128)
    if k == "SDG":
        return np.diag([1, -1j]).astype(np.complex128)
    if k == "T":
        return np.diag([1, np.exp(1j * math.pi / 4)])
    if k == "TDG":
        return np.diag([1, np.exp(-1j * math.pi / 4)])
    if k == "RX":
        return _expm_pauli(t, X)
    if k == "RY":
        return _expm_pauli(t, Y)
    if k == "RZ":
        return _expm_pauli(t, Z)
    if k == "PHASE":
        return np.diag([1, np.exp(1j * t)])
    if k == "CX":
        return np.kron(P0, I2) + np.kron(P1, X)
    if k == "CZ":
        return np.kron(P0, I2) + np.kron(P1, Z)
    if k == "CP":
        return np.kron(P0, I2) + np.kron(P1, np.diag([1, np.exp(1j * t)]))
    if k == "RZZ":
        return _expm_pauli(t, np.kron(Z, Z))
    if k == "SWAP":
        return np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
    if k == "ISWAP":
        return np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
    raise ValueError(f"unknown gate kind {k}")


def generator(g):
    """Hermitian G with d(matrix)/d(param) = -i/2 G matrix (rotation gates)."""
    k = g["kind"]
    if k == "RX":
        return X
    if k == "RY":
        return Y
    if k == "RZ":
        return Z
    if k == "RZZ":
        return np.kron(Z, Z)
    raise ValueError(f"{k} has no Pauli generator")
