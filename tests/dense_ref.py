"""Dense-matrix QAOA reference used to pin the oracle (tests only).

The state is built from the textbook definition with library routines: the
mixer is scipy.linalg.expm of the full 2^n x 2^n Hamiltonian sum_i X_i (built
from Kronecker products), the phase is the diagonal matrix exp(-i gamma C).
Qubit i is bit i of the basis index, so X_i = I_{2^(n-1-i)} (x) X (x) I_{2^i}.
"""
import numpy as np
import scipy.linalg


def mixer_hamiltonian(n):
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    N = 1 << n
    M = np.zeros((N, N))
    for i in range(n):
        M += np.kron(np.kron(np.eye(1 << (n - 1 - i)), X), np.eye(1 << i))
    return M


def dense_state(n, c, gamma, beta, psi0=None):
    N = 1 << n
    M = mixer_hamiltonian(n)
    psi = np.full(N, N ** -0.5, dtype=np.complex128) if psi0 is None else np.array(psi0, dtype=np.complex128)
    for g, b in zip(np.atleast_1d(gamma), np.atleast_1d(beta)):
        psi = np.exp(-1j * g * np.asarray(c, dtype=np.float64)) * psi
        psi = scipy.linalg.expm(-1j * b * M) @ psi
    return psi


def maxcut_p1_closed_form(n, edges, gamma, beta):
    """Expected cut of p=1 QAOA on an unweighted graph (Wang, Hadfield, Jiang,
    Rieffel, Phys. Rev. A 97, 022304 (2018), Theorem 1), in that paper's
    convention: cost = cut, phase exp(-i gamma cut), mixer exp(-i beta sum X)."""
    adj = {i: set() for i in range(n)}
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    tot = 0.0
    for u, v in edges:
        du, dv = len(adj[u]) - 1, len(adj[v]) - 1
        lam = len(adj[u] & adj[v])
        tot += (0.5
                + 0.25 * np.sin(4 * beta) * np.sin(gamma) * (np.cos(gamma) ** du + np.cos(gamma) ** dv)
                - 0.25 * np.sin(2 * beta) ** 2 * np.cos(gamma) ** (du + dv - 2 * lam)
                * (1 - np.cos(2 * gamma) ** lam))
    return tot


def xy_generator(n, i, j):
    """(X_i X_j + Y_i Y_j)/2 as a dense 2^n x 2^n matrix (Kronecker products)."""
    X = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
    Y = np.array([[0.0, -1.0j], [1.0j, 0.0]], dtype=np.complex128)

    def op(mats):  # mats: {qubit: 2x2}; qubit n-1 is the leftmost factor
        out = np.eye(1, dtype=np.complex128)
        for q in range(n - 1, -1, -1):
            out = np.kron(out, mats.get(q, np.eye(2)))
        return out
    return 0.5 * (op({i: X, j: X}) + op({i: Y, j: Y}))


def xy_layer_dense(n, edges, beta):
    """Product of scipy expm(-i beta G_e) over `edges`, first edge applied first."""
    U = np.eye(1 << n, dtype=np.complex128)
    for i, j in edges:
        U = scipy.linalg.expm(-1j * beta * xy_generator(n, i, j)) @ U
    return U
