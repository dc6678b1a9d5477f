"""Exact-diagonalisation helpers for the oracle pins (tests only).

Hamiltonians are built from Kronecker products of Pauli matrices, independently
of the oracle's local-energy code.  Basis: configuration sigma (lattice order,
site 0 first) <-> index sum_k sigma_k 2^(N-1-k); sigma = 0 is the +1 eigenstate
of Z.
"""
import itertools

import numpy as np
import scipy.sparse as sp

X = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
Y = sp.csr_matrix(np.array([[0.0, -1j], [1j, 0.0]]))
Z = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))
I2 = sp.identity(2, format="csr")


def all_configs(N):
    """All 2^N configurations, row r = binary digits of r (site 0 = MSB)."""
    r = np.arange(2 ** N, dtype=np.int64)
    return ((r[:, None] >> (N - 1 - np.arange(N))[None, :]) & 1).astype(np.uint8)


def op_at(ops, N):
    """Tensor product with ops = {site: 2x2 matrix} and identities elsewhere."""
    out = None
    for k in range(N):
        m = ops.get(k, I2)
        out = m if out is None else sp.kron(out, m, format="csr")
    return out


def bonds(Lx, Ly):
    res = []
    for j in range(Ly):
        for i in range(Lx):
            a = j * Lx + i
            if i + 1 < Lx:
                res.append((a, a + 1))
            if j + 1 < Ly:
                res.append((a, a + Lx))
    return res


def tfim(Lx, Ly, J, h):
    N = Lx * Ly
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=complex)
    for a, b in bonds(Lx, Ly):
        H = H - J * op_at({a: Z, b: Z}, N)
    for k in range(N):
        H = H - h * op_at({k: X}, N)
    return H


def heisenberg(Lx, Ly, J, marshall):
    """J/4 sum_<ab> (XX + YY + ZZ); with marshall=True the XX+YY part changes
    sign (conjugation by Z on one sublattice of the bipartite lattice)."""
    N = Lx * Ly
    s = -1.0 if marshall else 1.0
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=complex)
    for a, b in bonds(Lx, Ly):
        H = H + 0.25 * J * (s * op_at({a: X, b: X}, N) + s * op_at({a: Y, b: Y}, N) +
                            op_at({a: Z, b: Z}, N))
    return H


def sublattice_z(Lx, Ly):
    """Product of Z over the sites with (i + j) odd."""
    N = Lx * Ly
    ops = {}
    for j in range(Ly):
        for i in range(Lx):
            if (i + j) % 2 == 1:
                ops[j * Lx + i] = Z
    return op_at(ops, N)


def free_fermion_e0(N, J, h):
    """Ground energy of the open TFIM chain -J sum ZZ - h sum X: minus the sum
    of the singular values of the N x N upper-bidiagonal matrix with h on the
    diagonal and J above it (Jordan-Wigner / Lieb-Schultz-Mattis)."""
    M = np.diag(np.full(N, float(h))) + np.diag(np.full(N - 1, float(J)), 1)
    return -np.linalg.svd(M, compute_uv=False).sum()


def ground_energy(H):
    import scipy.sparse.linalg as sla
    if H.shape[0] <= 1024:
        return np.linalg.eigvalsh(H.toarray()).min()
    return sla.eigsh(H, k=1, which="SA")[0][0]


def lrtfim(N, J, h, alpha):
    """Long-range TFIM chain, Eq. (8): -J sum_{i<j} Z_i Z_j / |i-j|^alpha - h sum X."""
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=complex)
    for i in range(N):
        for j in range(i + 1, N):
            H = H - J / float(j - i) ** alpha * op_at({i: Z, j: Z}, N)
    for k in range(N):
        H = H - h * op_at({k: X}, N)
    return H


def cluster(n, J=1.0):
    """1D cluster Hamiltonian, Eq. (9), sites 1..n in the paper's numbering
    (0..n-1 here): -J [sum_{k=2}^{n-2} X_{k-1} Z_k X_{k+1} + Z_1 X_2
    + X_{n-1} X_n + X_{n-2} Z_{n-1} Z_n]."""
    H = sp.csr_matrix((2 ** n, 2 ** n), dtype=complex)
    s = lambda k: k - 1  # paper site k -> index
    for k in range(2, n - 1):
        H = H - J * op_at({s(k - 1): X, s(k): Z, s(k + 1): X}, n)
    H = H - J * op_at({s(1): Z, s(2): X}, n)
    H = H - J * op_at({s(n - 1): X, s(n): X}, n)
    H = H - J * op_at({s(n - 2): X, s(n - 1): Z, s(n): Z}, n)
    return H
