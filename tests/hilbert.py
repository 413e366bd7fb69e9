"""Textbook Hilbert-space constructions used to pin the oracle (tests only).

The Heisenberg Hamiltonian is assembled here from Kronecker products of the
spin-1/2 matrices, an independent route from the oracle's bond-by-bond bit
construction.  Single-site basis index 1 <-> spin up (sigma = +1), 0 <-> down,
and site i is bit i of the many-body index (site 0 least significant).
"""
import numpy as np
import scipy.sparse as sp

SZ = sp.csr_matrix(np.array([[-0.5, 0.0], [0.0, 0.5]]))
SP = sp.csr_matrix(np.array([[0.0, 0.0], [1.0, 0.0]]))   # |down> -> |up>
SM = SP.T.tocsr()
I2 = sp.identity(2, format="csr")


def site_op(op, i, N):
    # kron(A_{N-1}, ..., A_0): site 0 is the fastest-varying (least significant) factor
    out = sp.identity(1, format="csr")
    for k in range(N - 1, -1, -1):
        out = sp.kron(out, op if k == i else I2, format="csr")
    return out


def lattice_pairs(kind, Lx, Ly):
    if kind == 0:
        return [(i, (i + 1) % Lx) for i in range(Lx)]
    pairs = []
    for y in range(Ly):
        for x in range(Lx):
            r = x + Lx * y
            pairs.append((r, (x + 1) % Lx + Lx * y))
            pairs.append((r, x + Lx * ((y + 1) % Ly)))
    return pairs


def heisenberg_kron(kind, Lx, Ly=1, J=1.0):
    N = Lx * (Ly if kind == 1 else 1)
    H = sp.csr_matrix((1 << N, 1 << N))
    for (i, j) in lattice_pairs(kind, Lx, Ly):
        H = H + J * (site_op(SZ, i, N) @ site_op(SZ, j, N)
                     + 0.5 * (site_op(SP, i, N) @ site_op(SM, j, N) + site_op(SM, i, N) @ site_op(SP, j, N)))
    return H.tocsr()


def dense_amplitudes(logpsi):
    return np.exp(np.asarray(logpsi))
