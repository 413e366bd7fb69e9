"""Exact-vector references over the full 2^N configuration space (test infrastructure only).

* ``heisenberg_sparse``: H = J sum_<ij> S_i . S_j (Sec. VI) as a sparse matrix in
  the S^z basis, built bond by bond from the bit representation of each
  configuration (bit i set <-> sigma_i = +1).
* ``ground_state``: lowest eigenpair (exact diagonalisation).
* ``chebyshev_moments_exact``: the recursion |t_{n+1}> = 2 H~ |t_n> - |t_{n-1}>,
  |t_1> = H~ |t_0>, |t_0> = S^z_q |psi> / ||psi||, and mu_n = <t_0|t_n> (Sec. II),
  with H~ = (H - E_c)/W_scale.
* ``rescaling``: E_c and W_scale from E_0 per the spectral rescaling of Sec. II
  (H' = (H - E_0)/a - W', W' = 1 - 0.0125), with a = W_scale.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

W_PRIME = 1.0 - 0.0125   # rescaled half-bandwidth of Sec. II (W' = 1 - eps/4, eps = 0.05, Sec. VI)


def heisenberg_sparse(N, bonds, J=1.0):
    dim = 1 << N
    s = np.arange(dim, dtype=np.int64)
    diag = np.zeros(dim)
    rows, cols, vals = [], [], []
    for (i, j) in bonds:
        bi = (s >> i) & 1
        bj = (s >> j) & 1
        same = bi == bj
        diag += np.where(same, 0.25 * J, -0.25 * J)
        src = s[~same]
        dst = src ^ ((1 << i) | (1 << j))
        rows.append(dst)
        cols.append(src)
        vals.append(np.full(src.shape[0], 0.5 * J))
    rows.append(s)
    cols.append(s)
    vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(dim, dim))
    H.sum_duplicates()
    return H


def ground_state(H):
    dim = H.shape[0]
    if dim <= 4096:
        w, v = np.linalg.eigh(H.toarray())
        return float(w[0]), v[:, 0]
    w, v = spla.eigsh(H, k=1, which="SA", tol=1e-13)
    return float(w[0]), v[:, 0]


def rescaling(E0, W_scale_factor=1.5):
    """W_scale = factor * |E_0|; E_c = E_0 + W' W_scale so that E_0 maps to -W'."""
    W_scale = W_scale_factor * abs(E0)
    return E0 + W_PRIME * W_scale, W_scale


def sz_q_diag(N, positions, q):
    """Diagonal of S^z_q = N^{-1/2} sum_r e^{-i q.r} S^z_r over all 2^N configurations."""
    s = np.arange(1 << N, dtype=np.int64)
    out = np.zeros(1 << N, np.complex128)
    for r in range(N):
        sz = np.where((s >> r) & 1, 0.5, -0.5)
        ph = q[0] * positions[r][0] + q[1] * positions[r][1]
        out += np.exp(-1j * ph) * sz
    return out / np.sqrt(N)


def positions_of(kind, Lx, Ly, N):
    if kind == 0:
        return [(r, 0) for r in range(N)]
    return [(r % Lx, r // Lx) for r in range(N)]


def chebyshev_moments_exact(H, psi, fdiag, E_c, W_scale, n_max):
    """mu_n = <t_0|T_n(H~)|t_0>, |t_0> = fdiag * psi / ||psi||; also returns the vectors t_n."""
    psi = psi / np.linalg.norm(psi)
    t0 = fdiag * psi
    Ht = lambda v: (H @ v - E_c * v) / W_scale
    ts = [t0]
    if n_max >= 1:
        ts.append(Ht(t0))
    for n in range(1, n_max):
        ts.append(2.0 * Ht(ts[n]) - ts[n - 1])
    mu = np.array([np.vdot(t0, t) for t in ts])
    return mu, ts
