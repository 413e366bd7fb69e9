"""Pins for the symmetry-projected moment-correction matrices of App. A (oracle ``sym_matrices``).

The projected states are rebuilt here as dense vectors over all 2^N configurations from the
operators themselves: a lattice symmetry g acts by (g v)(s) = v(s o g) with (s o g)_r = s_{g(r)};
  t~_nk = N^{-1/2} sum_m e^{-i k.m} T_m P_R t_n00,   P_R = (1 + T_10 R + T_11 R^2 + T_01 R^3)/4,
R(x, y) = (L-1-y, x).  Then
* G^(k) and H^(k) of the oracle (enumeration weights) equal <t~_nk|t~_n'k>/<psi|psi> and
  <t~_nk|H|t~_n'k>/<psi|psi>, H from Kronecker products (square lattice with rotations, chain);
* the dense construction is a momentum eigenstate, T_a t~_k = e^{i k.a} t~_k, and for the
  (translation- and rotation-invariant) exact ground state, t~_0k = S^z_k psi_0 with the App. B
  normalisation, so <t~_0k|t~_0k> is the static structure factor S(k).
"""
import numpy as np
import pytest

import synth
from hilbert import heisenberg_kron
from oracle import exact


def _site_maps(kind, Lx, Ly):
    """translation maps T[m1][m2][r] and the rotation map R[r] (square lattice)."""
    N = Lx * (Ly if kind == 1 else 1)
    T = np.zeros((Lx, Ly if kind == 1 else 1, N), np.int64)
    for m1 in range(Lx):
        for m2 in range(T.shape[1]):
            for r in range(N):
                x, y = (r, 0) if kind == 0 else (r % Lx, r // Lx)
                T[m1, m2, r] = (x + m1) % Lx + (Lx * ((y + m2) % Ly) if kind == 1 else 0)
    R = None
    if kind == 1:
        R = np.array([(Lx - 1 - r // Lx) + Lx * (r % Lx) for r in range(N)], np.int64)
    return T, R


def _op(g, N):
    """index map of (g v)(s) = v(s o g) over the 2^N basis (bit r <-> site r, set = spin up)."""
    s = np.arange(1 << N, dtype=np.int64)
    out = np.zeros_like(s)
    for r in range(N):
        out |= ((s >> g[r]) & 1) << r
    return out


def _compose(g1, g2):
    return g1[g2]          # (g1 o g2)(r) = g1(g2(r))


def _project(v, k, kind, Lx, Ly, rotations):
    N = v.shape[0].bit_length() - 1
    T, R = _site_maps(kind, Lx, Ly)
    ident = np.arange(N)
    if kind == 1 and rotations:
        R2, R3 = _compose(R, R), _compose(R, _compose(R, R))
        terms = [ident, _compose(T[1, 0], R), _compose(T[1, 1], R2), _compose(T[0, 1], R3)]
        pv = sum(v[_op(g, N)] for g in terms) / 4.0
    else:
        pv = v
    out = np.zeros(v.shape, np.complex128)
    k1, k2 = k
    for m1 in range(T.shape[0]):
        for m2 in range(T.shape[1]):
            ph = 2 * np.pi * (k1 * m1 / Lx + (k2 * m2 / Ly if kind == 1 else 0.0))
            out += np.exp(-1j * ph) * pv[_op(T[m1, m2], N)]
    return out / np.sqrt(N)


@pytest.mark.parametrize("kind,Lx,Ly,M,rot", [(1, 3, 3, 4, True), (0, 8, 1, 6, False), (1, 3, 3, 3, False)])
def test_sym_matrices_dense(orc, kind, Lx, Ly, M, rot):
    lat = orc.Lattice(kind, Lx, Ly)
    N = lat.N
    gs = orc.RBM(*synth.random_rbm_arrays(31, N, M, 0.2, std_im=0.1))
    ts = [orc.RBM(*synth.random_rbm_arrays(32 + t, N, M, 0.2, std_im=0.1)) for t in range(2)]
    betas = np.array([0.8 - 0.3j, 1.2j])
    sig = orc.enumerate_configs(N)
    w = orc.enum_weights(orc.logpsi(gs, sig))
    G, H = orc.sym_matrices(gs, ts, betas, lat, sig, rotations=rot, weights=w)
    psi = np.exp(orc.logpsi(gs, sig))
    norm = np.vdot(psi, psi).real
    s0 = np.where(np.arange(1 << N) & 1, 0.5, -0.5)            # S^z at site 0
    vecs = [s0 * psi] + [b * np.exp(orc.logpsi(t, sig)) for b, t in zip(betas, ts)]
    Hk = heisenberg_kron(kind, Lx, Ly)
    for k2 in range(Ly if kind == 1 else 1):
        for k1 in range(Lx):
            kk = k1 + Lx * k2
            P = np.stack([_project(v, (k1, k2), kind, Lx, Ly, rot) for v in vecs], axis=1)
            Gd = P.conj().T @ P / norm
            Hd = P.conj().T @ (Hk @ P) / norm
            scale = max(np.abs(Gd).max(), 1e-300)
            assert np.allclose(G[kk], Gd, rtol=1e-10, atol=1e-12 * scale), (k1, k2)
            assert np.allclose(H[kk], Hd, rtol=1e-10, atol=1e-12 * np.abs(Hd).max()), (k1, k2)


def test_projection_momentum_and_structure_factor():
    """Dense construction on the 4x4 lattice: momentum eigenstates; for the exact ground state
    t~_0k = S^z_k psi_0, so <t~_0k|t~_0k> = S(k)."""
    kind, L = 1, 4
    N = L * L
    H = exact.heisenberg_sparse(N, [(r, (r % L + 1) % L + L * (r // L)) for r in range(N)] +
                                [(r, r % L + L * ((r // L + 1) % L)) for r in range(N)])
    E0, psi = exact.ground_state(H)
    psi = psi / np.linalg.norm(psi)
    s0 = np.where(np.arange(1 << N) & 1, 0.5, -0.5)
    T, _ = _site_maps(kind, L, L)
    pos = exact.positions_of(kind, L, L, N)
    rng = np.random.default_rng(0)
    v = rng.normal(size=1 << N) + 1j * rng.normal(size=1 << N)
    for k in [(0, 0), (1, 0), (2, 2), (3, 1)]:
        q = (2 * np.pi * k[0] / L, 2 * np.pi * k[1] / L)
        tk = _project(v, k, kind, L, L, True)
        for a in [(1, 0), (0, 1), (2, 3)]:
            shifted = tk[_op(T[a[0], a[1]], N)]
            assert np.allclose(shifted, np.exp(1j * (q[0] * a[0] + q[1] * a[1])) * tk, atol=1e-10)
        t0k = _project(s0 * psi, k, kind, L, L, True)
        fq = exact.sz_q_diag(N, pos, q) * psi
        assert np.allclose(t0k, fq, atol=1e-10)
        assert abs(np.vdot(t0k, t0k).real - np.vdot(fq, fq).real) < 1e-12
