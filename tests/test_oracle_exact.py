"""Pins for the exact-vector references (Heisenberg matrix, ED, exact Chebyshev moments).

* the oracle's bit-level Heisenberg matrix equals the Kronecker-product one;
* ED ground energies: the 4-site ring has E_0 = -2 J (closed form);
* sum rule (1/N) sum_q S(q) = 1/4 (Parseval; (S^z)^2 = 1/4);
* f-sum rule for the isotropic chain: <t_0|(H - E_0)|t_0> = -(2/3)(1 - cos q) E_0 / N;
* exact Chebyshev moments equal sum_k |<k|t_0>|^2 T_n(lambda_k) (numpy's
  Chebyshev evaluation on the eigen-decomposition), the KPM doubling
  identities, and |mu_n| <= mu_0;
* the Chebyshev window of Sec. II maps E_0 to -W' and keeps the spectrum in [-1, 1].
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from hilbert import heisenberg_kron
from oracle import exact


@pytest.mark.parametrize("kind,Lx,Ly", [(0, 8, 1), (0, 10, 1), (1, 3, 3), (1, 4, 2)])
def test_bit_matrix_equals_kron(orc, kind, Lx, Ly):
    lat = orc.Lattice(kind, Lx, Ly)
    Hb = exact.heisenberg_sparse(lat.N, lat.bonds())
    Hk = heisenberg_kron(kind, Lx, Ly)
    assert abs(Hb - Hk).max() < 1e-14


def test_four_site_ring(orc):
    lat = orc.Lattice(0, 4)
    E0, _ = exact.ground_state(exact.heisenberg_sparse(4, lat.bonds()))
    assert abs(E0 - (-2.0)) < 1e-12


def _ring10(orc):
    lat = orc.Lattice(0, 10)
    H = exact.heisenberg_sparse(10, lat.bonds())
    E0, gs = exact.ground_state(H)
    return lat, H, E0, gs


def test_structure_factor_sum_rule(orc):
    lat, H, E0, gs = _ring10(orc)
    pos = exact.positions_of(0, 10, 1, 10)
    S = []
    for k in range(10):
        f = exact.sz_q_diag(10, pos, (2 * np.pi * k / 10, 0.0))
        S.append(np.vdot(f * gs, f * gs).real)
    assert abs(np.mean(S) - 0.25) < 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_f_sum_rule_chain(orc, k):
    lat, H, E0, gs = _ring10(orc)
    q = 2 * np.pi * k / 10
    f = exact.sz_q_diag(10, exact.positions_of(0, 10, 1, 10), (q, 0.0))
    t0 = f * gs
    lhs = np.vdot(t0, H @ t0 - E0 * t0).real
    rhs = -(2.0 / 3.0) * (1.0 - np.cos(q)) * E0 / 10
    assert abs(lhs - rhs) < 1e-12


def test_exact_chebyshev_moments(orc):
    lat, H, E0, gs = _ring10(orc)
    E_c, W_scale = exact.rescaling(E0)
    f = exact.sz_q_diag(10, exact.positions_of(0, 10, 1, 10), (np.pi, 0.0))
    n_max = 40
    mu, ts = exact.chebyshev_moments_exact(H, gs, f, E_c, W_scale, n_max)
    lam, V = np.linalg.eigh(H.toarray())
    x = (lam - E_c) / W_scale
    assert abs(x[0] + exact.W_PRIME) < 1e-12          # E_0 -> -W'
    assert np.all(np.abs(x) <= 1.0)
    wts = np.abs(V.T @ (f * gs)) ** 2
    for n in range(n_max + 1):
        c = np.zeros(n + 1)
        c[n] = 1.0
        assert abs(mu[n] - np.sum(wts * npcheb.chebval(x, c))) < 1e-12
    for n in range(1, n_max // 2):
        assert abs(mu[2 * n] - (2 * np.vdot(ts[n], ts[n]) - mu[0])) < 1e-12
        assert abs(mu[2 * n + 1] - (2 * np.vdot(ts[n + 1], ts[n]) - mu[1])) < 1e-12
    assert np.all(np.abs(mu) <= mu[0].real + 1e-12)
