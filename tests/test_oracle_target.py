"""Pins for the Chebyshev target ratio R = phi / psi_{n+1} (Sec. III recursion of targets).

phi is assembled as a dense vector over all 2^N configurations with the
Kronecker-product Hamiltonian and the enumerated RBM amplitudes, then
compared pointwise with the oracle's per-configuration ratio, and its
|psi_{n+1}|^2-weighted mean is compared with <psi_{n+1}|phi>/<psi_{n+1}|psi_{n+1}>.
"""
import numpy as np
import pytest

import synth
from hilbert import heisenberg_kron
from oracle import exact


@pytest.mark.parametrize("order", [0, 1, 2, 5])
@pytest.mark.parametrize("kind,Lx,Ly", [(0, 8, 1), (1, 3, 2)])
def test_target_ratio_dense(orc, order, kind, Lx, Ly):
    N = Lx * Ly
    M = 5
    lat = orc.Lattice(kind, Lx, Ly)
    fit = orc.RBM(*synth.random_rbm_arrays(100 + order, N, M, 0.3))
    psn = orc.RBM(*synth.random_rbm_arrays(200 + order, N, M, 0.3))
    psm = orc.RBM(*synth.random_rbm_arrays(300 + order, N, M, 0.3))
    E_c, W_scale = -1.7, 3.1
    beta_n, beta_nm1 = 0.8 - 0.3j, 1.2 + 0.1j
    q = (np.pi / 2, np.pi) if kind == 1 else (2 * np.pi * 3 / N, 0.0)
    sig = orc.enumerate_configs(N)
    H = heisenberg_kron(kind, Lx, Ly)
    f = exact.sz_q_diag(N, exact.positions_of(kind, Lx, Ly, N), q)
    v1 = np.exp(orc.logpsi(fit, sig))
    vn = np.exp(orc.logpsi(psn, sig))
    Ht = lambda v: (H @ v - E_c * v) / W_scale
    if order == 0:
        phi = beta_n * Ht(f * vn)
        R = orc.target_ratio(fit, psn, None, lat, sig, 0, E_c, W_scale, beta_n, beta_nm1, q)
    elif order == 1:
        phi = 2 * beta_n * Ht(vn) - beta_nm1 * f * np.exp(orc.logpsi(psm, sig))
        R = orc.target_ratio(fit, psn, psm, lat, sig, 1, E_c, W_scale, beta_n, beta_nm1, q)
    else:
        phi = 2 * beta_n * Ht(vn) - beta_nm1 * np.exp(orc.logpsi(psm, sig))
        R = orc.target_ratio(fit, psn, psm, lat, sig, order, E_c, W_scale, beta_n, beta_nm1, q)
    assert np.allclose(R, phi / v1, rtol=1e-11, atol=1e-11)
    p = orc.enum_weights(orc.logpsi(fit, sig))
    assert abs(np.sum(p * R) - np.vdot(v1, phi) / np.vdot(v1, v1)) < 1e-11


def test_hpsi_is_local_energy(orc):
    N, M = 8, 4
    lat = orc.Lattice(0, N)
    fit = orc.RBM(*synth.random_rbm_arrays(1, N, M, 0.3))
    psn = orc.RBM(*synth.random_rbm_arrays(2, N, M, 0.3))
    sig = synth.random_spins(3, 40, N, True)
    _, hp = orc.target_ratio(fit, psn, psn, lat, sig, 3, 0.0, 1.0, return_hpsi=True)
    assert np.allclose(hp, orc.local_energy(psn, lat, sig), rtol=1e-13, atol=1e-13)
