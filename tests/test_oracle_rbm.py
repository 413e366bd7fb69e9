"""Pins for the oracle's RBM amplitude, local energy and log-derivatives.

* special cases with closed forms (all-zero parameters, W = 0);
* E_loc(sigma) = (H psi)(sigma) / psi(sigma) with H assembled from Kronecker
  products (independent of the oracle's bit-level construction);
* O_k = d log psi / d alpha_k against central finite differences of log psi,
  along both the real and the imaginary direction (holomorphy).
"""
import numpy as np
import pytest

import synth
from hilbert import heisenberg_kron


def _rbm(orc, seed, N, M, std=0.1, std_w=None):
    return orc.RBM(*synth.random_rbm_arrays(seed, N, M, std, std_w))


def test_zero_parameters_closed_form(orc):
    N, M = 10, 7
    rbm = orc.RBM(np.zeros(N), np.zeros(M), np.zeros((N, M)))
    sig = orc.enumerate_configs(N)
    lp = orc.logpsi(rbm, sig)
    assert np.allclose(lp, M * np.log(2.0), atol=1e-13)
    lat = orc.Lattice(0, N)
    el = orc.local_energy(rbm, lat, sig)
    # psi is constant, so every off-diagonal matrix element of each bond contributes
    # J/2 and the diagonal J/4 sigma_i sigma_j: the sum is J*N_b/4 for every sigma.
    assert np.allclose(el, 0.25 * N, atol=1e-12)
    lat2 = orc.Lattice(1, 4, 3)
    sig2 = synth.random_spins(3, 50, 12)
    rbm2 = orc.RBM(np.zeros(12), np.zeros(5), np.zeros((12, 5)))
    assert np.allclose(orc.local_energy(rbm2, lat2, sig2), 0.25 * 24, atol=1e-12)


def test_product_state_closed_form(orc):
    N, M = 8, 5
    a, b, _ = synth.random_rbm_arrays(4, N, M, 0.7)
    rbm = orc.RBM(a, b, np.zeros((N, M)))
    sig = synth.random_spins(5, 64, N)
    want = sig @ a + np.sum(np.log(2.0 * np.cosh(b)))
    got = orc.logpsi(rbm, sig)
    assert np.allclose(got.real, want.real, atol=1e-12)
    d = np.angle(np.exp(1j * (got.imag - want.imag)))
    assert np.all(np.abs(d) < 1e-12)


@pytest.mark.parametrize("kind,Lx,Ly,M", [(0, 8, 1, 8), (0, 6, 1, 3), (1, 3, 3, 4), (1, 4, 2, 6), (1, 2, 2, 3)])
def test_local_energy_equals_hamiltonian_action(orc, kind, Lx, Ly, M):
    N = Lx * Ly
    rbm = _rbm(orc, 10 + N + M, N, M, std=0.3)
    lat = orc.Lattice(kind, Lx, Ly)
    sig = orc.enumerate_configs(N)
    psi = np.exp(orc.logpsi(rbm, sig))
    H = heisenberg_kron(kind, Lx, Ly)
    want = (H @ psi) / psi
    got = orc.local_energy(rbm, lat, sig)
    assert np.allclose(got, want, rtol=1e-11, atol=1e-11)


def test_logderiv_finite_differences(orc):
    N, M = 6, 4
    rbm = _rbm(orc, 21, N, M, std=0.4)
    sig = synth.random_spins(22, 16, N)
    O = orc.logderiv(rbm, sig)
    v0 = rbm.vector()
    h = 1e-5
    for k in range(rbm.P):
        for dirn in (1.0, 1j):
            vp, vm = v0.copy(), v0.copy()
            vp[k] += h * dirn
            vm[k] -= h * dirn
            lp = orc.logpsi(orc.RBM.from_vector(vp, N, M), sig)
            lm = orc.logpsi(orc.RBM.from_vector(vm, N, M), sig)
            fd = (lp - lm) / (2 * h * dirn)
            assert np.allclose(fd, O[:, k], rtol=1e-7, atol=1e-8), (k, dirn)


def test_enum_weights(orc):
    N, M = 8, 6
    rbm = _rbm(orc, 31, N, M, std=0.5)
    sig = orc.enumerate_configs(N)
    lp = orc.logpsi(rbm, sig)
    p = orc.enum_weights(lp)
    psi = np.exp(lp)
    want = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    assert np.allclose(p, want, rtol=1e-12, atol=0)
    assert abs(p.sum() - 1.0) < 1e-13


def test_lattice_bonds(orc):
    assert orc.Lattice(0, 5).bonds().tolist() == [[0, 1], [1, 2], [2, 3], [3, 4], [4, 0]]
    b = orc.Lattice(1, 3, 2).bonds()
    assert b.shape == (12, 2)
    # every site has degree 4 on the square lattice (duplicates kept when a side is 2)
    deg = np.bincount(b.ravel(), minlength=6)
    assert np.all(deg == 4)
