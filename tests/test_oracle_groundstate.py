"""Pins for the ground-state natural-gradient step (energy minimisation of Sec. I with the
metric S of Sec. III).

* F = -lr dE/d conj(alpha) with E(alpha) = <psi|H psi>/<psi|psi> assembled from dense vectors and the
  Kronecker-product Hamiltonian; the derivative by central differences along Re and Im;
* iterating the step in enumeration mode lowers the energy and never goes below the exact ground
  energy (variational principle), approaching it on the 6-site ring.
"""
import numpy as np

import synth
from hilbert import heisenberg_kron
from oracle import exact


def _energy(orc, rbm, H, sig):
    v = np.exp(orc.logpsi(rbm, sig))
    return (np.vdot(v, H @ v) / np.vdot(v, v)).real


def test_energy_gradient_finite_differences(orc):
    N, M = 6, 4
    lat = orc.Lattice(0, N)
    rbm = orc.RBM(*synth.random_rbm_arrays(3, N, M, 0.3))
    sig = orc.enumerate_configs(N)
    H = heisenberg_kron(0, N)
    p = orc.enum_weights(orc.logpsi(rbm, sig))
    El = orc.local_energy(rbm, lat, sig)
    lr = 0.7
    _, info = orc.sr_energy_step(rbm, sig, El, lr, 1e-3, weights=p)
    assert abs(info["E"] - _energy(orc, rbm, H, sig)) < 1e-12
    v0 = rbm.vector()
    h = 1e-5
    for k in range(rbm.P):
        d = []
        for dirn in (1.0, 1j):
            vp, vm = v0.copy(), v0.copy()
            vp[k] += h * dirn
            vm[k] -= h * dirn
            d.append((_energy(orc, orc.RBM.from_vector(vp, N, M), H, sig)
                      - _energy(orc, orc.RBM.from_vector(vm, N, M), H, sig)) / (2 * h))
        dE_dconj = 0.5 * complex(d[0], d[1])
        assert abs(info["F"][k] - (-lr) * dE_dconj) < 1e-8, k


def test_energy_descent_is_variational(orc):
    N, M = 6, 6
    lat = orc.Lattice(0, N)
    sig = orc.enumerate_configs(N)
    E0, _ = exact.ground_state(exact.heisenberg_sparse(N, lat.bonds()))
    rbm = orc.RBM(*synth.random_rbm_arrays(4, N, M, 0.1))
    energies = []
    for _ in range(60):
        p = orc.enum_weights(orc.logpsi(rbm, sig))
        El = orc.local_energy(rbm, lat, sig)
        rbm, info = orc.sr_energy_step(rbm, sig, El, 0.1, 1e-3, weights=p)
        energies.append(info["E"].real)
        assert info["E"].real >= E0 - 1e-10          # variational bound
    assert energies[-1] < energies[0] - 0.5
    assert all(b <= a + 1e-9 for a, b in zip(energies[5:], energies[6:]))
    assert energies[-1] - E0 < 0.1
