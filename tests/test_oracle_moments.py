"""Pins for the sampled Chebyshev moments (Sec. II definition, App. A momentum form).

In enumeration mode with |psi_gs|^2 weights, mu_n must equal
beta_n <t_0|t~_n> / <psi_gs|psi_gs> with t_0 = S^z_q psi_gs built as dense
vectors, and mu_0 must satisfy the structure-factor sum rule on the full
Brillouin-zone grid for any state.  With exact Chebyshev vectors in place of
RBMs the recursion reproduces the exact moments.
"""
import numpy as np

import synth
from oracle import exact


def test_moments_dense_overlaps(orc):
    N, M = 8, 4
    lat = orc.Lattice(0, N)
    gs = orc.RBM(*synth.random_rbm_arrays(40, N, M, 0.4))
    ts = [orc.RBM(*synth.random_rbm_arrays(41 + n, N, M, 0.4)) for n in range(4)]
    betas = np.array([1.1, 0.9 - 0.2j, -0.5 + 0.1j, 0.3j])
    qs = np.array([[np.pi, 0.0], [2 * np.pi / N, 0.0]])
    sig = orc.enumerate_configs(N)
    lg = orc.logpsi(gs, sig)
    p = orc.enum_weights(lg)
    mu = orc.moments(gs, ts, betas, qs, lat, sig, weights=p)
    vg = np.exp(lg)
    for iq, q in enumerate(qs):
        f = exact.sz_q_diag(N, exact.positions_of(0, N, 1, N), q)
        t0 = f * vg
        assert abs(mu[iq, 0] - np.vdot(t0, t0) / np.vdot(vg, vg)) < 1e-12
        for n, t in enumerate(ts, start=1):
            vt = np.exp(orc.logpsi(t, sig))
            assert abs(mu[iq, n] - betas[n - 1] * np.vdot(t0, vt) / np.vdot(vg, vg)) < 1e-12


def test_mu0_sum_rule(orc):
    lat = orc.Lattice(1, 3, 3)
    gs = orc.RBM(*synth.random_rbm_arrays(3, 9, 5, 0.4))
    sig = orc.enumerate_configs(9)
    p = orc.enum_weights(orc.logpsi(gs, sig))
    qs = [[2 * np.pi * kx / 3, 2 * np.pi * ky / 3] for kx in range(3) for ky in range(3)]
    mu = orc.moments(gs, [], [], qs, lat, sig, weights=p)
    assert abs(mu[:, 0].real.mean() - 0.25) < 1e-13
