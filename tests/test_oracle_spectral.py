"""Pins for the moment-correction matrices (Sec. IV; App. A G and H), the corrected moments,
the Krylov / continued-fraction spectrum (Sec. V) and the Jackson-damped reconstruction (Eq. Aw).

* G and H by enumeration equal <t_n|t_m> and <t_n|H|t_m> from dense vectors and the
  Kronecker-product Hamiltonian (normalised by <psi_gs|psi_gs>);
* with the exact Chebyshev vectors t_0 .. t_{K-1} as basis, the corrected moments equal the exact
  moments for n <= 2K - 1 (the projected resolvent reproduces 2K moments of the true one), and
  they do not depend on the choice of basis of the same span;
* the projected poles reproduce the exact power moments <t_0|H^k|t_0>, k <= 2K - 1, and with a basis
  that spans the whole cyclic space the continued-fraction spectrum is the exact Lorentzian-broadened
  one from diagonalisation;
* Jackson reconstruction: g_0 = 1, the weight integrates to mu_0, the first moment to g_1 mu_1, and
  it is non-negative for exact moments.
"""
import numpy as np
import pytest

import synth
from hilbert import heisenberg_kron
from oracle import exact, spectral


def _ring(N):
    H = exact.heisenberg_sparse(N, [(i, (i + 1) % N) for i in range(N)])
    E0, psi = exact.ground_state(H)
    E_c, W_scale = exact.rescaling(E0)
    return H, E0, psi, E_c, W_scale


@pytest.mark.parametrize("kind,Lx,Ly,M,q", [(0, 8, 1, 8, (np.pi, 0.0)), (1, 3, 3, 6, (2 * np.pi / 3, 0.0))])
def test_moment_matrices_dense(orc, kind, Lx, Ly, M, q):
    N = Lx * Ly
    lat = orc.Lattice(kind, Lx, Ly)
    gs = orc.RBM(*synth.random_rbm_arrays(5, N, M, 0.2, std_im=0.1))
    ts = [orc.RBM(*synth.random_rbm_arrays(6 + t, N, M, 0.2, std_im=0.1)) for t in range(4)]
    betas = np.array([1.0, 0.7 - 0.2j, -0.4 + 0.3j, 1.3j])
    sig = orc.enumerate_configs(N)
    w = orc.enum_weights(orc.logpsi(gs, sig))
    G, H = orc.moment_matrices(gs, ts, betas, q, lat, sig, weights=w)
    psi = np.exp(orc.logpsi(gs, sig))
    norm = np.vdot(psi, psi).real
    f = exact.sz_q_diag(N, exact.positions_of(kind, Lx, Ly, N), q)
    T = np.stack([f * psi] + [b * np.exp(orc.logpsi(t, sig)) for b, t in zip(betas, ts)], axis=1)
    Hk = heisenberg_kron(kind, Lx, Ly)
    assert np.allclose(G, T.conj().T @ T / norm, rtol=1e-10, atol=1e-12)
    assert np.allclose(H, T.conj().T @ (Hk @ T) / norm, rtol=1e-10, atol=1e-12)
    # the first row of G is the moment definition used by the Chebyshev-moment estimator
    mu = orc.moments(gs, ts, betas, [q], lat, sig, weights=w)[0]
    assert np.allclose(G[0], mu, rtol=1e-12, atol=1e-14)


def test_jackson_factors():
    g = spectral.jackson(64)
    assert abs(g[0] - 1.0) < 1e-15
    assert np.all(np.diff(g) < 0) and np.all(g > 0)
    # a single moment gives the flat density of the Chebyshev weight, N = 1: g_0 = 1
    assert abs(spectral.jackson(1)[0] - 1.0) < 1e-15


def _random_problem(dim=40, seed=3):
    """A Hermitian H with spectrum in [-2, 3], a start vector, and the exact Chebyshev vectors of
    H' = (H - E_c)/W_scale (the identities below are statements of linear algebra)."""
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.normal(size=(dim, dim)) + 1j * r.normal(size=(dim, dim)))
    ev = np.sort(r.uniform(-2.0, 3.0, dim))
    H = (Q * ev) @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    t0 = r.normal(size=dim) + 1j * r.normal(size=dim)
    t0 /= np.linalg.norm(t0)
    E_c, W_scale = 0.5, 2.7
    Hp = (H - E_c * np.eye(dim)) / W_scale
    ts = [t0, Hp @ t0]
    for n in range(1, 60):
        ts.append(2.0 * Hp @ ts[n] - ts[n - 1])
    mu = np.array([np.vdot(t0, t) for t in ts])
    return H, t0, E_c, W_scale, ts, mu, ev, np.abs(Q.conj().T @ t0) ** 2


def test_corrected_moments_exact_krylov():
    H, t0, E_c, W_scale, ts, mu_ex, _, _ = _random_problem()
    for K in (3, 5, 8):
        T = np.stack(ts[:K], axis=1)
        G = T.conj().T @ T
        Hm = T.conj().T @ (H @ T)
        mu = spectral.corrected_moments(G, Hm, E_c, W_scale, 2 * K)
        assert np.allclose(mu, mu_ex[:2 * K].real, rtol=0, atol=1e-10), K
        # the span, not the basis, decides: an invertible mixing leaves the moments unchanged
        r = np.random.default_rng(K)
        A = 3 * np.eye(K) + r.normal(size=(K, K)) + 1j * r.normal(size=(K, K))
        A[:, 0] = np.eye(K)[0]               # t_0 itself stays the first vector
        T2 = T @ A
        mu2 = spectral.corrected_moments(T2.conj().T @ T2, T2.conj().T @ (H @ T2), E_c, W_scale, 2 * K)
        assert np.allclose(mu2, mu, atol=1e-9), K
        # beyond 2K - 1 the projected moments are no longer those of H
        mu_far = spectral.corrected_moments(G, Hm, E_c, W_scale, 2 * K + 6)
        assert np.max(np.abs(mu_far[2 * K:] - mu_ex[2 * K:2 * K + 6].real)) > 1e-6, K


def test_projected_poles_power_moments():
    H, t0, E_c, W_scale, ts, _, ev, amp = _random_problem()
    for K in (2, 5, 8):
        T = np.stack(ts[:K], axis=1)
        lam, w = spectral.projected_poles(T.conj().T @ T, T.conj().T @ (H @ T))
        for k in range(2 * K):
            want = np.sum(amp * ev ** k)
            assert abs(np.sum(w * lam ** k) - want) <= 1e-8 * max(1.0, abs(want)), (K, k)
        # Ritz values lie inside the spectrum
        assert lam.min() >= ev.min() - 1e-9 and lam.max() <= ev.max() + 1e-9


def test_cf_spectrum_exact_on_the_cyclic_space():
    N = 8
    H, E0, psi, E_c, W_scale = _ring(N)
    f = exact.sz_q_diag(N, exact.positions_of(0, N, 1, N), (np.pi, 0.0))
    t0 = f * psi / np.linalg.norm(psi)
    Hd = H.toarray()
    ev, V = np.linalg.eigh(Hd)
    amp = np.abs(V.conj().T @ t0) ** 2
    _, ts = exact.chebyshev_moments_exact(H, psi, f, E_c, W_scale, 10)
    # levels carrying weight: with that many Chebyshev vectors the span is the whole cyclic space
    levels = []
    for e, a in zip(ev, amp):
        if a > 1e-14:
            if levels and abs(e - levels[-1][0]) < 1e-9:
                levels[-1][1] += a
            else:
                levels.append([e, a])
    K = len(levels)
    T = np.stack(ts[:K], axis=1)
    omega = np.linspace(-0.5, 6.0, 301)
    eta = 0.1
    A = spectral.cf_spectrum(T.conj().T @ T, T.conj().T @ (Hd @ T), E0, eta, omega)
    ref = sum(a * eta / ((omega + E0 - e) ** 2 + eta ** 2) for e, a in levels) / np.pi
    assert np.allclose(A, ref, rtol=1e-7, atol=1e-9)


def test_kpm_reconstruction_sum_rules():
    N = 8
    H, E0, psi, E_c, W_scale = _ring(N)
    f = exact.sz_q_diag(N, exact.positions_of(0, N, 1, N), (np.pi, 0.0))
    n_mom = 64
    mu, _ = exact.chebyshev_moments_exact(H, psi, f, E_c, W_scale, n_mom - 1)
    # Chebyshev-Gauss nodes integrate polynomial x sqrt(1-x^2) A exactly
    m = 4 * n_mom
    x = np.cos(np.pi * (np.arange(m) + 0.5) / m)
    omega = x * W_scale + E_c - E0
    A = spectral.kpm_spectrum(mu, E0, E_c, W_scale, omega)
    wq = (np.pi / m) * np.sqrt(1 - x * x) * W_scale          # d omega = W_scale dx
    g = spectral.jackson(n_mom)
    assert abs(np.sum(wq * A) - mu[0].real) < 1e-12
    assert abs(np.sum(wq * A * x) - g[1] * mu[1].real) < 1e-12
    assert np.min(A) > -1e-12 * np.max(A)
    # without damping the same sum rules hold (g = 1), but positivity fails (Gibbs oscillations)
    A0 = spectral.kpm_spectrum(mu, E0, E_c, W_scale, omega, damping=False)
    assert abs(np.sum(wq * A0) - mu[0].real) < 1e-12
    assert np.min(A0) < -1e-3 * np.max(A0)
