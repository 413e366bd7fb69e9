"""Pins for the oracle's twin of the Chebyshev recursion (Sec. III, moments of Sec. II, correction of Sec. IV).

* Dense twin.  The same loop written over explicit vectors of all 2^N amplitudes: the RBM amplitudes
  from their formula (numpy), H from Kronecker products of spin matrices, the target vector
  phi = 2 beta_n H' t~_n - beta_{n-1} t~_{n-1} (phi = H' t_0 at order 0, t~_0 = t_0 = S^z_q psi_gs),
  R = phi / t~ elementwise, and each step's dalpha as the weighted ridge least-squares solution of
  sum_k dalpha_k (O_k - <O_k>) = dgamma gamma cot gamma (R/<R> - 1) (numpy's lstsq).  The oracle's
  recursion (its log psi, target ratio, step and moment routines) must reproduce the dense twin's
  betas, gammas and moments.
* mu_0 = <|f_q|^2> and, after the Sec. IV correction on the fitted basis, mu_1 = <t_0|H'|t_0>/<psi|psi>
  are exact whatever the fits: t_0 is the first basis vector, so H_P t_0 has the exact overlap with t_0.
"""
import numpy as np

import synth
from hilbert import heisenberg_kron
from oracle import exact, recursion, spectral


def _dense_amplitudes(rbm, sig):
    s = sig.astype(np.float64)
    return np.exp(s @ rbm.a + np.log(2.0 * np.cosh(rbm.b[None, :] + s @ rbm.W)).sum(axis=1))


def _dense_logderiv(rbm, sig):
    s = sig.astype(np.float64)
    T = np.tanh(rbm.b[None, :] + s @ rbm.W)
    return np.hstack([s, T, (s[:, :, None] * T[:, None, :]).reshape(sig.shape[0], -1)])


def _dense_recursion(orc, psi_gs, t1, N, q, E_c, W_scale, n_max, n_steps, dgamma, eps):
    sig = orc.enumerate_configs(N)
    H = heisenberg_kron(0, N).toarray()
    Hs = (H - E_c * np.eye(H.shape[0])) / W_scale
    fq = np.exp(-1j * q[0] * np.arange(N)) @ (0.5 * sig.T.astype(np.float64)) / np.sqrt(N)
    gs = _dense_amplitudes(psi_gs, sig)
    vec = [fq * gs]          # t~_0 = t_0
    betas = [1.0]            # beta_0
    ts, out_b, out_g = [], [], []
    cur = t1.copy()
    for n in range(n_max):
        phi = betas[n] * (Hs @ vec[0]) if n == 0 else 2.0 * betas[n] * (Hs @ vec[n]) - betas[n - 1] * vec[n - 1]
        P = cur.P
        for _ in range(n_steps + 1):
            t = _dense_amplitudes(cur, sig)
            p = np.abs(t) ** 2 / np.sum(np.abs(t) ** 2)
            R = phi / t
            Rm = np.sum(p * R)
            gamma = np.arccos(min(1.0, abs(Rm) / np.sqrt(np.sum(p * np.abs(R) ** 2))))
            if _ == n_steps:
                break
            O = _dense_logderiv(cur, sig)
            Ot = O - p @ O
            D = dgamma * gamma / np.tan(gamma) * (R / Rm - 1.0)
            A = np.vstack([np.sqrt(p)[:, None] * Ot, np.sqrt(eps) * np.eye(P)])
            y = np.concatenate([np.sqrt(p) * D, np.zeros(P)])
            x, *_ = np.linalg.lstsq(A, y, rcond=None)
            v = cur.vector() + x
            cur = orc.RBM.from_vector(v, N, cur.M)
        ts.append(cur.copy())
        vec.append(t)
        betas.append(Rm)
        out_b.append(Rm)
        out_g.append(gamma)
    p_gs = np.abs(gs) ** 2 / np.sum(np.abs(gs) ** 2)
    mu = [np.sum(p_gs * np.abs(fq) ** 2)]
    for n in range(1, n_max + 1):
        mu.append(np.sum(p_gs * np.conj(fq) * betas[n] * vec[n] / gs))
    return np.array(out_b), np.array(out_g), np.array(mu)


def _setup(orc, N, M, seed):
    lat = orc.Lattice(0, N)
    psi_gs = orc.RBM(*synth.random_rbm_arrays(seed, N, M, 0.2, std_im=0.05))
    q = (np.pi, 0.0)
    t1 = psi_gs.copy()
    t1.a = t1.a + 0.1 * np.exp(-1j * q[0] * np.arange(N))
    E0, _ = exact.ground_state(exact.heisenberg_sparse(N, lat.bonds()))
    W_scale = 5.0
    E_c = E0 + exact.W_PRIME * W_scale
    return lat, psi_gs, t1, q, E_c, W_scale


def test_recursion_matches_dense_twin(orc):
    N, M = 6, 3
    lat, psi_gs, t1, q, E_c, W_scale = _setup(orc, N, M, 71)
    n_max, n_steps, dgamma, eps = 4, 6, 0.2, 1e-3
    r = recursion.chebyshev_recursion(psi_gs, lat, q, E_c, W_scale, n_max, n_steps, dgamma, eps, t1)
    b, g, mu = _dense_recursion(orc, psi_gs, t1, N, q, E_c, W_scale, n_max, n_steps, dgamma, eps)
    assert np.allclose(r["betas"], b, rtol=1e-9, atol=0)
    assert np.allclose(r["gamma_last"], g, rtol=1e-8, atol=1e-12)
    assert np.allclose(r["mu"], mu, rtol=1e-9, atol=1e-12)


def test_recursion_fits_reduce_the_angle_and_mu0_mu1_are_exact(orc):
    N, M = 8, 8
    lat, psi_gs, t1, q, E_c, W_scale = _setup(orc, N, M, 72)
    r = recursion.chebyshev_recursion(psi_gs, lat, q, E_c, W_scale, 3, 20, 0.2, 1e-3, t1)
    assert np.all(r["gamma_last"] < r["gamma_first"])
    sig = orc.enumerate_configs(N)
    H = exact.heisenberg_sparse(N, lat.bonds())
    psi = np.exp(orc.logpsi(psi_gs, sig))
    fd = exact.sz_q_diag(N, exact.positions_of(0, N, 1, N), q)
    mu_ex, _ = exact.chebyshev_moments_exact(H, psi, fd, E_c, W_scale, 6)
    assert abs(r["mu"][0] - mu_ex[0]) < 1e-13
    p_gs = orc.enum_weights(orc.logpsi(psi_gs, sig))
    G, Hm = orc.moment_matrices(psi_gs, r["ts"], r["betas"], q, lat, sig, weights=p_gs)
    corr = spectral.corrected_moments(G, Hm, E_c, W_scale, 6)
    assert abs(corr[1] - mu_ex[1].real) < 1e-12
