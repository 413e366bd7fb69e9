"""FP64 twin of the Chebyshev recursion of variational states (test infrastructure only).

Sec. III fits each Chebyshev vector in turn.  The state t~_{n+1} is moved toward its target
phi_{n+1} by natural-gradient steps (Fubini-Study rotation by dgamma * gamma, projected onto the
RBM manifold through S), and once the steps are done its normalisation is beta_{n+1} = <R> with
R = phi_{n+1}/t~_{n+1} over samples of |t~_{n+1}|^2.  The targets are

    phi_1 = beta_0 H' t~_0,   phi_{n+1} = 2 beta_n H' t~_n - beta_{n-1} t~_{n-1}   (n >= 1),

with beta_0 = 1 and t~_0 = t_0 = S^z_q psi_gs (Sec. II: t_0 = A|psi>, the operator of App. B).
Here every expectation is exact: the samples are all 2^N configurations, weighted by
|t~_{n+1}|^2 / <t~_{n+1}|t~_{n+1}> (recomputed after every step).  The moments follow Sec. II:
mu_n = <t_0|beta_n t~_n> / <psi_gs|psi_gs>, by the configurations weighted with |psi_gs|^2.

Every step calls the oracle's definitions (log psi, the target ratio, the step with its dense
Cholesky solve, the moments); nothing here is shared with the GPU path.  The first fitted state
starts from a caller-given RBM, each later one from a copy of the state fitted before it (a warm
start; the paper does not say how a fit starts).
"""
from __future__ import annotations

import numpy as np

from . import enum_weights, enumerate_configs, logpsi, moments, sr_step, target_ratio


def fit_stats(fit, psi_n, psi_nm1, lat, sig, order, E_c, W_scale, beta_n, beta_nm1, q):
    """(gamma, beta) of the current fit: gamma = arccos sqrt(|<R>|^2/<|R|^2>), beta = <R> (Sec. III)."""
    p = enum_weights(logpsi(fit, sig))
    R = target_ratio(fit, psi_n, psi_nm1, lat, sig, order, E_c, W_scale, beta_n, beta_nm1, q)
    beta = complex(np.sum(p * R))
    r2 = float(np.sum(p * np.abs(R) ** 2))
    gamma = float(np.arccos(min(1.0, np.sqrt(abs(beta) ** 2 / r2))))
    return gamma, beta


def fit_order(n, start, psi_gs, ts, betas, lat, q, E_c, W_scale, n_steps, dgamma, diag_shift):
    """Fit t~_{n+1} from ``start`` by n_steps steps, the earlier states ts[k] = t~_{k+1} and betas[k] =
    beta_{k+1} given.  Returns (fitted RBM, beta_{n+1}, gamma before the first step, gamma after the last)."""
    sig = enumerate_configs(lat.N)
    fit = start.copy()
    psi_n = psi_gs if n == 0 else ts[n - 1]
    psi_nm1 = None if n == 0 else (psi_gs if n == 1 else ts[n - 2])
    beta_n = 1.0 if n == 0 else betas[n - 1]
    beta_nm1 = 1.0 if n <= 1 else betas[n - 2]
    g_first = None
    for k in range(n_steps):
        p = enum_weights(logpsi(fit, sig))
        R = target_ratio(fit, psi_n, psi_nm1, lat, sig, n, E_c, W_scale, beta_n, beta_nm1, q)
        fit, info = sr_step(fit, sig, R, dgamma, diag_shift, weights=p)
        if k == 0:
            g_first = info["gamma"]
    gamma, beta = fit_stats(fit, psi_n, psi_nm1, lat, sig, n, E_c, W_scale, beta_n, beta_nm1, q)
    return fit, beta, g_first, gamma


def moments_of(psi_gs, ts, betas, lat, q):
    """mu_0 .. mu_len(ts) of S^z_q on psi_gs with every configuration weighted by |psi_gs|^2 (Sec. II)."""
    sig = enumerate_configs(lat.N)
    p_gs = enum_weights(logpsi(psi_gs, sig))
    return moments(psi_gs, ts, betas, [q], lat, sig, weights=p_gs)[0]


def chebyshev_recursion(psi_gs, lat, q, E_c, W_scale, n_max, n_steps, dgamma, diag_shift, t1_start):
    """Fit t~_1 .. t~_{n_max} by n_steps natural-gradient steps each, in exact-enumeration mode.

    Returns dict(ts: list of fitted RBMs, betas: complex [n_max], gamma_first, gamma_last: the angle
    before the first and after the last step of each order, mu: complex [n_max + 1] the moments
    of S^z_q on psi_gs).  E_c, W_scale: H' = (H - E_c)/W_scale (Sec. II)."""
    ts, betas, g_first, g_last = [], [], [], []
    for n in range(n_max):
        start = t1_start if n == 0 else ts[-1]
        fit, beta, g0, g1 = fit_order(n, start, psi_gs, ts, betas, lat, q, E_c, W_scale, n_steps, dgamma,
                                      diag_shift)
        ts.append(fit)
        betas.append(beta)
        g_first.append(g0)
        g_last.append(g1)
    mu = moments_of(psi_gs, ts, betas, lat, q)
    return dict(ts=ts, betas=np.array(betas), gamma_first=np.array(g_first), gamma_last=np.array(g_last), mu=mu)
