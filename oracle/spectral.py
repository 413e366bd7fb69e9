"""FP64 reference for the post-processing of Chebyshev moments (arXiv:2103.08804).

TEST INFRASTRUCTURE ONLY: used by ``tests/`` and the benchmark's CPU leg,
never by the GPU library.

* ``jackson``: the damping factors g_n quoted with the results (Sec. VI).
* ``kpm_spectrum``: the Chebyshev reconstruction of A(omega), Eq. (Aw) of Sec. II.
* ``corrected_moments``: Sec. IV, the Chebyshev recursion repeated inside the
  span of the stored vectors, from their overlap matrix sigma (here G) and
  Hamiltonian matrix H.
* ``cf_spectrum``: Sec. V, the Krylov (continued-fraction) spectrum of the
  Hamiltonian projected onto that span, written as its plain definition: the
  spectral decomposition of the projected resolvent, from the generalised
  eigenproblem H u = lambda G u.  A continued fraction built by Lanczos on the
  same span is the same rational function of z.

Conventions.  G_nm = <t_n|t_m> and H_nm = <t_n|H|t_m> are normalised by
<psi_gs|psi_gs>, with t_0 = A|psi_gs>; H is the physical Hamiltonian.  The
rescaled operator is H' = (H - E_c)/W_scale, so its matrix in the basis is
(H - E_c G)/W_scale.  Both Hermitian-part readings (H <- (H + H^dagger)/2,
real parts of the moments) are applied here and in the GPU path alike.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def jackson(n_mom: int) -> np.ndarray:
    """g_n, n = 0 .. n_mom-1, with N = n_mom moments (Sec. VI):
    g_n = [(N - n + 1) cos(pi n/(N+1)) + sin(pi n/(N+1)) cot(pi/(N+1))] / (N + 1)."""
    N = n_mom
    n = np.arange(N, dtype=np.float64)
    a = np.pi / (N + 1)
    return ((N - n + 1) * np.cos(a * n) + np.sin(a * n) / np.tan(a)) / (N + 1)


def kpm_spectrum(mu, E0: float, E_c: float, W_scale: float, omega, damping: bool = True) -> np.ndarray:
    """A(omega) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (pi W_scale sqrt(1 - x^2)),
    x = (E0 + omega - E_c) / W_scale, omega the excitation energy (Eq. Aw with a = W_scale);
    T_n(x) = cos(n arccos x).  Zero outside |x| < 1.  Real parts of the moments are used."""
    mu = np.real(np.asarray(mu, np.complex128))
    g = jackson(len(mu)) if damping else np.ones(len(mu))
    x = (E0 + np.asarray(omega, np.float64) - E_c) / W_scale
    out = np.zeros_like(x)
    inside = np.abs(x) < 1.0
    xi = x[inside]
    th = np.arccos(xi)
    acc = g[0] * mu[0] * np.ones_like(xi)
    for n in range(1, len(mu)):
        acc += 2.0 * g[n] * mu[n] * np.cos(n * th)
    out[inside] = acc / (np.pi * W_scale * np.sqrt(1.0 - xi * xi))
    return out


def _hermitian(H):
    H = np.asarray(H, np.complex128)
    return 0.5 * (H + H.conj().T)


def corrected_moments(G, H, E_c: float, W_scale: float, n_out: int) -> np.ndarray:
    """mu'_n, n = 0 .. n_out-1, of |t'_n> = T_n(H_P)|t_0> (Sec. IV):
    c_0 = e_0;  G c_1 = H' c_0;  G c_{n+1} = 2 H' c_n - G c_{n-1};  mu'_n = sum_ml conj(c_m0) G_ml c_ln,
    with H' = (H - E_c G)/W_scale the rescaled Hamiltonian in the basis."""
    G = _hermitian(G)
    Hp = (_hermitian(H) - E_c * G) / W_scale
    K = G.shape[0]
    c_prev = np.zeros(K, np.complex128)
    c_prev[0] = 1.0
    mu = np.zeros(n_out, np.complex128)
    mu[0] = np.vdot(c_prev, G @ c_prev)
    if n_out == 1:
        return mu.real
    c = np.linalg.solve(G, Hp @ c_prev)
    mu[1] = np.vdot(c_prev, G @ c)
    for n in range(2, n_out):
        c_next = np.linalg.solve(G, 2.0 * (Hp @ c) - G @ c_prev)
        mu[n] = np.vdot(np.eye(K)[0], G @ c_next)
        c_prev, c = c, c_next
    return mu.real


def projected_poles(G, H):
    """(lambda_m, w_m): eigenvalues of H u = lambda G u (u G-orthonormal) and the weights
    w_m = |(G u_m)_0|^2 = |<t_0|u_m>|^2, so that <t_0|(z - H_P)^{-1}|t_0> = sum_m w_m/(z - lambda_m)."""
    G = _hermitian(G)
    lam, U = scipy.linalg.eigh(_hermitian(H), G)
    w = np.abs((G @ U)[0, :]) ** 2
    return lam, w


def cf_spectrum(G, H, E0: float, eta: float, omega) -> np.ndarray:
    """A(omega) = -(1/pi) Im <t_0|(omega + E0 + i eta - H_P)^{-1}|t_0>
                = (1/pi) sum_m w_m eta / ((omega + E0 - lambda_m)^2 + eta^2)."""
    lam, w = projected_poles(G, H)
    z = E0 + np.asarray(omega, np.float64)[:, None]
    return (w[None, :] * eta / ((z - lam[None, :]) ** 2 + eta * eta)).sum(axis=1) / np.pi
