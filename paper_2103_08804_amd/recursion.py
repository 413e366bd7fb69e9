"""Chebyshev recursion of variational states (Sec. III), driven through the C ABI only.

Each Chebyshev vector is fitted in turn.  The state t~_{n+1} takes ``n_steps`` natural-gradient steps
toward its target phi_{n+1} (crbm_local_estimators for R and tanh theta, crbm_sr_step for the step),
and its normalisation beta_{n+1} = <R> is read once the steps are done (crbm_fit_stats).  Targets:

    phi_1 = beta_0 H' t~_0,   phi_{n+1} = 2 beta_n H' t~_n - beta_{n-1} t~_{n-1}   (n >= 1),

beta_0 = 1 and t~_0 = t_0 = S^z_q psi_gs.  Two sampling modes:

* enumeration: ``samples`` lists every configuration once and the weights |t~_{n+1}|^2/Z are
  recomputed on the device after every step (crbm_enum_weights);
* Monte Carlo: ``chains`` (int8 [C][N]) run ``sweeps`` Metropolis sweeps of |t~_{n+1}|^2 before every
  step (crbm_sample), uniform weights.

This module does no arithmetic of the method.  It moves parameters (the warm start of t~_{n+1} is a
copy of t~_n, as the paper does not say how a fit starts), reads beta back to the host once per order
(the next target needs it as a call argument), and records the statistics the calls write.
"""
from __future__ import annotations

import dataclasses

import torch

from . import (CHOLESKY, EXCHANGE, FP32, RBM, Plan, chebyshev_moment, enum_weights, fit_stats, local_estimators,
               make_cheb, sample, sr_step)


@dataclasses.dataclass
class FitSettings:
    n_steps: int = 60
    dgamma: float = 0.3
    diag_shift: float = 1e-3
    solver: int = CHOLESKY
    precision: int = FP32
    cg_tol: float = 1e-10
    cg_maxit: int = 1000


@dataclasses.dataclass
class Recursion:
    """Fitted sequence: t_params complex64 [n_max][P] (packed [a|b|W] of t~_1..t~_n_max), betas complex128
    [n_max]; per order the step statistics before the first step (crbm_sr_step stats, float64 [n][8])
    and the fit statistics after the last one (crbm_fit_stats, float64 [n][5])."""
    t_params: torch.Tensor
    betas: torch.Tensor
    first_stats: torch.Tensor
    final_stats: torch.Tensor

    def rbm(self, k: int, N: int, M: int) -> RBM:
        """t~_{k+1} as views into t_params."""
        return RBM.from_packed(self.t_params[k], N, M)


class _Sampling:
    def __init__(self, plan, samples, chains, sweeps, seed):
        self.plan, self.N = plan, plan.N
        self.enum = samples is not None
        if self.enum:
            self.samples = samples
            self.n = samples.shape[0]
            self.weights = torch.empty(self.n, dtype=torch.float64, device=samples.device)
            self.logpsi = torch.empty(self.n, dtype=torch.complex64, device=samples.device)
        else:
            self.chains, self.sweeps, self.seed = chains, sweeps, seed
            C = chains.shape[0]
            self.n = C * sweeps
            self.buf = torch.empty(sweeps, C, self.N, dtype=torch.int8, device=chains.device)
            self.samples = self.buf.view(self.n, self.N)
            self.weights, self.logpsi = None, None
            self.step = 0

    def draw(self, fit):
        """Samples of |fit|^2 (Monte Carlo), or nothing to do (enumeration)."""
        if not self.enum:
            sample(self.plan, fit, self.chains, self.sweeps, EXCHANGE, self.seed, step_offset=self.step,
                   samples_out=self.buf)
            self.step += self.sweeps * self.N

    def reweight(self):
        if self.enum:
            enum_weights(self.plan, self.logpsi, self.weights)


def chebyshev_recursion(plan: Plan, psi_gs: RBM, t1_start: RBM, n_max: int, q, E_c: float, W_scale: float,
                        fit: FitSettings | None = None, samples=None, chains=None, sweeps: int = 1, seed: int = 0,
                        start_order: int = 0, t_params=None, betas=None) -> Recursion:
    """Fit t~_{start_order+1} .. t~_{n_max}.  Orders below start_order are taken from t_params / betas
    (given), so that one order can be refitted from stored predecessors."""
    fit = fit or FitSettings()
    N, M, P = plan.N, plan.M, plan.P
    dev = psi_gs.a.device
    if t_params is None:
        t_params = torch.zeros(n_max, P, dtype=torch.complex64, device=dev)
    if betas is None:
        betas = torch.zeros(n_max, dtype=torch.complex128, device=dev)
    first = torch.zeros(n_max, 8, dtype=torch.float64, device=dev)
    final = torch.zeros(n_max, 5, dtype=torch.float64, device=dev)
    smp = _Sampling(plan, samples, chains, sweeps, seed)
    R = torch.empty(smp.n, dtype=torch.complex64, device=dev)
    T = torch.empty(smp.n, M, dtype=torch.complex64, device=dev)
    stats = torch.empty(8, dtype=torch.float64, device=dev)
    beta_host = [complex(b) for b in betas[:start_order].cpu().tolist()]
    for n in range(start_order, n_max):
        cur = RBM.from_packed(t_params[n], N, M)
        src = t1_start if n == 0 else RBM.from_packed(t_params[n - 1], N, M)
        cur.a.copy_(src.a)
        cur.b.copy_(src.b)
        cur.W.copy_(src.W)
        psi_n = psi_gs if n == 0 else RBM.from_packed(t_params[n - 1], N, M)
        psi_nm1 = None if n == 0 else (psi_gs if n == 1 else RBM.from_packed(t_params[n - 2], N, M))
        cheb = make_cheb(n, E_c, W_scale, 1.0 if n == 0 else beta_host[n - 1],
                         1.0 if n <= 1 else beta_host[n - 2], q)
        for k in range(fit.n_steps + 1):
            smp.draw(cur)
            local_estimators(plan, cur, smp.samples, psi_n=psi_n, psi_nm1=psi_nm1, cheb=cheb, logpsi_out=smp.logpsi,
                             R_out=R, tanh_out=T if k < fit.n_steps else None)
            smp.reweight()
            if k == fit.n_steps:
                fit_stats(plan, R, final[n], weights=smp.weights)
                break
            sr_step(plan, cur, smp.samples, T, R, fit.dgamma, fit.diag_shift, fit.solver, fit.precision, fit.cg_tol,
                    fit.cg_maxit, stats, weights=smp.weights)
            if k == 0:
                first[n].copy_(stats)
        b = final[n, 1:3].cpu().tolist()   # the next target needs beta_{n+1} as a call argument
        beta_host.append(complex(b[0], b[1]))
        betas[n] = beta_host[-1]
    return Recursion(t_params, betas, first, final)


def sequence_moments(plan: Plan, psi_gs: RBM, rec: Recursion, qs, samples, enumeration: bool):
    """mu_n(q), n = 0 .. n_max, of the fitted sequence by samples of |psi_gs|^2 (Sec. II): complex128
    [n_q][n_max + 1].  enumeration: ``samples`` lists every configuration once and is weighted by
    |psi_gs|^2 / Z (crbm_enum_weights); otherwise the samples were drawn from |psi_gs|^2."""
    n = samples.shape[0]
    dev = samples.device
    w = None
    if enumeration:
        lp = torch.empty(n, dtype=torch.complex64, device=dev)
        local_estimators(plan, psi_gs, samples, logpsi_out=lp)
        w = torch.empty(n, dtype=torch.float64, device=dev)
        enum_weights(plan, lp, w)
    mu = torch.zeros(len(qs), rec.t_params.shape[0] + 1, dtype=torch.complex128, device=dev)
    chebyshev_moment(plan, psi_gs, rec.t_params, rec.betas, qs, samples, mu, weights=w)
    return mu
