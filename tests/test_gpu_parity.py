"""GPU parity: every entry point of the HIP library against the FP64 oracle.

Tolerances (FP32 kernels vs FP64 definitions): log psi (Re, relative to its
magnitude), local energies, R, tanh theta and O within 1e-5 relative; Im log psi
by the wrapped difference; Philox streams, chain starts, proposals and
Metropolis trajectories bit-exact (decisions replayed with a 1e-4 margin).
"""
import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth
from gpu_util import np_of, rel_err, to_device_rbm, to_oracle_rbm, wrapped

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()


def _plan(kind, Lx, Ly, M, n, flags=0):
    return crbm.Plan(kind, Lx, Ly, M, n, flags)


# ------------------------------------------------------------------ init
@pytest.mark.parametrize("N,M,seed,std", [(10, 10, 1001, 0.01), (100, 400, 1003, 0.01), (7, 3, 5, 0.7)])
def test_init_rbm(orc, N, M, seed, std):
    dev = crbm.RBM.empty(N, M)
    crbm.init_rbm(dev, seed, std)
    torch.cuda.synchronize()
    ref = orc.init_rbm(N, M, seed, std)
    got = to_oracle_rbm(orc, dev)
    for g, r in ((got.a, ref.a), (got.b, ref.b), (got.W, ref.W)):
        assert np.max(np.abs(g - r)) <= 2e-6 * std * 8, np.max(np.abs(g - r))


@pytest.mark.parametrize("N,C,zero", [(10, 33, 1), (40, 1024, 1), (100, 70, 1), (256, 5, 1), (13, 65, 0)])
def test_init_chains_bit_exact(orc, N, C, zero):
    kind, Lx, Ly = (0, N, 1)
    plan = _plan(kind, Lx, Ly, 4, 1)
    s = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, s, 2002, bool(zero))
    torch.cuda.synchronize()
    assert np.array_equal(np_of(s), orc.init_chains(N, C, 2002, zero))


# ------------------------------------------------------------------ local estimators
CASES = [
    # kind, Lx, Ly, M, n_samples (None = full enumeration), Re std, Im std
    (0, 10, 1, 10, None, 0.01, 0.01),
    (0, 10, 1, 10, None, 0.3, 0.02),
    (0, 40, 1, 80, 97, 0.05, 0.02),
    (1, 4, 4, 24, 333, 0.2, 0.02),
    (1, 10, 10, 400, 45, 0.01, 0.01),
    (1, 10, 10, 400, 19, 0.05, 0.02),
    (1, 16, 16, 512, 9, 0.02, 0.01),
]
# With |Im theta| well below pi/2 no theta comes near a zero of cosh, and the FP32 results
# meet the 1e-5 relative bound; test_rounding_bound_near_zeros covers arbitrary phases.


def _samples(orc, N, n, seed):
    if n is None:
        return orc.enumerate_configs(N)
    return synth.random_spins(seed, n, N, zero_magnetisation=(N % 2 == 0))


@pytest.mark.parametrize("kind,Lx,Ly,M,n,std,sim", CASES)
def test_local_energy_logpsi_tanh_O(orc, kind, Lx, Ly, M, n, std, sim):
    N = Lx * Ly
    lat = orc.Lattice(kind, Lx, Ly)
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(7 + N, N, M, std, std_im=sim)))
    fit = to_oracle_rbm(orc, fit_d)
    sig = _samples(orc, N, n, 11 + N)
    ns = sig.shape[0]
    plan = _plan(kind, Lx, Ly, M, ns)
    sig_d = torch.from_numpy(sig).cuda()
    lp = torch.zeros(ns, dtype=torch.complex64, device="cuda")
    el = torch.zeros_like(lp)
    T = torch.zeros(ns, M, dtype=torch.complex64, device="cuda")
    want_O = plan.P * ns <= 4_000_000
    O = torch.zeros(ns, plan.P, dtype=torch.complex64, device="cuda") if want_O else None
    crbm.local_estimators(plan, fit_d, sig_d, logpsi_out=lp, eloc_out=el, tanh_out=T, O_out=O)
    torch.cuda.synchronize()
    lp_ref = orc.logpsi(fit, sig)
    el_ref = orc.local_energy(fit, lat, sig)
    O_ref = orc.logderiv(fit, sig)
    got_lp = np_of(lp).astype(np.complex128)
    assert np.max(np.abs(got_lp.real - lp_ref.real) / np.maximum(np.abs(lp_ref.real), 1.0)) < TOL
    assert np.max(np.abs(wrapped(got_lp.imag - lp_ref.imag))) < TOL * max(1.0, np.abs(lp_ref).max())
    assert rel_err(np_of(el), el_ref) < TOL
    assert rel_err(np_of(T), O_ref[:, N:N + M]) < TOL
    if want_O:
        assert rel_err(np_of(O), O_ref) < TOL


def test_rounding_bound_near_zeros(orc):
    """Arbitrary complex parameters (std 0.3 in Re and Im): some theta_k lie close to a zero of cosh,
    where FP32 rounding of theta is amplified by |tanh theta|.  The errors must stay inside the
    first-order bound derived from that rounding (plus the 1e-5 relative floor)."""
    from gpu_util import eloc_rounding_bound, logpsi_rounding_bound
    N, M = 10, 10
    lat = orc.Lattice(0, N)
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(17, N, M, 0.3)))
    fit = to_oracle_rbm(orc, fit_d)
    sig = orc.enumerate_configs(N)
    plan = _plan(0, N, 1, M, sig.shape[0])
    lp = torch.zeros(sig.shape[0], dtype=torch.complex64, device="cuda")
    el = torch.zeros_like(lp)
    crbm.local_estimators(plan, fit_d, torch.from_numpy(sig).cuda(), logpsi_out=lp, eloc_out=el)
    torch.cuda.synchronize()
    lp_ref = orc.logpsi(fit, sig)
    el_ref = orc.local_energy(fit, lat, sig)
    blp = logpsi_rounding_bound(fit, sig) + TOL * np.maximum(np.abs(lp_ref.real), 1.0)
    assert np.all(np.abs(np_of(lp).real - lp_ref.real) <= blp)
    bel = eloc_rounding_bound(fit, lat.bonds(), sig) + TOL * np.abs(el_ref).max()
    assert np.all(np.abs(np_of(el) - el_ref) <= bel)


@pytest.mark.parametrize("order", [0, 1, 2, 6])
@pytest.mark.parametrize("kind,Lx,Ly,M,n,std,sim", [CASES[1], CASES[3], CASES[5]])
def test_target_ratio(orc, order, kind, Lx, Ly, M, n, std, sim):
    N = Lx * Ly
    lat = orc.Lattice(kind, Lx, Ly)
    rb = lambda s: to_device_rbm(orc.RBM(*synth.random_rbm_arrays(s, N, M, std, std_im=sim)))
    fit_d, psn_d, psm_d = rb(100 + order), rb(200 + order), rb(300 + order)
    fit, psn, psm = (to_oracle_rbm(orc, r) for r in (fit_d, psn_d, psm_d))
    sig = _samples(orc, N, n, 5 + order)
    ns = sig.shape[0]
    E_c, W_scale = -0.6 * N * 0.9875 + 0.1, 1.5 * 0.45 * N
    bn, bm = 0.8 - 0.3j, 1.2 + 0.1j
    q = (np.pi, 0.0) if kind == 0 else (np.pi / 2, np.pi)
    plan = _plan(kind, Lx, Ly, M, ns)
    cheb = crbm.make_cheb(order, E_c, W_scale, bn, bm, q)
    R = torch.zeros(ns, dtype=torch.complex64, device="cuda")
    hp = torch.zeros_like(R)
    crbm.local_estimators(plan, fit_d, torch.from_numpy(sig).cuda(), psi_n=psn_d,
                          psi_nm1=psm_d if order >= 1 else None, cheb=cheb, R_out=R, eloc_out=hp)
    torch.cuda.synchronize()
    R_ref, hp_ref = orc.target_ratio(fit, psn, psm if order >= 1 else None, lat, sig, order, E_c, W_scale, bn, bm,
                                     q, return_hpsi=True)
    assert rel_err(np_of(R), R_ref) < TOL
    assert rel_err(np_of(hp), hp_ref) < TOL


# ------------------------------------------------------------------ Metropolis sampling
@pytest.mark.parametrize("kind,Lx,Ly,M,C,sweeps,proposal,std", [
    (0, 10, 1, 10, 37, 20, 0, 0.3),
    (0, 10, 1, 10, 37, 20, 1, 0.3),
    (0, 40, 1, 80, 64, 8, 1, 0.05),
    (1, 10, 10, 400, 8, 3, 1, 0.02),
    (1, 16, 16, 512, 3, 1, 1, 0.02),
    (1, 4, 4, 24, 129, 10, 0, 0.4),
    (1, 8, 8, 128, 16, 4, 1, 0.05),    # M fills its 64-lane groups exactly
    (0, 6, 1, 1, 70, 30, 1, 0.5),      # one hidden unit: 63 padded lanes
])
def test_sample_replay(orc, kind, Lx, Ly, M, C, sweeps, proposal, std):
    N = Lx * Ly
    psi_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(31 + N, N, M, std, std_im=min(std, 0.02))))
    psi = to_oracle_rbm(orc, psi_d)
    plan = _plan(kind, Lx, Ly, M, 1)
    spins = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, spins, 2000 + N, proposal == 1)
    s0 = np_of(spins).copy()
    words = (sweeps * N + 31) // 32
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    nacc = torch.zeros(C, dtype=torch.int32, device="cuda")
    trace = torch.zeros(C, words, dtype=torch.int32, device="cuda")
    theta = torch.zeros(C, M, dtype=torch.complex64, device="cuda")
    lp = torch.zeros(C, dtype=torch.complex64, device="cuda")
    seed, off = 77 + N, 1234
    crbm.sample(plan, psi_d, spins, sweeps, proposal, seed, off, theta_out=theta, logpsi_out=lp,
                samples_out=samples, n_accept=nacc, trace=trace)
    torch.cuda.synchronize()
    s_ref = s0.copy()
    tr = np_of(trace).view(np.uint32)
    smp_ref, nacc_ref, amb, mis = orc.metropolis(psi, s_ref, sweeps, proposal, seed, off, trace=tr)
    assert mis == 0
    assert np.array_equal(np_of(samples), smp_ref)
    assert np.array_equal(np_of(spins), s_ref)
    assert np.array_equal(np_of(nacc).view(np.uint32), nacc_ref)
    total_moves = sweeps * N * C
    assert amb <= max(3, 1e-3 * total_moves)
    # state of the chains at the end
    lp_ref = orc.logpsi(psi, s_ref)
    got = np_of(lp).astype(np.complex128)
    assert np.max(np.abs(got.real - lp_ref.real) / np.maximum(np.abs(lp_ref.real), 1.0)) < TOL
    th_ref = orc.RBM(psi.a, psi.b, psi.W)
    theta_ref = psi.b[None, :] + s_ref.astype(np.float64) @ psi.W
    assert rel_err(np_of(theta), theta_ref) < 1e-5


def test_sample_continuation_matches_single_call(orc):
    """Two calls with step_offset continue the same Philox streams as one longer call."""
    N, M, C = 12, 6, 20
    psi_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(3, N, M, 0.3)))
    plan = _plan(0, N, 1, M, 1)
    a = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, a, 9, True)
    b = a.clone()
    sa = torch.zeros(6, C, N, dtype=torch.int8, device="cuda")
    crbm.sample(plan, psi_d, a, 6, 1, 5, 0, samples_out=sa)
    s1 = torch.zeros(2, C, N, dtype=torch.int8, device="cuda")
    s2 = torch.zeros(4, C, N, dtype=torch.int8, device="cuda")
    crbm.sample(plan, psi_d, b, 2, 1, 5, 0, samples_out=s1)
    crbm.sample(plan, psi_d, b, 4, 1, 5, 2 * N, samples_out=s2)
    torch.cuda.synchronize()
    assert torch.equal(torch.cat([s1, s2]), sa)
    assert torch.equal(a, b)


def test_degenerate_calls(orc):
    """Zero-length calls: no sweeps (spins untouched, no accepted moves, theta and log psi of the start
    states against the oracle, one chain and five), no samples (the call succeeds and writes nothing),
    one sample, and moments up to order 0 only (mu_0 against the oracle)."""
    kind, Lx, Ly, M = 1, 4, 4, 24
    N = Lx * Ly
    lat = orc.Lattice(kind, Lx, Ly)
    psi_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(41, N, M, 0.2, std_im=0.02)))
    psi = to_oracle_rbm(orc, psi_d)
    plan = _plan(kind, Lx, Ly, M, 64)
    for C in (1, 5):
        spins = torch.zeros(C, N, dtype=torch.int8, device="cuda")
        crbm.init_chains(plan, spins, 17, True)
        s0 = spins.clone()
        theta = torch.zeros(C, M, dtype=torch.complex64, device="cuda")
        lp = torch.zeros(C, dtype=torch.complex64, device="cuda")
        nacc = torch.full((C,), 7, dtype=torch.int32, device="cuda")
        crbm.sample(plan, psi_d, spins, 0, crbm.EXCHANGE, 5, 0, theta_out=theta, logpsi_out=lp, n_accept=nacc)
        torch.cuda.synchronize()
        assert torch.equal(spins, s0)
        assert int(nacc.abs().sum()) == 0
        sig = np_of(s0)
        assert rel_err(np_of(theta), psi.b[None, :] + sig.astype(np.float64) @ psi.W) < TOL
        lp_ref = orc.logpsi(psi, sig)
        assert np.all(np.abs(np_of(lp).real - lp_ref.real) <= TOL * np.maximum(np.abs(lp_ref.real), 1.0))
        assert np.all(np.abs(wrapped(np_of(lp).imag - lp_ref.imag)) <= 1e-4)

    # no samples: energy mode and Chebyshev mode return without writing
    cheb = crbm.make_cheb(1, -5.0, 8.0, 0.9, 1.1, (np.pi, np.pi))
    empty = torch.zeros(0, N, dtype=torch.int8, device="cuda")
    out0 = torch.zeros(0, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, psi_d, empty, logpsi_out=out0, eloc_out=out0)
    crbm.local_estimators(plan, psi_d, empty, psi_n=psi_d, psi_nm1=psi_d, cheb=cheb, R_out=out0)
    # one sample
    one = synth.random_spins(3, 1, N, zero_magnetisation=True)
    el = torch.zeros(1, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, psi_d, torch.from_numpy(one).cuda(), eloc_out=el)
    torch.cuda.synchronize()
    assert rel_err(np_of(el), orc.local_energy(psi, lat, one)) < TOL

    # moments with no Chebyshev vectors: mu_0 alone
    sig = synth.random_spins(8, 64, N, zero_magnetisation=True)
    qs = [(np.pi, np.pi), (np.pi / 2, 0.0)]
    mu = torch.zeros(len(qs), 1, dtype=torch.complex128, device="cuda")
    crbm.chebyshev_moment(plan, psi_d, None, None, qs, torch.from_numpy(sig).cuda(), mu)
    torch.cuda.synchronize()
    assert rel_err(np_of(mu), orc.moments(psi, [], [], qs, lat, sig)) < TOL


# ------------------------------------------------------------------ natural-gradient step
def _sr_inputs(orc, N, M, std, seed):
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(seed, N, M, std)))
    fit = to_oracle_rbm(orc, fit_d)
    sig = orc.enumerate_configs(N)
    p = orc.enum_weights(orc.logpsi(fit, sig))
    r = np.random.default_rng(seed)
    R = (1.0 + 0.4 * r.normal(size=sig.shape[0]) + 0.3j * r.normal(size=sig.shape[0])).astype(np.complex64)
    return fit_d, fit, sig, p, R


@pytest.mark.parametrize("solver,flags", [(crbm.CG_DENSE, crbm.PLAN_DENSE_S), (crbm.CG_MATFREE, 0),
                                          (crbm.CHOLESKY, crbm.PLAN_CHOLESKY)])
def test_sr_step_enumeration(orc, solver, flags):
    N, M = 10, 10
    fit_d, fit, sig, p, R = _sr_inputs(orc, N, M, 0.3, 4)
    ns = sig.shape[0]
    plan = _plan(0, N, 1, M, ns, flags)
    sig_d = torch.from_numpy(sig).cuda()
    T = torch.zeros(ns, M, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fit_d, sig_d, tanh_out=T)
    R_d = torch.from_numpy(R).cuda()
    w_d = torch.from_numpy(p).cuda()
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    eps, dg = 1e-3, 0.1
    crbm.sr_step(plan, fit_d, sig_d, T, R_d, dg, eps, solver, crbm.FP32, 1e-10, 2000, stats, weights=w_d)
    F = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
    dx = torch.zeros_like(F)
    Om = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
    crbm.copy_plan_buffer(plan, crbm.BUF_OMEAN, Om)
    torch.cuda.synchronize()
    new_ref, info = orc.sr_step(fit, sig, R.astype(np.complex128), dg, eps, weights=p, want_S=True)
    st = np_of(stats)
    assert abs(st[0] - info["gamma"]) < 1e-6
    assert abs(complex(st[1], st[2]) - info["beta"]) < 1e-6 * abs(info["beta"])
    assert int(st[6]) == 0, st
    O = orc.logderiv(fit, sig)
    assert rel_err(np_of(Om), p @ O) < TOL
    assert rel_err(np_of(F), info["F"]) < 1e-5
    # S is stored in FP32: the solution carries its rounding times the condition number
    assert rel_err(np_of(dx), info["dalpha"]) < 2e-3
    got_new = to_oracle_rbm(orc, fit_d).vector()
    assert rel_err(got_new - fit.vector(), info["dalpha"]) < 2e-3
    if solver == crbm.CG_DENSE:
        S = torch.zeros(plan.P, plan.P, dtype=torch.complex64, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_S, S)
        torch.cuda.synchronize()
        assert rel_err(np_of(S), info["S"]) < 1e-5


def test_sr_step_mc_weights_dense_vs_matfree(orc):
    """Uniform MC weights, square lattice: dense and matrix-free CG agree and match the oracle's F."""
    kind, Lx, Ly, M = 1, 4, 4, 8
    N = 16
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(8, N, M, 0.2)))
    fit = to_oracle_rbm(orc, fit_d)
    sig = synth.random_spins(9, 777, N, True)
    r = np.random.default_rng(1)
    R = (1 + 0.3 * r.normal(size=777) + 0.2j * r.normal(size=777)).astype(np.complex64)
    res = []
    for solver, flags in ((crbm.CG_DENSE, crbm.PLAN_DENSE_S), (crbm.CG_MATFREE, 0)):
        fd = crbm.RBM(fit_d.a.clone(), fit_d.b.clone(), fit_d.W.clone())
        plan = _plan(kind, Lx, Ly, M, 777, flags)
        sd = torch.from_numpy(sig).cuda()
        T = torch.zeros(777, M, dtype=torch.complex64, device="cuda")
        crbm.local_estimators(plan, fd, sd, tanh_out=T)
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        crbm.sr_step(plan, fd, sd, T, torch.from_numpy(R).cuda(), 0.2, 1e-2, solver, crbm.FP32, 1e-10, 1000, stats)
        dx = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
        torch.cuda.synchronize()
        assert int(np_of(stats)[6]) == 0
        res.append(np_of(dx))
    _, info = orc.sr_step(fit, sig, R.astype(np.complex128), 0.2, 1e-2)
    assert rel_err(res[0], info["dalpha"]) < 1e-3
    assert rel_err(res[1], info["dalpha"]) < 1e-3


@pytest.mark.parametrize("kind,Lx,Ly,M,n", [(1, 4, 4, 16, 1500), (0, 40, 1, 80, 8192), (0, 15, 1, 19, 2000)])
def test_cholesky_solve_residual(orc, kind, Lx, Ly, M, n):
    """Blocked FP64 Cholesky solve of (S + eps I) x = F: P = 288 (four 64-column panels and a ragged one,
    also checked against the oracle's update), P = 3320 (the 40-site chain with alpha = 2, 52 panels) and
    P = 319 (odd: rows of S start on 8 bytes, so the dense CG product reads one column per load; two
    tiles, the second ragged).
    The residual against the stored FP32 S is taken in complex128 with torch; a backward-stable solve
    leaves it below a few P * 2^-53 of |S + eps I| |x|."""
    N = Lx * Ly
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(31 + N, N, M, 0.1)))
    sig = synth.random_spins(32 + N, n, N, True)
    r = np.random.default_rng(N)
    R = (1 + 0.3 * r.normal(size=n) + 0.2j * r.normal(size=n)).astype(np.complex64)
    plan = _plan(kind, Lx, Ly, M, n, crbm.PLAN_DENSE_S | crbm.PLAN_CHOLESKY)
    P = plan.P
    sig_d = torch.from_numpy(sig).cuda()
    T = torch.zeros(n, M, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fit_d, sig_d, tanh_out=T)
    fit = to_oracle_rbm(orc, fit_d)
    fit0 = crbm.RBM(fit_d.a.clone(), fit_d.b.clone(), fit_d.W.clone())
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    eps, dg = 1e-2, 0.1
    crbm.sr_step(plan, fit_d, sig_d, T, torch.from_numpy(R).cuda(), dg, eps, crbm.CHOLESKY, crbm.FP32, 1e-10, 1,
                 stats)
    S = torch.zeros(P, P, dtype=torch.complex64, device="cuda")
    F = torch.zeros(P, dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_S, S)
    crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, x)
    torch.cuda.synchronize()
    assert int(np_of(stats)[6]) == 0
    S64 = S.to(torch.complex128)
    herm = (torch.linalg.matrix_norm(S64 - S64.mH) / torch.linalg.matrix_norm(S64)).item()
    # the factorisation reads the lower triangle: the matrix it solves is that triangle's Hermitian completion
    L = torch.tril(S64)
    A = L + torch.tril(S64, -1).mH + eps * torch.eye(P, dtype=torch.complex128, device="cuda")
    xs = x                                      # (S + eps I) dalpha = F, F carrying the step size
    res = torch.linalg.vector_norm(A @ xs - F).item()
    scale = torch.linalg.matrix_norm(A).item() * torch.linalg.vector_norm(xs).item()
    print("P", P, "residual", res, "scale", scale, "ratio", res / scale, "hermitian defect of S", herm)
    assert herm < 1e-6
    assert res < 8 * P * 2.0 ** -53 * scale
    if P < 1000:
        _, info = orc.sr_step(fit, sig, R.astype(np.complex128), dg, eps)
        assert rel_err(np_of(x), info["dalpha"]) < 1e-3
    # dense CG on the same S and F: its product reads the 256 x 256 tiles on and below the diagonal (the
    # diagonal tiles in full) and mirrors the ones below; the solution must solve that operator to the tolerance
    stats2 = torch.zeros(8, dtype=torch.float64, device="cuda")
    crbm.sr_step(plan, fit0, sig_d, T, torch.from_numpy(R).cuda(), dg, eps, crbm.CG_DENSE, crbm.FP32, 1e-11, 3000,
                 stats2)
    xc = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, xc)
    torch.cuda.synchronize()
    st2 = np_of(stats2)
    assert int(st2[6]) == 0, st2
    tile = torch.arange(P, device="cuda") // 256
    upper = tile[:, None] < tile[None, :]
    Ah = torch.where(upper, S64.mH, S64) + eps * torch.eye(P, dtype=torch.complex128, device="cuda")
    res_cg = (torch.linalg.vector_norm(Ah @ xc - F) / torch.linalg.vector_norm(F)).item()
    print("dense CG iterations", st2[5], "residual", res_cg, "reported", st2[4])
    assert res_cg < 1e-10
    assert abs(st2[4] - res_cg) <= 1e-3 * res_cg + 1e-14
    assert rel_err(np_of(xc), np_of(x)) < 1e-3


# ------------------------------------------------------------------ moments and gradient
@pytest.mark.parametrize("kind,Lx,Ly,M,n,std,sim", [CASES[1], CASES[3]])
def test_chebyshev_moments(orc, kind, Lx, Ly, M, n, std, sim):
    N = Lx * Ly
    lat = orc.Lattice(kind, Lx, Ly)
    gs_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(50, N, M, std, std_im=sim)))
    gs = to_oracle_rbm(orc, gs_d)
    n_max = 5
    P = N + M + N * M
    tvec = []
    for t in range(n_max):
        tvec.append(orc.RBM(*synth.random_rbm_arrays(51 + t, N, M, std, std_im=sim)).vector())
    tp = torch.from_numpy(np.stack(tvec).astype(np.complex64)).cuda()
    ts = [orc.RBM.from_vector(np_of(tp[t]).astype(np.complex128), N, M) for t in range(n_max)]
    betas = np.array([1.0, 0.9 - 0.2j, -0.5 + 0.1j, 0.3j, 2.0])
    sig = _samples(orc, N, n, 3)
    ns = sig.shape[0]
    w = orc.enum_weights(orc.logpsi(gs, sig)) if n is None else None
    qs = [(np.pi, 0.0), (2 * np.pi / Lx, 0.0)] if kind == 0 else [(np.pi, np.pi), (np.pi / 2, 0.0), (0.0, np.pi)]
    plan = _plan(kind, Lx, Ly, M, ns)
    mu = torch.zeros(len(qs), n_max + 1, dtype=torch.complex128, device="cuda")
    crbm.chebyshev_moment(plan, gs_d, tp, torch.from_numpy(betas).cuda(), qs, torch.from_numpy(sig).cuda(), mu,
                          weights=None if w is None else torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    ref = orc.moments(gs, ts, betas, qs, lat, sig, weights=w)
    assert rel_err(np_of(mu), ref) < TOL


def test_fidelity_grad(orc):
    kind, Lx, Ly, M = 1, 4, 4, 8
    N = 16
    lat = orc.Lattice(kind, Lx, Ly)
    rb = lambda s: to_device_rbm(orc.RBM(*synth.random_rbm_arrays(s, N, M, 0.2)))
    fit_d, psn_d, psm_d = rb(1), rb(2), rb(3)
    fit, psn, psm = (to_oracle_rbm(orc, r) for r in (fit_d, psn_d, psm_d))
    sig = synth.random_spins(4, 300, N, True)
    plan = _plan(kind, Lx, Ly, M, 300)
    cheb = crbm.make_cheb(3, -10.0, 16.0, 0.9, 1.1)
    sd = torch.from_numpy(sig).cuda()
    R = torch.zeros(300, dtype=torch.complex64, device="cuda")
    T = torch.zeros(300, M, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fit_d, sd, psi_n=psn_d, psi_nm1=psm_d, cheb=cheb, R_out=R, tanh_out=T)
    g = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    crbm.fidelity_grad(plan, fit_d, sd, T, R, g, loss)
    torch.cuda.synchronize()
    R_ref = orc.target_ratio(fit, psn, psm, lat, sig, 3, -10.0, 16.0, 0.9, 1.1)
    L_ref, g_ref = orc.fidelity_grad(fit, sig, R_ref)
    assert abs(np_of(loss)[0] - L_ref) < 1e-5 * max(1.0, L_ref)
    assert rel_err(np_of(g), g_ref) < 1e-5


# ------------------------------------------------------------------ matrix-core S contraction
@pytest.mark.parametrize("kind,Lx,Ly,M,n,bias", [(0, 10, 1, 10, 1000, 0.0), (1, 4, 4, 40, 777, 0.0),
                                                  (0, 40, 1, 80, 130, 0.0), (0, 7, 1, 3, 200, 0.0),
                                                  (0, 12, 1, 24, 600, 0.0), (0, 10, 1, 40, 500, 0.0),
                                                  (0, 18, 1, 56, 300, 0.0), (0, 12, 1, 72, 300, 0.0),
                                                  (1, 4, 4, 40, 777, 1.5), (0, 10, 1, 10, 1000, 3.0)])
def test_dense_s_matrix_cores(orc, kind, Lx, Ly, M, n, bias):
    """S from the FP32 and BF16 matrix-core contractions (uniform weights) against the oracle's S, with
    the last site block of the N + 1 extended sites full (N = 7) or ragged with 1 (N = 16, 40), 2
    (N = 10, 18) or 3 (N = 12) live 2-site fragments.  Those counts of real sites are odd, so site N of
    two hidden blocks shares one mixed fragment wherever a next hidden block exists (M = 24, 40, 56, 72,
    80), the other fragments of every second hidden block pair up across two blocks (M = 56, 72), and a
    last unpaired block keeps its padding half (M = 10, 40, 72, 80).  Every entry is bounded relative
    to the centred diagonal: |dS_kk'| <= tol sqrt(S_kk S_k'k').  The bias
    added to Re b puts |<tanh theta>| at about 5 (bias 1.5) and 200 (bias 3) times the spread of tanh
    theta, where sums of raw products less the product of the means would lose those digits.
    FP32 operands: tol 1e-5.  BF16 operands (8-bit significands, each of the two shifted operands
    rounded once: 2 * 2^-9 per product): tol 2^-7.
    With BF16 operands F is formed from the same rounded operands as S (one ridge problem), so it
    differs from the oracle's F by that rounding too.
    The solve: the relative error of dalpha within the first-order bound
    kappa (|dS|_2 / |S + eps|_2 + |dF| / |F|) (4 times), and the residual of the GPU's dalpha in the
    oracle's system within what the perturbation of S and F allows."""
    N = Lx * Ly
    a0, b0, W0 = synth.random_rbm_arrays(70 + N, N, M, 0.2, std_im=0.05)
    fit_d = to_device_rbm(orc.RBM(a0, b0 + bias, W0))
    fit = to_oracle_rbm(orc, fit_d)
    sig = synth.random_spins(71, n, N, True)
    r = np.random.default_rng(2)
    R = (1 + 0.3 * r.normal(size=n) + 0.2j * r.normal(size=n)).astype(np.complex64)
    eps = 1e-2
    _, info = orc.sr_step(fit, sig, R.astype(np.complex128), 0.1, eps, want_S=True)
    S_ref = info["S"]
    d = np.real(np.diag(S_ref))
    scale = np.sqrt(np.outer(d, d))
    if bias:
        Om = orc.logderiv(fit, sig).mean(axis=0)
        ratio = np.abs(Om[N:N + M]) ** 2 / d[N:N + M]
        print("|<tanh>|^2 / var: median", np.median(ratio), "max", ratio.max())
    A = S_ref + eps * np.eye(S_ref.shape[0])
    errs = {}
    for prec in (crbm.FP32, crbm.BF16):
        fd = crbm.RBM(fit_d.a.clone(), fit_d.b.clone(), fit_d.W.clone())
        plan = _plan(kind, Lx, Ly, M, n, crbm.PLAN_DENSE_S)
        sd = torch.from_numpy(sig).cuda()
        T = torch.zeros(n, M, dtype=torch.complex64, device="cuda")
        crbm.local_estimators(plan, fd, sd, tanh_out=T)
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        crbm.sr_step(plan, fd, sd, T, torch.from_numpy(R).cuda(), 0.1, eps, crbm.CG_DENSE, prec, 1e-10, 3000, stats)
        S = torch.zeros(plan.P, plan.P, dtype=torch.complex64, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_S, S)
        dx = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
        F = torch.zeros_like(dx)
        crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
        torch.cuda.synchronize()
        assert int(np_of(stats)[6]) == 0, np_of(stats)
        Sg = np_of(S)
        assert np.max(np.abs(Sg - Sg.conj().T)) <= 1e-6 * np.abs(Sg).max()
        assert np.all(np.diag(Sg).imag == 0)
        x, Fg = np_of(dx), np_of(F)
        dS = Sg.astype(np.complex128) - S_ref
        spec = np.linalg.norm(dS, 2) / np.linalg.norm(A, 2)
        centred = np.max(np.abs(dS) / scale)
        res = np.linalg.norm(A @ x - info["F"]) / np.linalg.norm(info["F"])
        dF = np.linalg.norm(Fg - info["F"]) / np.linalg.norm(info["F"])
        res_bound = np.linalg.norm(dS, 2) * np.linalg.norm(x) / np.linalg.norm(info["F"]) + dF
        errs[prec] = (centred, rel_err(x, info["dalpha"]), spec, res, res_bound, dF)
    # first-order perturbation bound of the solve: |d x|/|x| <= kappa |d S|_2/|S + eps|_2
    ev = np.linalg.eigvalsh(A)
    kappa = ev.max() / ev.min()
    print("kappa", kappa, "(centred S error, dalpha error, S spectral error, oracle residual, its bound, F error) FP32:",
          errs[crbm.FP32], "BF16:", errs[crbm.BF16])
    assert errs[crbm.FP32][0] < 1e-5
    assert errs[crbm.BF16][0] < 2 ** -7
    for prec in (crbm.FP32, crbm.BF16):
        centred, ex, spec, res, res_bound, dF = errs[prec]
        assert ex < max(1e-4, 4 * kappa * (spec + dF)), prec
        # the CG stops at 1e-10 of |F|; (S_ref + eps) x - F_ref = F_gpu - F_ref - dS x + that residual
        assert res <= 1.01 * res_bound + 1e-9, prec


def test_ceiling_probes():
    """The roofline probes return finite positive rates of plausible size for an MI355X-class device."""
    tf = crbm.probe_mfma()
    gbs = crbm.probe_hbm(1 << 28)
    lc = crbm.probe_logcosh()
    gg = crbm.probe_gather(100, 400)
    print("matrix cores TFLOP/s", tf, "HBM GB/s", gbs, "log-cosh/s", lc, "row gather GB/s", gg)
    assert 100.0 < tf < 5000.0
    assert 500.0 < gbs < 20000.0
    assert 1e11 < lc < 1e14
    assert 100.0 < gg < 100000.0


@pytest.mark.parametrize("kind,Lx,Ly,M,n", [(1, 4, 4, 40, 777), (1, 10, 10, 80, 1100)])
def test_sbuild_k_tiles_bit_identical(orc, kind, Lx, Ly, M, n):
    """The BF16 S contraction with K tiles of 64 and 128 samples gives the same S and the same update
    bit for bit (split over samples for the small model, one pass per tile pair for the larger), and the
    autotuner picks one of them."""
    N = Lx * Ly
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(80 + N, N, M, 0.2, std_im=0.05)))
    sig = synth.random_spins(81, n, N, True)
    r = np.random.default_rng(4)
    R = torch.from_numpy((1 + 0.3 * r.normal(size=n) + 0.2j * r.normal(size=n)).astype(np.complex64)).cuda()
    plan = _plan(kind, Lx, Ly, M, n, crbm.PLAN_DENSE_S)
    sd = torch.from_numpy(sig).cuda()
    T = torch.zeros(n, M, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fit_d, sd, tanh_out=T)
    out = {}
    for kt in (128, 64):
        crbm.set_sbuild_tile(plan, kt)
        fd = crbm.RBM(fit_d.a.clone(), fit_d.b.clone(), fit_d.W.clone())
        stats = torch.zeros(8, dtype=torch.float64, device="cuda")
        crbm.sr_step(plan, fd, sd, T, R, 0.1, 1e-2, crbm.CG_DENSE, crbm.BF16, 1e-8, 2000, stats)
        S = torch.zeros(plan.P, plan.P, dtype=torch.complex64, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_S, S)
        dx = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
        torch.cuda.synchronize()
        out[kt] = (S, dx)
    assert torch.equal(out[128][0], out[64][0])
    assert torch.equal(out[128][1], out[64][1])
    kt, ms = crbm.sbuild_autotune(plan, sd, T)
    print("autotuned K tile", kt, "ms", ms)
    assert kt in (64, 128) and ms > 0
