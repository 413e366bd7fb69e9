"""GPU parity at the full size of the 10x10, alpha = 4 workload (N = 100, M = 400, P = 40,500;
4096 chains x 128 sweeps = 524,288 samples per step), in the launch configuration the benchmark
step uses: one plan with the dense S, every call over all 524,288 samples.  Outputs the oracle
can compute one at a time are compared on a sample of them; the rest through properties that
hold at any size.

* Metropolis: 8 of the 4096 chains, spread over the launch (first, last, both halves), replayed
  by the oracle under their own chain indices: trajectories, acceptance counts and end states
  bit-exact (decisions within the 1e-4 margin adopted from the trace).
* Local estimators (Chebyshev order 2, momentum (pi, pi)): log psi, (H t_n)/t_{n+1}, R and
  tanh theta on 130 sampled samples, 1e-5 relative as at the small sizes.
* Natural-gradient step, BF16 S: gamma and beta (1e-6 relative); F on 36 parameter indices of all
  three kinds at tile edges (1e-5 of max |F|); S on all 1296 pairs of those indices against the
  oracle's FP64 sums over the 524,288 samples, within 2^-7 sqrt(<|O_k|^2> <|O_k'|^2>) (each BF16
  operand carries 2^-9 relative rounding, the subtracted means the same, both bounded by
  Cauchy-Schwarz); the CG solution's relative residual against the operator the solver applies
  (the 256 x 256 tiles on and below the diagonal, mirrored above) recomputed in complex128 and
  within the 1e-6 tolerance; the update exactly a + complex64(dalpha).
* FP32 S (the plain path) at full P on the benchmark's 32,768-sample FP32 comparison: the same
  entries within 4 sqrt(n) 2^-24 sqrt(<|O_k|^2> <|O_k'|^2>), the random-walk size of rounding in an
  FP32 accumulator that adds all n products of a sample range (4.3e-5 at n = 32,768).
* Moments n <= 4 at q = (pi, pi) over all 524,288 samples (the benchmark runs 20 orders as 20
  launches of the same kernels): 1e-5 relative to max |mu_n| as at the small sizes.
"""
import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth
from gpu_util import np_of, rel_err, to_device_rbm, to_oracle_rbm, wrapped

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL = 1e-5
WL = synth.SQUARE10
N, M = WL.Lx * WL.Ly, WL.M
P = N + M + N * M
NS = WL.chains * WL.sweeps


@pytest.fixture(scope="module")
def big(orc):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()
    rb = lambda s: to_device_rbm(orc.RBM(*synth.random_rbm_arrays(s, N, M, WL.param_std)))
    fit_d, psn_d, psm_d, gs_d = rb(WL.param_seed), rb(WL.param_seed + 1), rb(WL.param_seed + 2), rb(WL.param_seed + 3)
    plan = crbm.Plan(WL.kind, WL.Lx, WL.Ly, M, NS, crbm.PLAN_DENSE_S)
    sig = synth.random_spins(WL.chain_seed, NS, N, True)
    return dict(plan=plan, fit_d=fit_d, psn_d=psn_d, psm_d=psm_d, gs_d=gs_d,
                fit=to_oracle_rbm(orc, fit_d), psn=to_oracle_rbm(orc, psn_d), psm=to_oracle_rbm(orc, psm_d),
                gs=to_oracle_rbm(orc, gs_d), sig=sig, sig_d=torch.from_numpy(sig).cuda(),
                lat=orc.Lattice(WL.kind, WL.Lx, WL.Ly))


def _param_indices():
    """a, b and W indices at the edges of the 8-site x 16-unit tiles, the extended site N (the b rows),
    the last site and unit, and a seeded scatter."""
    a = [0, 1, 57, N - 1]
    b = [N + j for j in (0, 15, 16, M - 1)]
    w_ij = [(0, 0), (0, 15), (0, 16), (7, 15), (8, 16), (7, M - 1), (8, 0), (63, 200), (95, 384), (96, 385),
            (N - 1, 0), (N - 1, M - 1), (50, 17), (23, 311)]
    r = np.random.default_rng(77)
    w_ij += [(int(i), int(j)) for i, j in zip(r.integers(0, N, 14), r.integers(0, M, 14))]
    return np.array(a + b + [N + M + i * M + j for i, j in w_ij], np.int64)


def test_fullsize_sampler_replay(orc, big):
    plan, fit_d, fit = big["plan"], big["fit_d"], big["fit"]
    C, sweeps = WL.chains, WL.sweeps
    spins = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, spins, WL.chain_seed, True)
    start = orc.init_chains(N, C, WL.chain_seed, 1)
    torch.cuda.synchronize()
    assert np.array_equal(np_of(spins), start)
    words = (sweeps * N + 31) // 32
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    nacc = torch.zeros(C, dtype=torch.int32, device="cuda")
    trace = torch.zeros(C, words, dtype=torch.int32, device="cuda")
    seed, off = 11, 16 * N
    crbm.sample(plan, fit_d, spins, sweeps, crbm.EXCHANGE, seed, off, samples_out=samples, n_accept=nacc,
                trace=trace)
    torch.cuda.synchronize()
    ids = np.array([0, 1, 777, 2047, 2048, 3333, C - 2, C - 1], np.int32)
    sub = np.ascontiguousarray(start[ids])
    smp_ref, nacc_ref, amb, mis = orc.metropolis(fit, sub, sweeps, 1, seed, off,
                                                 trace=np_of(trace).view(np.uint32)[ids], chain_ids=ids)
    print("ambiguous decisions", amb)
    assert mis == 0
    assert amb <= max(3, 1e-3 * sweeps * N * len(ids))
    assert np.array_equal(np_of(samples)[:, ids], smp_ref)
    assert np.array_equal(np_of(spins)[ids], sub)
    assert np.array_equal(np_of(nacc).view(np.uint32)[ids], nacc_ref)


def test_fullsize_local_estimators(orc, big):
    plan, sig = big["plan"], big["sig"]
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    E_c = E0 + (1.0 - 0.0125) * W_scale
    q = (np.pi, np.pi)
    bn, bm = 0.9 - 0.1j, 1.1 + 0.2j
    cheb = crbm.make_cheb(2, E_c, W_scale, bn, bm, q)
    lp = torch.zeros(NS, dtype=torch.complex64, device="cuda")
    hp = torch.zeros_like(lp)
    R = torch.zeros_like(lp)
    T = torch.zeros(NS, M, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, big["fit_d"], big["sig_d"], psi_n=big["psn_d"], psi_nm1=big["psm_d"], cheb=cheb,
                          logpsi_out=lp, eloc_out=hp, R_out=R, tanh_out=T)
    torch.cuda.synchronize()
    idx = np.concatenate([[0, NS - 1], np.random.default_rng(5).choice(NS, 128, replace=False)])
    s = np.ascontiguousarray(sig[idx])
    R_ref, hp_ref = orc.target_ratio(big["fit"], big["psn"], big["psm"], big["lat"], s, 2, E_c, W_scale, bn, bm, q,
                                     return_hpsi=True)
    lp_ref = orc.logpsi(big["fit"], s)
    T_ref = orc.logderiv(big["fit"], s)[:, N:N + M]
    got_lp = np_of(lp)[idx].astype(np.complex128)
    assert np.max(np.abs(got_lp.real - lp_ref.real) / np.maximum(np.abs(lp_ref.real), 1.0)) < TOL
    assert np.max(np.abs(wrapped(got_lp.imag - lp_ref.imag))) < TOL * max(1.0, np.abs(lp_ref).max())
    assert rel_err(np_of(R)[idx], R_ref) < TOL
    assert rel_err(np_of(hp)[idx], hp_ref) < TOL
    assert rel_err(np_of(T)[idx], T_ref) < TOL


def _tile_operator_residual(S, x, F, eps):
    """|F - (S_t + eps I) x| / |F| with S_t the operator of the dense CG product: the 256 x 256 tiles on
    and below the diagonal as stored (the diagonal tiles in full), those above mirrored from below."""
    y = torch.empty_like(x)
    for i0 in range(0, P, 256):
        i1 = min(i0 + 256, P)
        rows = S[i0:i1, :i1].to(torch.complex128) @ x[:i1]
        if i1 < P:
            rows = rows + S[i1:, i0:i1].to(torch.complex128).mH.contiguous() @ x[i1:]
        y[i0:i1] = rows + eps * x[i0:i1]
    return (torch.linalg.vector_norm(y - F) / torch.linalg.vector_norm(F)).item()


def _sr_step(big, n, prec, R):
    plan = big["plan"]
    fd = crbm.RBM(big["fit_d"].a.clone(), big["fit_d"].b.clone(), big["fit_d"].W.clone())
    sd = big["sig_d"][:n]
    T = torch.zeros(n, M, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fd, sd, tanh_out=T)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    crbm.sr_step(plan, fd, sd, T, torch.from_numpy(R).cuda(), 0.1, WL.diag_shift, crbm.CG_DENSE, prec, 1e-6, 500,
                 stats)
    return fd, stats


def _cs_scale(e):
    """sqrt(<|O_k|^2> <|O_k'|^2>) for every pair of the chosen indices (S_kk = <|O_k|^2> - |<O_k>|^2)."""
    m2 = np.real(np.diag(e["S"])) + np.abs(e["Om"]) ** 2
    return np.sqrt(np.outer(m2, m2))


def test_fullsize_sr_step_bf16(orc, big):
    ks = _param_indices()
    r = np.random.default_rng(3)
    R = (1 + 0.3 * r.normal(size=NS) + 0.2j * r.normal(size=NS)).astype(np.complex64)
    before = [t.clone() for t in (big["fit_d"].a, big["fit_d"].b, big["fit_d"].W)]
    fd, stats = _sr_step(big, NS, crbm.BF16, R)
    plan = big["plan"]
    S = torch.zeros(P, P, dtype=torch.complex64, device="cuda")
    F = torch.zeros(P, dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_S, S)
    crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, x)
    torch.cuda.synchronize()
    st = np_of(stats)
    assert int(st[6]) == 0, st
    e = orc.sr_entries(big["fit"], big["sig"], R.astype(np.complex128), 0.1, ks)
    assert abs(st[0] - e["gamma"]) < 1e-6 * e["gamma"]
    assert abs(complex(st[1], st[2]) - e["beta"]) < 1e-6 * abs(e["beta"])
    Fg = np_of(F)
    assert np.max(np.abs(Fg[ks] - e["F"])) < TOL * np.abs(Fg).max()
    kt = torch.from_numpy(ks).cuda()
    Sk = np_of(S.index_select(0, kt).index_select(1, kt)).astype(np.complex128)
    bound = 2.0 ** -7 * _cs_scale(e)
    err = np.abs(Sk - e["S"])
    print("BF16 S: max error / bound", (err / bound).max(), "max error", err.max())
    assert np.all(err <= bound)
    assert np.all(np.diag(Sk).imag == 0)
    # the solve: residual of the operator the CG applies, and the reported one
    res = _tile_operator_residual(S, x, F, WL.diag_shift)
    print("CG iterations", st[5], "residual", res, "reported", st[4])
    assert res <= 1e-6 * (1 + 1e-6)
    assert abs(res - st[4]) <= 1e-3 * st[4] + 1e-12
    # the update adds dalpha rounded to complex64
    dx = x.to(torch.complex64)
    for got, old, part in zip((fd.a, fd.b, fd.W), before, (dx[:N], dx[N:N + M], dx[N + M:].view(N, M))):
        assert torch.equal(got, old + part)


def test_fullsize_s_contraction_fp32(orc, big):
    n = 32768
    ks = _param_indices()
    R = (1 + 0.25j * np.random.default_rng(4).normal(size=n)).astype(np.complex64)
    _, stats = _sr_step(big, n, crbm.FP32, R)
    S = torch.zeros(P, P, dtype=torch.complex64, device="cuda")
    crbm.copy_plan_buffer(big["plan"], crbm.BUF_S, S)
    kt = torch.from_numpy(ks).cuda()
    Sk = np_of(S.index_select(0, kt).index_select(1, kt)).astype(np.complex128)
    torch.cuda.synchronize()
    assert int(np_of(stats)[6]) == 0
    e = orc.sr_entries(big["fit"], np.ascontiguousarray(big["sig"][:n]), R.astype(np.complex128), 0.1, ks)
    err = np.abs(Sk - e["S"])
    bound = 4.0 * np.sqrt(n) * 2.0 ** -24 * _cs_scale(e)
    print("FP32 S: max error / bound", (err / bound).max())
    assert np.all(err <= bound)


def test_fullsize_moments(orc, big):
    n_max = 4
    tv = [orc.RBM(*synth.random_rbm_arrays(WL.param_seed + 10 + t, N, M, WL.param_std)).vector()
          for t in range(n_max)]
    tp = torch.from_numpy(np.stack(tv).astype(np.complex64)).cuda()
    ts = [orc.RBM.from_vector(np_of(tp[t]).astype(np.complex128), N, M) for t in range(n_max)]
    betas = np.array([1.0, 0.8 - 0.4j, -0.6 + 0.2j, 0.5j])
    q = [(np.pi, np.pi)]
    mu = torch.zeros(1, n_max + 1, dtype=torch.complex128, device="cuda")
    crbm.chebyshev_moment(big["plan"], big["gs_d"], tp, torch.from_numpy(betas).cuda(), q, big["sig_d"], mu)
    torch.cuda.synchronize()
    ref = orc.moments(big["gs"], ts, betas, q, big["lat"], big["sig"])
    print("moments", np_of(mu), ref)
    assert rel_err(np_of(mu), ref) < TOL
