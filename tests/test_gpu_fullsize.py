"""GPU parity at the full sizes of the benchmark workloads, in the launch configurations the
benchmark uses.  Outputs the oracle can compute one at a time are compared on a sample of them;
the rest through properties that hold at any size.

10x10, alpha = 4 (N = 100, M = 400, P = 40,500; 4096 chains x 128 sweeps = 524,288 samples per
step; one plan with the dense S, every call over all samples):

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

40-site chain, alpha = 2 (P = 3320; 1024 chains x 256 sweeps = 262,144 samples; FP32 S and the
FP64 Cholesky solve): 6 chains replayed bit-exact; gamma, beta, F and S entries as above with the
FP32 accumulation bound; the Cholesky solution's residual against the matrix it factors (the lower
triangle's Hermitian completion plus eps I) within 8 P 2^-53 |A|_F |x|; the update exact.

8x8, alpha = 2, batched moments (2048 (q, n) instances, 256-2048 chains each, 2.37 M chains, 4 + 16
sweeps, one persistent launch after the autotuner): the launch records every accept bit, and the
oracle replays six instances (first, second, middle, last, fewest and most chains) under their global
chain indices: no mismatch, per-instance moments within 1e-5 relative.

16x16, alpha = 2 (P = 131,840; 8192 frozen samples): the fidelity surrogate's loss within 1e-5 and
the hand-written backward on 36 parameter indices within 1e-4 of their largest (complex64 output),
against the oracle's target ratio over all 8192 samples and its per-index gradient.
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


def _centred_scale(e):
    """sqrt(S_kk S_k'k') for every pair of the chosen indices: the scale of the centred S."""
    d = np.real(np.diag(e["S"]))
    return np.sqrt(np.outer(d, d))


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
    # F from the BF16-rounded operands (as S): |dF_k| <= dgamma gamma cot(gamma) 2^-9 <|O'_k| |R - <R>|> / |<R>|
    # <= dgamma gamma 2^-9 sqrt(S_kk) by Cauchy-Schwarz (tan gamma = rms(R - <R>) / |<R>|), O' the shifted
    # operand; asserted with a factor 2
    Fg = np_of(F)
    f_bound = 2.0 ** -8 * 0.1 * e["gamma"] * np.sqrt(np.real(np.diag(e["S"])))
    print("BF16 F: max error / bound", (np.abs(Fg[ks] - e["F"]) / f_bound).max())
    assert np.all(np.abs(Fg[ks] - e["F"]) <= f_bound + 1e-12)
    kt = torch.from_numpy(ks).cuda()
    Sk = np_of(S.index_select(0, kt).index_select(1, kt)).astype(np.complex128)
    bound = 2.0 ** -7 * _centred_scale(e)
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
    """FP32 matrix-core S over all 524,288 samples against the oracle, on the tile-edge indices and on the
    full diagonal.  Each entry sums n products in FP32 accumulators, so the bound is the probabilistic
    one for n rounded additions, 4 sqrt(n) 2^-24 (Higham and Mary, 2019), times the centred scale
    sqrt(S_kk S_k'k')."""
    n = NS
    ks = _param_indices()
    R = (1 + 0.25j * np.random.default_rng(4).normal(size=n)).astype(np.complex64)
    _, stats = _sr_step(big, n, crbm.FP32, R)
    S = torch.zeros(P, P, dtype=torch.complex64, device="cuda")
    crbm.copy_plan_buffer(big["plan"], crbm.BUF_S, S)
    kt = torch.from_numpy(ks).cuda()
    Sk = np_of(S.index_select(0, kt).index_select(1, kt)).astype(np.complex128)
    diag = np_of(torch.diagonal(S)).astype(np.complex128)
    torch.cuda.synchronize()
    del S
    assert int(np_of(stats)[6]) == 0
    tol = 4.0 * np.sqrt(n) * 2.0 ** -24
    e = orc.sr_entries(big["fit"], big["sig"], R.astype(np.complex128), 0.1, ks)
    err = np.abs(Sk - e["S"]) / _centred_scale(e)
    print("FP32 S at n =", n, ": max error / centred scale", err.max(), "bound", tol)
    assert np.all(err <= tol)
    d_ref, _ = orc.sr_diagonal(big["fit"], big["sig"])
    assert np.all(diag.imag == 0)
    derr = np.abs(diag.real - d_ref) / d_ref
    print("FP32 S diagonal: max relative error", derr.max(), "median", np.median(derr))
    assert np.all(derr <= tol)


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


# ------------------------------------------------------------------ 40-site chain, FP32 S + Cholesky
def test_fullsize_chain40_cholesky_step(orc):
    wl = synth.CHAIN40
    n_, m_ = wl.N, wl.M
    p_ = n_ + m_ + n_ * m_
    C, sweeps = wl.chains, wl.sweeps
    ns = C * sweeps
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(wl.param_seed, n_, m_, wl.param_std)))
    fit = to_oracle_rbm(orc, fit_d)
    plan = crbm.Plan(wl.kind, wl.Lx, wl.Ly, m_, ns, crbm.PLAN_CHOLESKY | crbm.PLAN_DENSE_S)
    # sampler at 1024 x 256: six chains replayed under their own indices
    spins = torch.zeros(C, n_, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, spins, wl.chain_seed, True)
    start = orc.init_chains(n_, C, wl.chain_seed, 1)
    words = (sweeps * n_ + 31) // 32
    samples = torch.zeros(sweeps, C, n_, dtype=torch.int8, device="cuda")
    trace = torch.zeros(C, words, dtype=torch.int32, device="cuda")
    crbm.sample(plan, fit_d, spins, sweeps, crbm.EXCHANGE, 21, 16 * n_, samples_out=samples, trace=trace)
    torch.cuda.synchronize()
    ids = np.array([0, 1, 511, 512, C - 2, C - 1], np.int32)
    sub = np.ascontiguousarray(start[ids])
    smp_ref, _, amb, mis = orc.metropolis(fit, sub, sweeps, 1, 21, 16 * n_, trace=np_of(trace).view(np.uint32)[ids],
                                          chain_ids=ids)
    assert mis == 0 and amb <= max(3, 1e-3 * sweeps * n_ * len(ids))
    assert np.array_equal(np_of(samples)[:, ids], smp_ref)
    # the SR step over all 262,144 samples (seeded configurations)
    sig = synth.random_spins(wl.chain_seed, ns, n_, True)
    sd = torch.from_numpy(sig).cuda()
    T = torch.zeros(ns, m_, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fit_d, sd, tanh_out=T)
    r = np.random.default_rng(6)
    R = (1 + 0.3 * r.normal(size=ns) + 0.2j * r.normal(size=ns)).astype(np.complex64)
    before = [t.clone() for t in (fit_d.a, fit_d.b, fit_d.W)]
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    crbm.sr_step(plan, fit_d, sd, T, torch.from_numpy(R).cuda(), 0.1, wl.diag_shift, crbm.CHOLESKY, crbm.FP32, 1e-6,
                 1, stats)
    S = torch.zeros(p_, p_, dtype=torch.complex64, device="cuda")
    F = torch.zeros(p_, dtype=torch.complex128, device="cuda")
    x = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_S, S)
    crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, x)
    torch.cuda.synchronize()
    st = np_of(stats)
    assert int(st[6]) == 0, st
    a_ = [0, 1, 20, n_ - 1]
    b_ = [n_ + j for j in (0, 15, 16, m_ - 1)]
    w_ij = [(0, 0), (0, 15), (0, 16), (7, 15), (8, 16), (7, m_ - 1), (8, 0), (n_ - 1, 0), (n_ - 1, m_ - 1), (31, 47)]
    rr = np.random.default_rng(78)
    w_ij += [(int(i), int(j)) for i, j in zip(rr.integers(0, n_, 18), rr.integers(0, m_, 18))]
    ks = np.array(a_ + b_ + [n_ + m_ + i * m_ + j for i, j in w_ij], np.int64)
    e = orc.sr_entries(fit, sig, R.astype(np.complex128), 0.1, ks)
    assert abs(st[0] - e["gamma"]) < 1e-6 * e["gamma"]
    assert abs(complex(st[1], st[2]) - e["beta"]) < 1e-6 * abs(e["beta"])
    Fg = np_of(F)
    assert np.max(np.abs(Fg[ks] - e["F"])) < TOL * np.abs(Fg).max()
    kt = torch.from_numpy(ks).cuda()
    Sk = np_of(S.index_select(0, kt).index_select(1, kt)).astype(np.complex128)
    err = np.abs(Sk - e["S"])
    bound = 4.0 * np.sqrt(ns) * 2.0 ** -24 * _centred_scale(e)
    print("chain40 FP32 S: max error / bound", (err / bound).max())
    assert np.all(err <= bound)
    S64 = S.to(torch.complex128)
    A = torch.tril(S64) + torch.tril(S64, -1).mH + wl.diag_shift * torch.eye(p_, dtype=torch.complex128,
                                                                             device="cuda")
    res = torch.linalg.vector_norm(A @ x - F).item()
    scale = torch.linalg.matrix_norm(A).item() * torch.linalg.vector_norm(x).item()
    print("chain40 Cholesky residual ratio", res / scale)
    assert res < 8 * p_ * 2.0 ** -53 * scale
    dx = x.to(torch.complex64)
    for got, old, part in zip((fit_d.a, fit_d.b, fit_d.W), before, (dx[:n_], dx[n_:n_ + m_], dx[n_ + m_:].view(n_, m_))):
        assert torch.equal(got, old + part)


# ------------------------------------------------------------------ 8x8 batched moments
def test_fullsize_batched_instances(orc):
    wl = synth.SQUARE8
    n_, m_ = wl.N, wl.M
    counts, offsets, qs = synth.batched_instances()
    n_inst = counts.shape[0]
    total = int(offsets[-1])
    lat = orc.Lattice(wl.kind, wl.Lx, wl.Ly)
    gs_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(wl.param_seed, n_, m_, wl.param_std)))
    gs = to_oracle_rbm(orc, gs_d)
    tv = np.stack([orc.RBM(*synth.random_rbm_arrays(wl.param_seed + 1 + i, n_, m_, wl.param_std)).vector()
                   for i in range(n_inst)]).astype(np.complex64)
    r = np.random.default_rng(8)
    betas = r.normal(size=n_inst) + 1j * r.normal(size=n_inst)
    plan = crbm.Plan(wl.kind, wl.Lx, wl.Ly, m_, total)
    tp, bd = torch.from_numpy(tv).cuda(), torch.from_numpy(betas).cuda()
    qd, od = torch.from_numpy(np.ascontiguousarray(qs)).cuda(), torch.from_numpy(offsets).cuda()
    n_burn, n_sweeps = 4, wl.sweeps
    w, b, lanes, _ = crbm.batched_autotune(plan, gs_d, tp, bd, qd, od, 1, crbm.EXCHANGE, wl.chain_seed)
    print("launch shape", w, "waves x", b, "blocks,", lanes, "lanes per chain; psi_gs rows from LDS:",
          lanes == 64 and crbm.batched_lds_rows(plan, crbm.EXCHANGE, w))
    words = ((n_burn + n_sweeps) * n_ + 31) // 32
    trace = torch.zeros(total, words, dtype=torch.int32, device="cuda")
    mu = torch.zeros(n_inst, 2, dtype=torch.complex128, device="cuda")
    crbm.batched_moments(plan, gs_d, tp, bd, qd, od, n_burn, n_sweeps, crbm.EXCHANGE, wl.chain_seed, mu, trace=trace)
    torch.cuda.synchronize()
    tr = np_of(trace).view(np.uint32)
    mu_g = np_of(mu)
    sel = sorted({0, 1, n_inst // 2, n_inst - 1, int(np.argmin(counts)), int(np.argmax(counts))})
    for i in sel:
        o = offsets[i:i + 2]
        ref, amb, mis = orc.batched_moments(gs, tv[i:i + 1].astype(np.complex128), betas[i:i + 1], qs[i:i + 1], o,
                                            lat, n_burn, n_sweeps, 1, wl.chain_seed, trace=tr[o[0]:o[1]])
        print("instance", i, "chains", counts[i], "ambiguous", amb, "mismatch", mis)
        assert mis == 0
        assert amb <= max(3, 1e-4 * counts[i] * (n_burn + n_sweeps) * n_)
        assert rel_err(mu_g[i], ref[0]) < TOL


# ------------------------------------------------------------------ 16x16 fidelity gradient
def test_fullsize_grad16_fidelity(orc):
    from paper_2103_08804_amd.autograd import fidelity_loss
    wl = synth.SQUARE16
    n_, m_ = wl.N, wl.M
    C = wl.chains
    lat = orc.Lattice(wl.kind, wl.Lx, wl.Ly)
    rb = lambda s: to_device_rbm(orc.RBM(*synth.random_rbm_arrays(s, n_, m_, wl.param_std)))
    psm_d, psn_d, fit_d = rb(wl.param_seed + 1), rb(wl.param_seed + 2), rb(wl.param_seed + 3)
    plan = crbm.Plan(wl.kind, wl.Lx, wl.Ly, m_, C)
    E0 = synth.E0_PER_SITE_SQUARE * n_
    W_scale = 1.5 * abs(E0)
    E_c = E0 + 0.9875 * W_scale
    q = (np.pi, np.pi)
    cheb = crbm.make_cheb(2, E_c, W_scale, 1.0, 1.0, q)
    sig = synth.random_spins(wl.chain_seed, C, n_, True)
    a, b, W = (t.clone().requires_grad_(True) for t in (fit_d.a, fit_d.b, fit_d.W))
    L = fidelity_loss(crbm.RBM(a, b, W), plan, torch.from_numpy(sig).cuda(), psn_d, psm_d, cheb)
    L.backward()
    torch.cuda.synchronize()
    g = np.concatenate([np_of(a.grad), np_of(b.grad), np_of(W.grad).ravel()])
    fit, psn, psm = (to_oracle_rbm(orc, r_) for r_ in (fit_d, psn_d, psm_d))
    R_ref = orc.target_ratio(fit, psn, psm, lat, sig, 2, E_c, W_scale, 1.0, 1.0, q)
    a_ = [0, 1, 128, n_ - 1]
    b_ = [n_ + j for j in (0, 15, 16, m_ - 1)]
    rr = np.random.default_rng(79)
    w_ij = [(0, 0), (n_ - 1, m_ - 1), (7, 15), (8, 16)] + [(int(i), int(j)) for i, j in
                                                          zip(rr.integers(0, n_, 24), rr.integers(0, m_, 24))]
    ks = np.array(a_ + b_ + [n_ + m_ + i * m_ + j for i, j in w_ij], np.int64)
    L_ref, g_ref = orc.fidelity_grad_entries(fit, sig, R_ref, ks)
    print("16x16 loss", float(L.detach()), L_ref, "grad error", np.abs(g[ks] - g_ref).max(), np.abs(g_ref).max())
    assert abs(float(L.detach()) - L_ref) < TOL * max(1.0, L_ref)
    assert np.max(np.abs(g[ks] - g_ref)) < 1e-4 * np.abs(g_ref).max()

