"""Benchmark of the Chebyshev-RBM hot path on one MI355X.

Workload: 2D Heisenberg model on a periodic 10 x 10 square lattice (N = 100),
complex RBMs with alpha = 4 (M = 400, P = 40,500 parameters), 4096 Markov
chains x 128 sweeps of N pair-exchange proposals at total S^z = 0.

One step = one pass over every stage of the hot path on one batch:
  1. sample the fitted state t~_{n+1}: 4096 chains x 128 sweeps -> 524,288 samples
  2. local estimators: theta, tanh(theta), local energy of t~_n and the
     Chebyshev target ratio R = (2 beta_n H~ t~_n - beta_{n-1} t~_{n-1}) / t~_{n+1}
  3. natural-gradient step: <R>, gamma, F, dense S = <O^* O> - <O>^*<O> on the
     matrix cores (BF16 operands, FP32 accumulation), CG with double vectors
     (diagonal shift 1e-4, tol 1e-6, at most 500 iterations), parameter update
  4. sample psi_gs: 4096 chains x 128 sweeps
  5. Chebyshev moments mu_n(q), n <= 20, q = (pi, pi), double accumulation
Inputs are synthetic (seeded complex-normal parameters, Fisher-Yates starts).

Prints one JSON line.  value = fitted samples per second of the whole step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sbuild_mfma_bf16_square10x10_alpha4_traffic.json")


# the S contraction's source and every header it includes, in this order
TRAFFIC_SOURCES = ("paper_2103_08804_amd/csrc/kernels_mfma.hip", "paper_2103_08804_amd/csrc/device.hpp",
                   "paper_2103_08804_amd/csrc/internal.hpp", "include/chebrbm.h")


def traffic_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def s_rows_run(N, M):
    """Rows of the b and W blocks (R = M + N M useful ones) that the S contraction runs on the matrix cores,
    padding included: tiles of 8 extended sites x 16 units over the full site blocks; in the last block, when
    it holds r < 7 of the N + 1 extended sites, 2-site fragments of 16 units, with the lone site N of two
    hidden blocks sharing one fragment when r is odd."""
    full, last = divmod(N + 1, 8)
    n_hb = (M + 15) // 16
    rows = 8 * full * 16 * n_hb
    if last == 0:
        return rows
    if last >= 7:
        return rows + 8 * 16 * n_hb
    rf = (last + 1) // 2
    if last % 2:
        pairs, odd = divmod(n_hb, 2)
        return rows + 32 * (pairs * (2 * rf - 1) + odd * rf)
    return rows + 32 * n_hb * rf


def measured_traffic():
    """HBM bytes per launch of the S contraction from the committed counter runs, or None when the
    kernel or a header it includes has changed since the counters were taken."""
    try:
        d = json.load(open(TRAFFIC_FILE))
        now = traffic_source_hash()
    except OSError:
        return None
    if now != d.get("sources_sha256"):
        return None
    return d["traffic_bytes_per_launch"]


BF16_PEAK_TFLOPS = 2500.0
FP32_MATRIX_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["bf16", "fp32"], default="bf16")
    ap.add_argument("--solver", choices=["dense", "matfree"], default="dense")
    ap.add_argument("--chains", type=int, default=synth.SQUARE10.chains)
    ap.add_argument("--sweeps", type=int, default=synth.SQUARE10.sweeps)
    ap.add_argument("--cg-maxit", type=int, default=500)
    ap.add_argument("--n-moments", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--no-plain-path", action="store_true",
                    help="batched8x8: skip the per-instance comparison run")
    ap.add_argument("--fit-steps", type=int, default=60,
                    help="natural-gradient steps per order in the BF16-vs-FP32 fit-quality comparison")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--workload", choices=["square10", "batched8x8", "chain40", "grad16x16", "spectral10x10",
                                           "groundstate10x10", "symmetry6x6"], default="square10",
                    help="square10: the metric's 10x10 alpha=4 step (default); batched8x8: 2048 (q, n) moment "
                         "instances of the 8x8 alpha=2 lattice in one persistent launch; chain40: the 40-site "
                         "chain, alpha=2, FP32 dense SR with the FP64 Cholesky solve; grad16x16: forward and "
                         "hand-written backward of the fidelity surrogate on the 16x16 alpha=2 lattice")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import paper_2103_08804_amd as crbm

    torch.cuda.set_device(0)
    if args.workload == "batched8x8":
        return bench_batched(crbm, args)
    if args.workload == "chain40":
        return bench_chain40(crbm, args)
    if args.workload == "grad16x16":
        return bench_grad16(crbm, args)
    if args.workload == "spectral10x10":
        return bench_spectral(crbm, args)
    if args.workload == "groundstate10x10":
        return bench_groundstate(crbm, args)
    if args.workload == "symmetry6x6":
        return bench_symmetry(crbm, args)
    wl = synth.SQUARE10
    N, M, P = wl.N, wl.M, wl.P
    C, sweeps = args.chains, args.sweeps
    ns = C * sweeps
    prec = crbm.BF16 if args.precision == "bf16" else crbm.FP32
    solver = crbm.CG_DENSE if args.solver == "dense" else crbm.CG_MATFREE
    flags = crbm.PLAN_DENSE_S if solver == crbm.CG_DENSE else 0
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, ns, flags)

    # synthetic RBMs: psi_gs, t~_{n-1}, t~_n and the fitted t~_{n+1}; n_moments stored RBMs for mu_n
    def new_rbm(seed):
        r = crbm.RBM.empty(N, M)
        crbm.init_rbm(r, seed, wl.param_std)
        return r

    gs, psm, psn, fit = new_rbm(wl.param_seed), new_rbm(wl.param_seed + 1), new_rbm(wl.param_seed + 2), \
        new_rbm(wl.param_seed + 3)
    n_max = args.n_moments
    tp = torch.zeros(n_max, P, dtype=torch.complex64, device="cuda")
    for t in range(n_max):
        crbm.init_rbm(crbm.RBM.from_packed(tp[t], N, M), wl.param_seed + 10 + t, wl.param_std)
    betas = torch.ones(n_max, dtype=torch.complex128, device="cuda")
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    E_c = E0 + (1.0 - 0.0125) * W_scale
    cheb = crbm.make_cheb(2, E_c, W_scale, 1.0, 1.0, (math.pi, math.pi))

    chains_fit = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    chains_gs = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains_fit, wl.chain_seed, True)
    crbm.init_chains(plan, chains_gs, wl.chain_seed + 1, True)
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    samples_gs = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    flat, flat_gs = samples.view(ns, N), samples_gs.view(ns, N)
    T = torch.zeros(ns, M, dtype=torch.complex64, device="cuda")
    R = torch.zeros(ns, dtype=torch.complex64, device="cuda")
    El = torch.zeros(ns, dtype=torch.complex64, device="cuda")
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    mu = torch.zeros(1, n_max + 1, dtype=torch.complex128, device="cuda")
    # burn-in (untimed)
    crbm.sample(plan, fit, chains_fit, 16, crbm.EXCHANGE, 11, 0)
    crbm.sample(plan, gs, chains_gs, 16, crbm.EXCHANGE, 12, 0)
    offset = [16 * N]

    def step(s_prec=prec):
        crbm.sample(plan, fit, chains_fit, sweeps, crbm.EXCHANGE, 11, offset[0], samples_out=samples)
        crbm.local_estimators(plan, fit, flat, psi_n=psn, psi_nm1=psm, cheb=cheb, eloc_out=El, R_out=R, tanh_out=T)
        crbm.sr_step(plan, fit, flat, T, R, 0.1, wl.diag_shift, solver, s_prec, 1e-6, args.cg_maxit, stats)
        crbm.sample(plan, gs, chains_gs, sweeps, crbm.EXCHANGE, 12, offset[0], samples_out=samples_gs)
        crbm.chebyshev_moment(plan, gs, tp, betas, [(math.pi, math.pi)], flat_gs, mu)
        offset[0] += sweeps * N

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sb_tile = None
    if solver == crbm.CG_DENSE and prec == crbm.BF16 and args.warmup > 0:
        # K tile of the S contraction, timed on the warm-up step's samples (both tiles give the same S)
        kt, kt_ms = crbm.sbuild_autotune(plan, flat, T)
        sb_tile = {"k_tile": kt, "probe_ms": kt_ms, "candidates": [64, 128]}
    plan.profile(True)
    per_step = torch.zeros(args.steps, 8, dtype=torch.float64, device="cuda")   # each step's SR stats
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        per_step[k].copy_(stats, non_blocking=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    st = stats.cpu().numpy()
    ms_per_step = 1e3 * elapsed / args.steps
    value = ns / (elapsed / args.steps)

    phases = {k: {"launches": c, "avg_ms": t / c} for k, (c, t) in prof.items()}
    # dominant kernel: the dense S contraction (matrix cores) when it runs, else the O^H c contraction
    if "sbuild" in prof and solver == crbm.CG_DENSE:
        c, t = prof["sbuild"]
        avg_s = t / c / 1e3
        # the contraction builds the rows and columns of b and W (R = M + N M of the P parameters):
        # R(R+1)/2 complex entries x N_s samples x 8 real flops; the N rows of a are the border kernel's.
        # One launch takes the tile pairs of the full 8-site blocks and the ragged pairs of the last.
        R_rows = P - N
        flops = 4.0 * R_rows * (R_rows + 1) * ns
        peak = BF16_PEAK_TFLOPS if prec == crbm.BF16 else FP32_MATRIX_PEAK_TFLOPS
        achieved = flops / avg_s / 1e12
        traffic = measured_traffic() if (prec == crbm.BF16 and C == wl.chains and sweeps == wl.sweeps) else None
        esz = 2 if prec == crbm.BF16 else 4
        roof = {"kernel": "k_sbuild_mfma (all tile pairs of the b and W rows, one launch)", "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "algorithmic_flops": flops,
                # each operand read once (T re and im of M units, the sign rows of the N + 1 extended sites)
                # and both triangles of the block written
                "algorithmic_bytes": (2 * M + N + 1) * ns * esz + 8 * R_rows * R_rows,
                "rows_run_per_useful_row": s_rows_run(N, M) / R_rows,
                "note": ("the b and W rows (R = P - N = %d) in one launch: the tile pairs of the full 8-site blocks "
                         "and the ragged pairs of the last block; the N rows of a in k_sbuild_border (phase "
                         "'sborder')" % R_rows)}
    else:
        c, t = prof["ot"]
        avg_s = t / c / 1e3
        byts = ns * (M * 8 + N + 16)
        achieved = byts / avg_s / 1e9
        roof = {"kernel": "k_ot", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": byts}

    # sustained ceilings of this device, measured after the timed region
    if roof["bound"] == "mfma" and prec == crbm.BF16:
        ceil = crbm.probe_mfma()
        roof["measured_ceiling"] = {"value": ceil, "unit": "TFLOP/s",
                                    "probe": "v_mfma_f32_32x32x16_bf16, 8 independent accumulators per wave, "
                                             "2 workgroups x 4 waves per CU, no memory traffic"}
        roof["frac_of_measured"] = roof["achieved"] / ceil
    elif roof["bound"] == "hbm":
        ceil = crbm.probe_hbm(1 << 30)
        roof["measured_ceiling"] = {"value": ceil, "unit": "GB/s", "probe": "16-byte copy of 1 GiB, read + write"}
        roof["frac_of_measured"] = roof["achieved"] / ceil
    # the Metropolis sweep against its own ceilings (it has no datasheet roofline): half of the pair
    # exchanges are null moves at S^z = 0 in expectation; every other proposal evaluates M Re log 2cosh
    # and reads the rows W_i and W_j (2 M complex64) from L2
    sampler = None
    if "sample" in prof:
        c, t = prof["sample"]
        rate = C * sweeps * N / (t / c / 1e3)
        lc = 0.5 * rate * M
        gb = 0.5 * rate * 2 * M * 8 / 1e9
        lc_ceil = crbm.probe_logcosh()
        g_ceil = crbm.probe_gather(N, M)
        sampler = {"proposals_per_s": rate, "logcosh_per_s": lc, "logcosh_ceiling": lc_ceil,
                   "logcosh_frac": lc / lc_ceil, "row_gather_GBps": gb, "row_gather_ceiling_GBps": g_ceil,
                   "row_gather_frac": gb / g_ceil,
                   "probes": "Re log 2cosh in the sweep's form, 8 independent per lane, no memory traffic; whole-row "
                             "reads of the N x M complex64 W at random rows"}
    line = {
        "metric": "MC samples/s + SR steps/s, 10x10 RBM alpha=4, BF16/batched vs plain FP32 at equal mu_n error",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if prec == crbm.BF16 else "f32", "data": "synthetic",
        "config": {"workload": "heisenberg_square10x10_rbm_alpha4", "lattice": "10x10 periodic", "N": N, "M": M,
                   "P": P, "chains": C, "sweeps": sweeps, "samples_per_step": ns, "proposal": "pair_exchange",
                   "solver": args.solver, "s_precision": args.precision, "diag_shift": wl.diag_shift,
                   "cg_tol": 1e-6, "cg_maxit": args.cg_maxit, "n_moments": n_max, "parallelism": "single_gpu"},
        "sr_steps_per_s": 1e3 / ms_per_step,
        "sampler_samples_per_s": (C * sweeps) / (prof["sample"][1] / prof["sample"][0] / 1e3) if "sample" in prof else None,
        "cg_iterations": float(st[5]), "cg_rel_residual": float(st[4]), "sr_flags": int(st[6]),
        "gamma": float(st[0]),
        "sbuild_autotune": sb_tile,
        "per_step": {"gamma": [float(x) for x in per_step[:, 0].cpu()],
                     "cg_iterations": [float(x) for x in per_step[:, 5].cpu()]},
        "phases": phases,
        "roofline": roof,
        "sampler_roofline": sampler,
    }
    if solver == crbm.CG_DENSE:
        line["cg_launch_overhead"] = cg_overhead(crbm, plan, fit, flat, T, R, wl, args, s_prec=prec)
    if not args.no_fp32_compare and solver == crbm.CG_DENSE and prec == crbm.BF16:
        line["matfree_compare"] = matfree_compare(crbm, plan, fit, flat, T, R, wl, args, ms_per_step, prof)
        line["fp32_compare"] = fp32_compare(crbm, plan, fit, step, flat, T, R, wl, args, ms_per_step, stats)
        line["fit_quality_bf16_vs_fp32"] = fit_quality_compare(crbm, args.fit_steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["moments_vs_oracle"] = cpu_baseline(args.cpu_budget_s, ns, sweeps, C)
    print(json.dumps(line))
    plan.close()


def bench_batched(crbm, args):
    """Moments of 32 momenta x 64 Chebyshev orders (2048 instances) of the 8x8, alpha = 2 lattice,
    256..2048 chains per instance, 4 burn-in + 16 recorded sweeps, one persistent launch."""
    wl = synth.SQUARE8
    N, M, P = wl.N, wl.M, wl.P
    n_q, n_ord = 32, 64
    n_inst = n_q * n_ord
    counts, offsets, qs = synth.batched_instances(n_q, n_ord)
    total = int(offsets[-1])
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, total)
    gs = crbm.RBM.empty(N, M)
    crbm.init_rbm(gs, wl.param_seed, wl.param_std)
    tp = torch.zeros(n_inst, P, dtype=torch.complex64, device="cuda")
    for i in range(n_inst):
        crbm.init_rbm(crbm.RBM.from_packed(tp[i], N, M), wl.param_seed + 1 + i, wl.param_std)
    betas = torch.ones(n_inst, dtype=torch.complex128, device="cuda")
    qd = torch.from_numpy(np.ascontiguousarray(qs)).cuda()
    od = torch.from_numpy(offsets).cuda()
    mu = torch.zeros(n_inst, 2, dtype=torch.complex128, device="cuda")
    n_burn, n_sweeps = 4, wl.sweeps
    w, b, lanes, tune_ms = crbm.batched_autotune(plan, gs, tp, betas, qd, od, 4, crbm.EXCHANGE, wl.chain_seed)
    for _ in range(args.warmup):
        crbm.batched_moments(plan, gs, tp, betas, qd, od, n_burn, n_sweeps, crbm.EXCHANGE, wl.chain_seed, mu)
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        crbm.batched_moments(plan, gs, tp, betas, qd, od, n_burn, n_sweeps, crbm.EXCHANGE, wl.chain_seed, mu)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    prof = plan.profile_read()
    plan.profile(False)
    samples = total * n_sweeps
    line = {"metric": "batched moment samples/s (instance-weighted)", "value": samples / el, "unit": "samples/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "heisenberg_square8x8_rbm_alpha2_batched_moments", "instances": n_inst,
                       "momenta": n_q, "orders": n_ord, "total_chains": total, "burn_in_sweeps": n_burn,
                       "recorded_sweeps": n_sweeps, "chains_per_instance": [int(counts.min()), int(counts.max())]},
            "autotuned": {"waves_per_block": w, "blocks": b, "lanes_per_chain": lanes, "probe_ms": tune_ms,
                          "psi_gs_rows_in_lds": lanes == 64 and crbm.batched_lds_rows(plan, crbm.EXCHANGE, w)},
            "kernel_ms": prof["batched"][1] / prof["batched"][0],
            "chain_steps_per_s": total * (n_burn + n_sweeps) * N / el}
    # tail of the persistent launch: per-wave (start, end) clocks of the last timed launch
    clk = torch.zeros(crbm.MAX_CLOCK_WAVES, 2, dtype=torch.int64, device="cuda")
    crbm.copy_plan_buffer(plan, crbm.BUF_WAVE_CLOCKS, clk)
    c = clk.cpu().numpy().astype(np.float64)
    c = c[c[:, 1] > 0]
    t_end, t_beg = c[:, 1].max(), c[:, 0].min()
    line["tail"] = {"waves": int(c.shape[0]), "launch_us": (t_end - t_beg) / 100.0,
                    "tail_idle_frac": float(np.sum(t_end - c[:, 1]) / np.sum(t_end - c[:, 0])),
                    "start_spread_us": float(c[:, 0].max() - t_beg) / 100.0,
                    "first_idle_before_end_us": float(t_end - c[:, 1].min()) / 100.0,
                    "note": ("per-wave clocks (100 MHz): tail_idle_frac = sum over waves of (launch end - wave end) / "
                             "sum of (launch end - wave start), the share of resident wave time spent idle once the "
                             "chain counter ran out")}
    # against its ceilings: half of the pair exchanges are live at S^z = 0 (independent uniform sites); a
    # live one evaluates M Re log 2cosh of psi_gs and reads rows W_i, W_j of psi_gs (2 M complex64, from
    # LDS when the kernel keeps a copy there); an accepted one also reads rows W_i, W_j of t~ (from L2);
    # the recorded sweeps add 2 M log cosh per chain (t~ and psi_gs).  The accepted moves are counted
    # from the accept trace of one more launch after the timed region.
    kern_s = line["kernel_ms"] / 1e3
    props = total * (n_burn + n_sweeps) * N
    words = ((n_burn + n_sweeps) * N + 31) // 32
    tr = torch.zeros(total, words, dtype=torch.int32, device="cuda")
    crbm.batched_moments(plan, gs, tp, betas, qd, od, n_burn, n_sweeps, crbm.EXCHANGE, wl.chain_seed, mu, trace=tr)
    accepted = sum(int(((tr >> b) & 1).sum().item()) for b in range(32))
    del tr
    in_lds = line["autotuned"]["psi_gs_rows_in_lds"]
    lc = (0.5 * props * M + 2.0 * total * n_sweeps * M) / kern_s
    gs_rows = 0.5 * props * 2 * M * 8 / kern_s / 1e9
    t_rows = accepted * 2 * M * 8 / kern_s / 1e9
    l2 = t_rows + (0.0 if in_lds else gs_rows)
    lc_ceil, g_ceil = crbm.probe_logcosh(), crbm.probe_gather(N, M)
    line["roofline"] = {"kernel": "k_batched", "bound": "alu", "achieved": lc / 1e12, "peak": lc_ceil / 1e12,
                        "unit": "Tlogcosh/s", "frac": lc / lc_ceil, "traffic": None,
                        "accepted_frac": accepted / props,
                        "l2_row_gather_GBps": l2, "row_gather_ceiling_GBps": g_ceil, "l2_row_gather_frac": l2 / g_ceil,
                        "lds_row_GBps": gs_rows if in_lds else 0.0,
                        "bound_note": ("VALU issue: per proposal about 39 VALU instructions (SQ counters), of which the "
                                       "log-cosh of a live move is about 9; the rest is the per-move control of one "
                                       "chain per wave"),
                        "peak_note": ("measured ceilings of this device: k_probe_logcosh (Re log 2cosh in the sweep's "
                                      "form, 8 independent per lane) and k_probe_gather (whole W rows at random "
                                      "rows from L2); the L2 row gathers are the rows of t~ on accepted moves and, "
                                      "unless psi_gs's W sits in LDS, the rows of psi_gs on live moves")}
    if not args.no_plain_path:
        line["plain_path"] = plain_path_batched(crbm, plan, gs, tp, betas, qs, counts, offsets, n_burn, n_sweeps, wl,
                                                line["kernel_ms"])
    print(json.dumps(line))
    plan.close()


def plain_path_batched(crbm, plan, gs, tp, betas, qs, counts, offsets, n_burn, n_sweeps, wl, batched_ms):
    """The same instances through the per-instance calls: for instance i, its c_i chains start at S^z = 0
    (crbm_init_chains), take n_burn + n_sweeps pair-exchange sweeps of psi_gs (crbm_sample, the recorded
    sweeps kept), and mu_i = crbm_chebyshev_moment of t~_i at q_i over those samples.  Timed end to end
    (one pass, host loop over the 2048 instances, one stream)."""
    N = wl.N
    cmax = int(counts.max())
    spins = torch.zeros(cmax, N, dtype=torch.int8, device="cuda")
    smp = torch.zeros(n_sweeps * cmax * N, dtype=torch.int8, device="cuda")
    mu = torch.zeros(1, 2, dtype=torch.complex128, device="cuda")
    n_inst = len(counts)

    def one_pass():
        for i in range(n_inst):
            c = int(counts[i])
            sp = spins[:c]
            crbm.init_chains(plan, sp, wl.chain_seed + i, True)
            crbm.sample(plan, gs, sp, n_burn, crbm.EXCHANGE, wl.chain_seed, 0)
            out = smp[:n_sweeps * c * N].view(n_sweeps, c, N)
            crbm.sample(plan, gs, sp, n_sweeps, crbm.EXCHANGE, wl.chain_seed, n_burn * N, samples_out=out)
            crbm.chebyshev_moment(plan, gs, tp[i:i + 1], betas[i:i + 1], [tuple(qs[i])], out.view(-1, N), mu)

    one_pass()          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one_pass()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    return {"ms": ms, "batched_speedup": ms / batched_ms, "launches": 4 * n_inst,
            "note": "per instance: init_chains, burn-in sweeps, recorded sweeps, one moment; same chain counts"}


def _timed(plan, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    prof = plan.profile_read()
    plan.profile(False)
    return el, {k: {"launches": c, "avg_ms": t / c} for k, (c, t) in prof.items()}


def bench_chain40(crbm, args):
    """40-site chain, alpha = 2 (P = 3320): 1024 chains x 256 sweeps, local estimators, FP32 dense S on the
    matrix cores and the FP64 Cholesky solve with diagonal shift 1e-3."""
    wl = synth.CHAIN40
    N, M, P = wl.N, wl.M, wl.P
    C, sweeps = wl.chains, wl.sweeps
    ns = C * sweeps
    plan = crbm.Plan(crbm.CHAIN, N, 1, M, ns, crbm.PLAN_CHOLESKY)
    mk = lambda sd: (lambda r: (crbm.init_rbm(r, sd, wl.param_std), r)[1])(crbm.RBM.empty(N, M))
    gs, psm, psn, fit = mk(wl.param_seed), mk(wl.param_seed + 1), mk(wl.param_seed + 2), mk(wl.param_seed + 3)
    E0 = synth.E0_PER_SITE_CHAIN * N
    W_scale = 1.5 * abs(E0)
    cheb = crbm.make_cheb(2, E0 + 0.9875 * W_scale, W_scale, 1.0, 1.0, (math.pi, 0.0))
    chains = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains, wl.chain_seed, True)
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    flat = samples.view(ns, N)
    T = torch.zeros(ns, M, dtype=torch.complex64, device="cuda")
    R = torch.zeros(ns, dtype=torch.complex64, device="cuda")
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    crbm.sample(plan, fit, chains, 16, crbm.EXCHANGE, 21, 0)
    off = [16 * N]

    def step():
        crbm.sample(plan, fit, chains, sweeps, crbm.EXCHANGE, 21, off[0], samples_out=samples)
        crbm.local_estimators(plan, fit, flat, psi_n=psn, psi_nm1=psm, cheb=cheb, R_out=R, tanh_out=T)
        crbm.sr_step(plan, fit, flat, T, R, 0.1, wl.diag_shift, crbm.CHOLESKY, crbm.FP32, 1e-6, 1, stats)
        off[0] += sweeps * N

    el, phases = _timed(plan, step, args.steps, args.warmup)
    st = stats.cpu().numpy()
    # the FP32 S contraction of the b and W rows (R = P - N): 4 R (R + 1) N_s FLOP on the FP32 matrix cores;
    # its row tiles are 8 sites x 16 units; the last site block (site 40 alone) runs as one fragment per
    # two hidden blocks (ragged pairs)
    t_sb = phases["sbuild"]["avg_ms"] / 1e3
    R_rows = P - N
    flops = 4.0 * R_rows * (R_rows + 1) * ns
    rows_run = s_rows_run(N, M)
    roof = {"kernel": "k_sbuild_mfma<false> (FP32 operands, one launch)", "bound": "mfma",
            "achieved": flops / t_sb / 1e12,
            "peak": FP32_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": flops / t_sb / 1e12 / FP32_MATRIX_PEAK_TFLOPS,
            "traffic": None, "algorithmic_flops": flops, "rows_run_per_useful_row": rows_run / R_rows}
    print(json.dumps({"metric": "MC samples/s + SR steps/s", "value": ns / el, "unit": "samples/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "heisenberg_chain40_rbm_alpha2", "N": N, "M": M, "P": P, "chains": C,
                                 "sweeps": sweeps, "samples_per_step": ns, "solver": "cholesky_fp64",
                                 "s_precision": "fp32", "diag_shift": wl.diag_shift},
                      "sr_steps_per_s": 1.0 / el, "sr_flags": int(st[6]), "rel_residual": float(st[4]),
                      "phases": phases, "roofline": roof}))
    plan.close()


def bench_spectral(crbm, args):
    """Moment correction and both spectra on the 10x10 alpha = 4 lattice: 4096 chains x 128 sweeps of psi_gs,
    G and H (K = n_moments + 1) over the 524,288 samples, corrected moments (10 K of them), Lanczos,
    Jackson-damped and continued-fraction spectra on 1001 frequencies."""
    wl = synth.SQUARE10
    N, M, P = wl.N, wl.M, wl.P
    C, sweeps = args.chains, args.sweeps
    ns = C * sweeps
    n_max = args.n_moments
    K = n_max + 1
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, ns, crbm.PLAN_BASIS, basis_k_max=K)
    gs = crbm.RBM.empty(N, M)
    crbm.init_rbm(gs, wl.param_seed, wl.param_std)
    tp = torch.zeros(n_max, P, dtype=torch.complex64, device="cuda")
    for t in range(n_max):
        crbm.init_rbm(crbm.RBM.from_packed(tp[t], N, M), wl.param_seed + 10 + t, wl.param_std)
    betas = torch.ones(n_max, dtype=torch.complex128, device="cuda")
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    E_c = E0 + (1.0 - 0.0125) * W_scale
    q = (math.pi, math.pi)
    chains = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains, wl.chain_seed + 1, True)
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    flat = samples.view(ns, N)
    G = torch.zeros(K, K, dtype=torch.complex128, device="cuda")
    H = torch.zeros_like(G)
    n_out = 10 * K
    mu = torch.zeros(n_out, dtype=torch.float64, device="cuda")
    info = torch.zeros(3, dtype=torch.float64, device="cuda")
    a = torch.zeros(K, dtype=torch.float64, device="cuda")
    b2 = torch.zeros(K, dtype=torch.float64, device="cuda")
    linfo = torch.zeros(2, dtype=torch.float64, device="cuda")
    omega = torch.linspace(0.0, 2.0 * W_scale, 1001, dtype=torch.float64, device="cuda")
    A_kpm = torch.zeros_like(omega)
    A_cf = torch.zeros_like(omega)
    crbm.sample(plan, gs, chains, 16, crbm.EXCHANGE, 12, 0)
    off = [16 * N]

    def step():
        crbm.sample(plan, gs, chains, sweeps, crbm.EXCHANGE, 12, off[0], samples_out=samples)
        crbm.moment_matrices(plan, gs, tp, betas, q, flat, G, H)
        crbm.corrected_moments(plan, G, H, E_c, W_scale, mu, info)
        crbm.lanczos(plan, G, H, a, b2, linfo)
        crbm.spectrum_kpm(mu, E0, E_c, W_scale, omega, A_kpm)
        crbm.spectrum_cf(a, b2, K, E0, 0.1, omega, A_cf)
        off[0] += sweeps * N

    el, phases = _timed(plan, step, args.steps, args.warmup)
    inf, linf = info.cpu().numpy(), linfo.cpu().numpy()
    print(json.dumps({"metric": "samples/s of the moment-correction pass (G and H over n_max RBMs) with both spectra",
                      "value": ns / el, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "heisenberg_square10x10_rbm_alpha4_moment_correction", "N": N, "M": M,
                                 "P": P, "chains": C, "sweeps": sweeps, "samples_per_step": ns, "K": K,
                                 "corrected_moments": n_out, "omega_points": 1001},
                      "correction_flags": int(inf[0]), "moment_growth": float(inf[1]),
                      "lanczos_steps": int(linf[1]), "phases": phases}))
    plan.close()


def bench_symmetry(crbm, args):
    """Symmetry-projected moment correction on the 6x6 lattice of the paper's 2D results (alpha = 2):
    1024 chains x 64 sweeps of psi_gs, every sample evaluated on its 36 translations x 4 rotations for
    psi_gs and the 20 stored local-operator RBMs, G^(k) and H^(k) for all 36 momenta, then per momentum
    the corrected moments (10 K), Lanczos and both spectra on 1001 frequencies."""
    wl = synth.SQUARE6
    N, M, P = wl.N, wl.M, wl.P
    C, sweeps = wl.chains, wl.sweeps
    ns = C * sweeps
    n_max = args.n_moments
    K = n_max + 1
    ng = 4 * N
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, ns * ng, crbm.PLAN_SYM_BASIS, basis_k_max=K)
    gs = crbm.RBM.empty(N, M)
    crbm.init_rbm(gs, wl.param_seed, wl.param_std)
    tp = torch.zeros(n_max, P, dtype=torch.complex64, device="cuda")
    for t in range(n_max):
        crbm.init_rbm(crbm.RBM.from_packed(tp[t], N, M), wl.param_seed + 10 + t, wl.param_std)
    betas = torch.ones(n_max, dtype=torch.complex128, device="cuda")
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    E_c = E0 + (1.0 - 0.0125) * W_scale
    chains = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains, wl.chain_seed, True)
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    flat = samples.view(ns, N)
    G = torch.zeros(N, K, K, dtype=torch.complex128, device="cuda")
    H = torch.zeros_like(G)
    n_out = 10 * K
    mu = torch.zeros(N, n_out, dtype=torch.float64, device="cuda")
    info = torch.zeros(N, 3, dtype=torch.float64, device="cuda")
    a = torch.zeros(N, K, dtype=torch.float64, device="cuda")
    b2 = torch.zeros(N, K, dtype=torch.float64, device="cuda")
    linfo = torch.zeros(N, 2, dtype=torch.float64, device="cuda")
    omega = torch.linspace(0.0, 2.0 * W_scale, 1001, dtype=torch.float64, device="cuda")
    A_kpm = torch.zeros(N, 1001, dtype=torch.float64, device="cuda")
    A_cf = torch.zeros(N, 1001, dtype=torch.float64, device="cuda")
    crbm.sample(plan, gs, chains, 16, crbm.EXCHANGE, 51, 0)
    off = [16 * N]

    def step():
        crbm.sample(plan, gs, chains, sweeps, crbm.EXCHANGE, 51, off[0], samples_out=samples)
        crbm.sym_matrices(plan, gs, tp, betas, flat, G, H, rotations=True)
        for k in range(N):
            crbm.corrected_moments(plan, G[k], H[k], E_c, W_scale, mu[k], info[k])
            crbm.lanczos(plan, G[k], H[k], a[k], b2[k], linfo[k])
            crbm.spectrum_kpm(mu[k], E0, E_c, W_scale, omega, A_kpm[k])
            crbm.spectrum_cf(a[k], b2[k], K, E0, 0.1, omega, A_cf[k])
        off[0] += sweeps * N

    el, phases = _timed(plan, step, args.steps, args.warmup)
    inf, linf = info.cpu().numpy(), linfo.cpu().numpy()
    print(json.dumps({"metric": "samples/s of the symmetry-projected moment correction (all momenta) with both "
                                "spectra", "value": ns / el, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "heisenberg_square6x6_rbm_alpha2_symmetry_projection", "N": N, "M": M,
                                 "P": P, "chains": C, "sweeps": sweeps, "samples_per_step": ns, "K": K,
                                 "group_elements": ng, "image_rows": ns * ng, "momenta": N,
                                 "corrected_moments_per_momentum": n_out, "omega_points": 1001},
                      "image_rows_per_s": ns * ng / el,
                      "correction_flags": int(np.max(inf[:, 0])), "max_moment_growth": float(np.max(inf[:, 1])),
                      "lanczos_steps": [int(v) for v in linf[:, 1][:4]], "phases": phases}))
    plan.close()


def bench_groundstate(crbm, args):
    """Ground-state natural-gradient step on the 10x10 alpha = 4 lattice: 4096 chains x 128 sweeps, local
    energies, BF16 dense S on the matrix cores and CG (diagonal shift 1e-4, tol 1e-6)."""
    wl = synth.SQUARE10
    N, M, P = wl.N, wl.M, wl.P
    C, sweeps = args.chains, args.sweeps
    ns = C * sweeps
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, ns, crbm.PLAN_DENSE_S)
    psi = crbm.RBM.empty(N, M)
    crbm.init_rbm(psi, wl.param_seed, wl.param_std)
    chains = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains, wl.chain_seed, True)
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    flat = samples.view(ns, N)
    T = torch.zeros(ns, M, dtype=torch.complex64, device="cuda")
    El = torch.zeros(ns, dtype=torch.complex64, device="cuda")
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    crbm.sample(plan, psi, chains, 16, crbm.EXCHANGE, 41, 0)
    off = [16 * N]

    def step():
        crbm.sample(plan, psi, chains, sweeps, crbm.EXCHANGE, 41, off[0], samples_out=samples)
        crbm.local_estimators(plan, psi, flat, eloc_out=El, tanh_out=T)
        crbm.sr_energy_step(plan, psi, flat, T, El, 0.05, wl.diag_shift, crbm.CG_DENSE, crbm.BF16, 1e-6,
                            args.cg_maxit, stats)
        off[0] += sweeps * N

    el, phases = _timed(plan, step, args.steps, args.warmup)
    st = stats.cpu().numpy()
    print(json.dumps({"metric": "MC samples/s + SR steps/s of the ground-state search", "value": ns / el,
                      "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "bf16", "data": "synthetic",
                      "config": {"workload": "heisenberg_square10x10_rbm_alpha4_ground_state", "N": N, "M": M,
                                 "P": P, "chains": C, "sweeps": sweeps, "samples_per_step": ns,
                                 "diag_shift": wl.diag_shift, "lr": 0.05},
                      "energy_per_site": float(st[1]) / N, "cg_iterations": float(st[5]), "sr_flags": int(st[6]),
                      "phases": phases}))
    plan.close()


def bench_grad16(crbm, args):
    """16x16 lattice, alpha = 2 (P = 131,840): 8192 frozen samples (64 burn-in sweeps, one recorded),
    forward (R and tanh theta) and the hand-written backward of the fidelity surrogate."""
    from paper_2103_08804_amd.autograd import fidelity_loss
    wl = synth.SQUARE16
    N, M, P = wl.N, wl.M, wl.P
    C = wl.chains
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, C)
    mk = lambda sd: (lambda r: (crbm.init_rbm(r, sd, wl.param_std), r)[1])(crbm.RBM.empty(N, M))
    psm, psn, fit = mk(wl.param_seed + 1), mk(wl.param_seed + 2), mk(wl.param_seed + 3)
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    cheb = crbm.make_cheb(2, E0 + 0.9875 * W_scale, W_scale, 1.0, 1.0, (math.pi, math.pi))
    chains = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains, wl.chain_seed, True)
    crbm.sample(plan, fit, chains, 64, crbm.EXCHANGE, 31, 0)
    samples = chains.clone()
    a, b, W = (t.clone().requires_grad_(True) for t in (fit.a, fit.b, fit.W))

    def step():
        a.grad = b.grad = W.grad = None
        L = fidelity_loss(crbm.RBM(a, b, W), plan, samples, psn, psm, cheb)
        L.backward()

    el, phases = _timed(plan, step, args.steps, args.warmup)
    # forward local estimators (k_local): per sample and anti-aligned bond, every hidden unit multiplies its
    # bond factor (X + w Y: 4 FMA) into the running complex product (6 FLOP): 14 FLOP per (sample, bond, unit),
    # on the vector units; a bond's table row (M x 16 B) is read once per wave of 4 samples if any of them has
    # the bond anti-aligned.  The O^H c contraction of the backward (k_ot, one coefficient vector):
    # 8 (N + 1)(M + 1) n FLOP on the FP32 matrix cores.
    sg = samples.cpu().numpy().astype(np.int8).reshape(C, wl.Ly, wl.Lx)
    anti = np.stack([sg != np.roll(sg, -1, axis=2), sg != np.roll(sg, -1, axis=1)], axis=1).reshape(C, -1)
    n_anti = int(anti.sum())
    rows_read = int(anti[: C // 4 * 4].reshape(C // 4, 4, -1).any(axis=1).sum())
    t_loc = phases["local"]["avg_ms"] / 1e3
    f_loc = 14.0 * n_anti * M
    t_ot = phases["ot"]["avg_ms"] / 1e3
    f_ot = 8.0 * (N + 1) * (M + 1) * C
    roof = {"kernel": "k_local (forward local estimators)", "bound": "alu", "achieved": f_loc / t_loc / 1e12,
            "peak": 157.3, "unit": "TFLOP/s", "frac": f_loc / t_loc / 1e12 / 157.3, "traffic": None,
            "anti_aligned_bonds_per_sample": n_anti / C,
            "bond_table_read_TBps": rows_read * M * 16 / t_loc / 1e12,
            "peak_note": "FP32 vector peak (256 CUs x 4 SIMD x 64 lanes x 2 FLOP x 2.4 GHz)"}
    roof_ot = {"kernel": "k_ot (O^H c of the backward)", "bound": "mfma", "achieved": f_ot / t_ot / 1e12,
               "peak": FP32_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": f_ot / t_ot / 1e12 / FP32_MATRIX_PEAK_TFLOPS}
    print(json.dumps({"metric": "fidelity-surrogate gradients/s", "value": 1.0 / el, "unit": "gradients/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": "heisenberg_square16x16_rbm_alpha2_gradient", "N": N, "M": M, "P": P,
                                 "samples": C, "burn_in_sweeps": 64},
                      "samples_per_s": C / el, "phases": phases, "roofline": roof, "ot_roofline": roof_ot}))
    plan.close()


def cg_overhead(crbm, plan, fit, flat, T, R, wl, args, s_prec):
    """What the iterations enqueued past convergence cost: the dense SR step of the last timed step's
    inputs, from the same state, with the configured iteration cap and with the cap set to the
    iterations it needed (both converge identically); the difference of the two 'cg' phases."""
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = {}
    its = None
    for cap in (args.cg_maxit, None):
        f = crbm.RBM(fit.a.clone(), fit.b.clone(), fit.W.clone())
        torch.cuda.synchronize()
        plan.profile(True)
        crbm.sr_step(plan, f, flat, T, R, 0.1, wl.diag_shift, crbm.CG_DENSE, s_prec, 1e-6,
                     args.cg_maxit if cap else max(1, int(its)), stats)
        torch.cuda.synchronize()
        c, t = plan.profile_read()["cg"]
        plan.profile(False)
        if cap:
            its = float(stats[5].item())
            out["cg_ms"] = t / c
        else:
            out["cg_ms_cap_at_iterations"] = t / c
    out.update({"iterations": its, "cap": args.cg_maxit, "early_exit_launches": 5 * (args.cg_maxit - int(its)),
                "overhead_ms": out["cg_ms"] - out["cg_ms_cap_at_iterations"],
                "note": ("every iteration up to the cap is enqueued (5 launches) so that the host never waits on "
                         "a device flag; the ones after convergence return at once")})
    return out


def fp32_compare(crbm, plan, fit, step, flat, T, R, wl, args, ms_per_step, stats):
    """The plain FP32 path, measured: one whole step (sampling, local estimators, the natural-gradient step
    with FP32 operands in the S contraction, the moments) timed end to end after the BF16 steps; then the
    BF16 step is re-run from the state and samples that FP32 step started from, and the two updates dalpha
    are compared over all N_s = 524,288 samples (N_s > P)."""
    P = wl.P
    f0 = crbm.RBM(fit.a.clone(), fit.b.clone(), fit.W.clone())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(crbm.FP32)
    torch.cuda.synchronize()
    fp32_ms = (time.perf_counter() - t0) * 1e3
    st32 = stats.cpu().numpy().copy()
    d32 = torch.zeros(P, dtype=torch.complex128, device="cuda")
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, d32)
    # the BF16 step on the same state (f0) and the same samples, T and R (flat, T and R still hold them)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    crbm.sr_step(plan, f0, flat, T, R, 0.1, wl.diag_shift, crbm.CG_DENSE, crbm.BF16, 1e-6, args.cg_maxit, stats)
    torch.cuda.synchronize()
    bf16_sr_ms = (time.perf_counter() - t0) * 1e3
    st16 = stats.cpu().numpy().copy()
    d16 = torch.zeros(P, dtype=torch.complex128, device="cuda")
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, d16)
    torch.cuda.synchronize()
    diff = d16 - d32
    rel2 = float(torch.linalg.vector_norm(diff) / torch.linalg.vector_norm(d32))
    relmax = float(diff.abs().max() / d32.abs().max())
    ns = flat.shape[0]
    return {"fp32_ms_per_step": fp32_ms, "fp32_samples_per_s": ns / (fp32_ms / 1e3),
            "bf16_speedup_vs_fp32": fp32_ms / ms_per_step,
            "bf16_sr_step_ms_same_inputs": bf16_sr_ms,
            "samples": ns, "P": P,
            "dalpha_rel_diff_l2": rel2, "dalpha_rel_diff_max": relmax,
            "gamma": float(st32[0]), "cg_iterations": {"fp32": float(st32[5]), "bf16": float(st16[5])},
            "note": ("fp32_ms_per_step: one whole step with FP32 S timed end to end (not scaled); dalpha of a BF16 "
                     "and an FP32 solve from the same state and samples")}


def fit_quality_compare(crbm, n_steps, n_orders=2):
    """Fit quality with BF16 and with FP32 operands in the S contraction: the first Chebyshev vectors
    t~_1, t~_2 of S^z(pi, pi) psi_gs on the 4x4 lattice, alpha = 4 (P = 1,104), fitted by Monte Carlo
    natural-gradient steps (256 chains x 32 pair-exchange sweeps per step, dense CG, n_steps per order), from
    identical starting states, chains and sampler seeds.  Per precision, by exact enumeration of the 12,870
    configurations with S^z = 0 (the sector the pair-exchange chains and H keep): the infidelity gamma of each
    fitted vector to its target, and the moments mu_1, mu_2 of the fitted sequence."""
    from paper_2103_08804_amd import recursion as rc
    wl = synth.SQUARE4
    N, M = wl.N, wl.M
    q = (math.pi, math.pi)
    cfg = synth.all_configs(N)
    sector = torch.from_numpy(np.ascontiguousarray(cfg[cfg.astype(np.int32).sum(axis=1) == 0])).cuda()
    n_enum = sector.shape[0]
    plan = crbm.Plan(crbm.SQUARE, wl.Lx, wl.Ly, M, max(wl.n_samples, n_enum), crbm.PLAN_DENSE_S)
    gs = crbm.RBM.empty(N, M)
    crbm.init_rbm(gs, wl.param_seed, wl.param_std)
    t1 = crbm.RBM(gs.a.clone(), gs.b.clone(), gs.W.clone())
    r = torch.arange(N, device="cuda")
    t1.a += (0.1 * torch.exp(-1j * (q[0] * (r % wl.Lx) + q[1] * (r // wl.Lx)))).to(torch.complex64)
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    E_c = E0 + (1.0 - 0.0125) * W_scale
    chains0 = torch.zeros(wl.chains, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, chains0, wl.chain_seed, True)
    crbm.sample(plan, gs, chains0, 16, crbm.EXCHANGE, wl.chain_seed, 0)
    out = {}
    lp = torch.empty(n_enum, dtype=torch.complex64, device="cuda")
    w = torch.empty(n_enum, dtype=torch.float64, device="cuda")
    R = torch.empty(n_enum, dtype=torch.complex64, device="cuda")
    fs = torch.empty(5, dtype=torch.float64, device="cuda")
    for name, pr in (("bf16", crbm.BF16), ("fp32", crbm.FP32)):
        settings = rc.FitSettings(n_steps=n_steps, dgamma=0.2, diag_shift=wl.diag_shift, solver=crbm.CG_DENSE,
                                  precision=pr, cg_tol=1e-8, cg_maxit=2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = rc.chebyshev_recursion(plan, gs, t1, n_orders, q, E_c, W_scale, settings, chains=chains0.clone(),
                                     sweeps=wl.sweeps, seed=wl.chain_seed + 1)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        # exact infidelity of every fitted vector to its target (target built from the fitted predecessors)
        gam = []
        for n in range(n_orders):
            cur = rec.rbm(n, N, M)
            psi_n = gs if n == 0 else rec.rbm(n - 1, N, M)
            psi_nm1 = None if n == 0 else (gs if n == 1 else rec.rbm(n - 2, N, M))
            b_n = 1.0 if n == 0 else complex(rec.betas[n - 1].item())
            b_nm1 = 1.0 if n <= 1 else complex(rec.betas[n - 2].item())
            cheb = crbm.make_cheb(n, E_c, W_scale, b_n, b_nm1, q)
            crbm.local_estimators(plan, cur, sector, psi_n=psi_n, psi_nm1=psi_nm1, cheb=cheb, logpsi_out=lp, R_out=R)
            crbm.enum_weights(plan, lp, w)
            crbm.fit_stats(plan, R, fs, weights=w)
            gam.append(float(fs[0].item()))
        mu = rc.sequence_moments(plan, gs, rec, [q], sector, True)[0].cpu().numpy()
        out[name] = {"gamma_exact": gam, "gamma_mc_last_step": rec.final_stats[:, 0].cpu().numpy().tolist(),
                     "mu": [[float(z.real), float(z.imag)] for z in mu], "fit_seconds": secs}
    mb, mf = np.array(out["bf16"]["mu"]), np.array(out["fp32"]["mu"])
    out["mu_abs_diff_bf16_vs_fp32"] = np.abs((mb[:, 0] - mf[:, 0]) + 1j * (mb[:, 1] - mf[:, 1])).tolist()
    out["config"] = {"lattice": "4x4 periodic", "N": N, "M": M, "P": wl.P, "q": "(pi, pi)",
                     "steps_per_order": n_steps, "orders": n_orders, "chains": wl.chains, "sweeps": wl.sweeps,
                     "dgamma": 0.2, "diag_shift": wl.diag_shift, "E_c": E_c, "W_scale": W_scale,
                     "enumerated_configs": n_enum}
    plan.close()
    return out


def matfree_compare(crbm, plan, fit, flat, T, R, wl, args, ms_per_step, prof):
    """The library's matrix-free solver on the same samples: S v = <O^*(O v)> - <O>^*(<O> v) formed from
    the factored O at every CG iteration (theta product of V, O v, O^H u on the matrix cores) instead of
    the dense S.  Context only: the configured workload is the dense BF16 S contraction.  Its SR step is
    timed on the step's full sample set and swapped into the measured step time; dalpha is compared
    with a dense BF16 solve of the same inputs."""
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    P = wl.P
    dal, ms, its = {}, {}, {}
    for name, sv in (("dense", crbm.CG_DENSE), ("matfree", crbm.CG_MATFREE)):
        f = crbm.RBM(fit.a.clone(), fit.b.clone(), fit.W.clone())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        crbm.sr_step(plan, f, flat, T, R, 0.1, wl.diag_shift, sv, crbm.BF16, 1e-6, args.cg_maxit, stats)
        torch.cuda.synchronize()
        ms[name] = (time.perf_counter() - t0) * 1e3
        its[name] = float(stats[5].item())
        dx = torch.zeros(P, dtype=torch.complex128, device="cuda")
        crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
        torch.cuda.synchronize()
        dal[name] = dx
    dense_sr = sum(prof[k][1] / prof[k][0] for k in ("ot", "pack", "sbuild", "sborder", "cg") if k in prof)
    step = ms_per_step - dense_sr + ms["matfree"]
    rel = float((dal["matfree"] - dal["dense"]).abs().max() / dal["dense"].abs().max())
    return {"sr_ms": ms["matfree"], "cg_iterations": its["matfree"], "dense_sr_ms": dense_sr,
            "ms_per_step": step, "samples_per_s": flat.shape[0] / (step / 1e3),
            "speedup_vs_dense": ms_per_step / step, "dalpha_vs_dense_bf16_rel_diff": rel,
            "note": "context only; the configured workload is the dense BF16 S contraction"}


def cpu_baseline(budget_s, ns, sweeps, C):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload.

    Per-sample stages are timed on a few hundred samples and scaled to the step's
    sample count; the natural-gradient step is left out because the oracle's
    dense S for P = 40,500 (26 GB in double) and its O(P^2 n + P^3) cost do not fit
    a bounded run."""
    import oracle as orc

    wl = synth.SQUARE10
    N, M = wl.N, wl.M
    lat = orc.Lattice(1, wl.Lx, wl.Ly)
    mk = lambda s: orc.init_rbm(N, M, s, wl.param_std)
    fit, psn, psm, gs = mk(wl.param_seed + 3), mk(wl.param_seed + 2), mk(wl.param_seed + 1), mk(wl.param_seed)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate: sampler on a few chains x 1 sweep
    n_ch = 32
    spins = orc.init_chains(N, n_ch, wl.chain_seed, 1)
    t0 = time.perf_counter()
    smp, _, _, _ = orc.metropolis(fit, spins, 1, 1, 11, 0)
    t_sweep = (time.perf_counter() - t0) / n_ch           # seconds per chain-sweep
    sig = smp.reshape(-1, N)
    n_loc = 32
    E0 = synth.E0_PER_SITE_SQUARE * N
    W_scale = 1.5 * abs(E0)
    E_c = E0 + (1.0 - 0.0125) * W_scale
    t0 = time.perf_counter()
    orc.target_ratio(fit, psn, psm, lat, sig[:n_loc], 2, E_c, W_scale, q=(math.pi, math.pi))
    t_loc = (time.perf_counter() - t0) / n_loc
    ts = [mk(wl.param_seed + 10 + t) for t in range(20)]
    t0 = time.perf_counter()
    orc.moments(gs, ts, np.ones(20), [(math.pi, math.pi)], lat, sig[:n_loc])
    t_mom = (time.perf_counter() - t0) / n_loc
    # scale the bounded sample up to the budget
    per_sample = 2 * t_sweep + t_loc + t_mom
    n_big = max(n_loc, int(budget_s / max(per_sample, 1e-9)))
    n_big = min(n_big, 1 << 17)
    spins = orc.init_chains(N, n_big, wl.chain_seed, 1)
    t0 = time.perf_counter()
    smp, _, _, _ = orc.metropolis(fit, spins, 1, 1, 11, 0)
    t1 = time.perf_counter()
    sig = smp.reshape(-1, N)
    orc.target_ratio(fit, psn, psm, lat, sig, 2, E_c, W_scale, q=(math.pi, math.pi))
    t2 = time.perf_counter()
    orc.moments(gs, ts, np.ones(20), [(math.pi, math.pi)], lat, sig)
    t3 = time.perf_counter()
    per_sample = 2 * (t1 - t0) / n_big + (t2 - t1) / n_big + (t3 - t2) / n_big
    base = {"value": 1.0 / per_sample, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": (f"{n_big} chains x 1 sweep (x2 for the psi_gs chains), local estimators and 20 moments on "
                       f"{n_big} samples of the 10x10 alpha=4 workload, {t3 - t0:.1f} s of CPU time; "
                       "natural-gradient step excluded (oracle dense S of 26 GB)"),
            "seconds": t3 - t0}
    return base, moments_vs_oracle(orc, gs, ts, sig, lat, ns)


def moments_vs_oracle(orc, gs, ts, sig, lat, ns_step):
    """Error of the GPU moments mu_n (n <= 20, q = (pi, pi)) against the FP64 oracle on the same samples,
    beside the Monte-Carlo standard error at the step's sample count.  The moments do not go through S
    (their precision is the same in the BF16 and the FP32 step; the fit-quality comparison carries the
    precision of S into mu_n).  The RBMs are rounded to complex64 once and both sides use those values; the
    samples are the oracle sampler's own."""
    import torch
    import paper_2103_08804_amd as crbm
    r32 = lambda r: orc.RBM(*(np.asarray(x, np.complex64).astype(np.complex128) for x in (r.a, r.b, r.W)))
    gs32, ts32 = r32(gs), [r32(t) for t in ts]
    N, M, n_max = gs32.N, gs32.M, len(ts32)
    n = sig.shape[0]
    q = [(math.pi, math.pi)]
    betas = np.ones(n_max, np.complex128)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.complex64)).cuda()
    plan = crbm.Plan(crbm.SQUARE, lat.Lx, lat.Ly, M, n)
    mu = torch.zeros(1, n_max + 1, dtype=torch.complex128, device="cuda")
    crbm.chebyshev_moment(plan, crbm.RBM(dev(gs32.a), dev(gs32.b), dev(gs32.W)),
                          torch.from_numpy(np.stack([t.vector() for t in ts32]).astype(np.complex64)).cuda(),
                          torch.from_numpy(betas).cuda(), q, torch.from_numpy(np.ascontiguousarray(sig)).cuda(), mu)
    got = mu.cpu().numpy()[0]
    plan.close()
    ref = orc.moments(gs32, ts32, betas, q, lat, sig)[0]
    scale = np.abs(ref).max()
    err = float(np.abs(got - ref).max() / scale)
    # per-sample terms on a subset give the spread; the standard error is for the step's sample count
    sub = np.ascontiguousarray(sig[:min(n, 8192)])
    f = orc.fq(lat, q[0], sub)
    lg = orc.logpsi(gs32, sub)
    terms = [np.abs(f) ** 2] + [np.conj(f) * np.exp(orc.logpsi(t, sub) - lg) for t in ts32]
    sigma = float(max(np.std(t) for t in terms) / math.sqrt(ns_step) / scale)
    return {"n_samples": n, "rel_error": err, "sigma_mc_rel": sigma,
            "note": ("max_n |mu_n - mu_n(FP64 oracle)| / max_n |mu_n| on the oracle's samples; sigma_mc: largest "
                     "standard error of the mean at the step's sample count (per-sample spread on "
                     f"{sub.shape[0]} samples), same scale")}


if __name__ == "__main__":
    main()
