"""GPU parity of the ground-state natural-gradient step (crbm_sr_energy_step) against the oracle's
FP64 twin, and an end-to-end Monte-Carlo ground-state search checked against exact diagonalisation.

Tolerances: <E>, F and the variance within 1e-5 relative (FP32 local energies, double sums);
dalpha within 2e-3 (S is stored in FP32 and the solve multiplies its rounding by the condition
number, as for the fit step)."""
import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth
from gpu_util import np_of, rel_err, to_device_rbm, to_oracle_rbm
from oracle import exact

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()


def _energy_step_gpu(plan, fit_d, sig_d, lr, eps, solver, prec, weights=None, tol=1e-10, maxit=2000):
    n = sig_d.shape[0]
    T = torch.zeros(n, plan.M, dtype=torch.complex64, device="cuda")
    El = torch.zeros(n, dtype=torch.complex64, device="cuda")
    crbm.local_estimators(plan, fit_d, sig_d, eloc_out=El, tanh_out=T)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    crbm.sr_energy_step(plan, fit_d, sig_d, T, El, lr, eps, solver, prec, tol, maxit, stats, weights=weights)
    return stats, El


@pytest.mark.parametrize("solver,flags", [(crbm.CG_DENSE, crbm.PLAN_DENSE_S), (crbm.CG_MATFREE, 0),
                                          (crbm.CHOLESKY, crbm.PLAN_CHOLESKY)])
def test_energy_step_enumeration(orc, solver, flags):
    N, M = 10, 10
    lat = orc.Lattice(0, N)
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(21, N, M, 0.2, std_im=0.05)))
    fit = to_oracle_rbm(orc, fit_d)
    sig = orc.enumerate_configs(N)
    p = orc.enum_weights(orc.logpsi(fit, sig))
    plan = crbm.Plan(0, N, 1, M, sig.shape[0], flags)
    sig_d = torch.from_numpy(sig).cuda()
    lr, eps = 0.05, 1e-3
    stats, El = _energy_step_gpu(plan, fit_d, sig_d, lr, eps, solver, crbm.FP32, weights=torch.from_numpy(p).cuda())
    F = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
    dx = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
    torch.cuda.synchronize()
    El_ref = orc.local_energy(fit, lat, sig)
    assert rel_err(np_of(El), El_ref) < 1e-5
    _, info = orc.sr_energy_step(fit, sig, El_ref, lr, eps, weights=p)
    st = np_of(stats)
    assert int(st[6]) == 0, st
    assert abs(complex(st[1], st[2]) - info["E"]) < 1e-5 * abs(info["E"])
    assert abs(st[0] - info["var"]) < 1e-5 * abs(info["E"]) ** 2
    assert rel_err(np_of(F), info["F"]) < 1e-5
    assert rel_err(np_of(dx), info["dalpha"]) < 2e-3
    got_new = to_oracle_rbm(orc, fit_d).vector()
    assert rel_err(got_new - fit.vector(), info["dalpha"]) < 2e-3


@pytest.mark.parametrize("prec", [crbm.FP32, crbm.BF16])
def test_energy_step_mc_square(orc, prec):
    """Uniform weights on Monte-Carlo-like samples of the 4x4 square lattice, dense S on the matrix
    cores.  FP32 operands: F to 1e-5, dalpha to 1e-3.  BF16 operands: F is formed from the same rounded
    operands as S, |dF_k| <= lr 2^-9 <|O'_k| |E - <E>|> <= lr 2^-9 sqrt(S_kk var E) (Cauchy-Schwarz, O' the
    shifted operand; asserted with a factor 2), and dalpha within the first-order bound of the S and F
    perturbations."""
    Lx = Ly = 4
    N, M, n = 16, 16, 1500
    lat = orc.Lattice(1, Lx, Ly)
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(31, N, M, 0.1, std_im=0.03)))
    fit = to_oracle_rbm(orc, fit_d)
    sig = synth.random_spins(32, n, N, True)
    plan = crbm.Plan(1, Lx, Ly, M, n, crbm.PLAN_DENSE_S)
    lr, eps = 0.05, 1e-2
    stats, El = _energy_step_gpu(plan, fit_d, torch.from_numpy(sig).cuda(), lr, eps, crbm.CG_DENSE, prec)
    F = torch.zeros(plan.P, dtype=torch.complex128, device="cuda")
    dx = torch.zeros_like(F)
    crbm.copy_plan_buffer(plan, crbm.BUF_F, F)
    crbm.copy_plan_buffer(plan, crbm.BUF_DALPHA, dx)
    torch.cuda.synchronize()
    _, info = orc.sr_energy_step(fit, sig, orc.local_energy(fit, lat, sig), lr, eps, want_S=True)
    st = np_of(stats)
    assert int(st[6]) == 0, st
    assert abs(complex(st[1], st[2]) - info["E"]) < 1e-5 * abs(info["E"])
    if prec == crbm.FP32:
        assert rel_err(np_of(F), info["F"]) < 1e-5
        assert rel_err(np_of(dx), info["dalpha"]) < 1e-3
    else:
        f_bound = 2.0 ** -8 * lr * np.sqrt(np.real(np.diag(info["S"])) * info["var"])
        dF = np.abs(np_of(F) - info["F"])
        print("BF16 F: max error / bound", (dF / f_bound).max())
        assert np.all(dF <= f_bound + 1e-15)
        ev = np.linalg.eigvalsh(info["S"] + eps * np.eye(plan.P))
        rel_f = np.linalg.norm(dF) / np.linalg.norm(info["F"])
        assert rel_err(np_of(dx), info["dalpha"]) < max(1e-3, 4 * ev.max() / ev.min() * (2 ** -7 + rel_f))


def test_energy_descent_enumeration_tracks_oracle(orc):
    """Thirty exact-expectation steps on the 10-site ring: the GPU trajectory stays on the oracle's,
    the energy never crosses the exact ground energy, and it decreases."""
    N, M = 10, 10
    lat = orc.Lattice(0, N)
    sig = orc.enumerate_configs(N)
    E0, _ = exact.ground_state(exact.heisenberg_sparse(N, lat.bonds()))
    fit_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(41, N, M, 0.05, std_im=0.02)))
    ref = to_oracle_rbm(orc, fit_d)
    plan = crbm.Plan(0, N, 1, M, sig.shape[0], crbm.PLAN_CHOLESKY)
    sig_d = torch.from_numpy(sig).cuda()
    lr, eps = 0.1, 1e-3
    eg, er = [], []
    for _ in range(30):
        lp = torch.zeros(sig.shape[0], dtype=torch.complex64, device="cuda")
        crbm.local_estimators(plan, fit_d, sig_d, logpsi_out=lp)
        re = lp.real.double()
        w = torch.exp(2.0 * (re - re.max()))
        w = (w / w.sum()).contiguous()
        stats, _ = _energy_step_gpu(plan, fit_d, sig_d, lr, eps, crbm.CHOLESKY, crbm.FP32, weights=w)
        eg.append(float(np_of(stats)[1]))
        p = orc.enum_weights(orc.logpsi(ref, sig))
        ref, info = orc.sr_energy_step(ref, sig, orc.local_energy(ref, lat, sig), lr, eps, weights=p)
        er.append(info["E"].real)
    eg, er = np.array(eg), np.array(er)
    print("E0", E0, "gpu", eg[[0, 9, 19, 29]], "oracle", er[[0, 9, 19, 29]])
    assert np.all(eg >= E0 - 1e-5 * abs(E0))
    assert np.max(np.abs(eg - er)) < 2e-3 * abs(E0)
    assert eg[-1] < eg[0] - 1.0


def test_ground_state_monte_carlo_ring():
    """Monte-Carlo ground-state search on the 10-site ring (alpha = 2, exchange moves, BF16 dense S):
    the sampled energy approaches the exact E0 to within 1 percent."""
    N, M = 10, 20
    E0, _ = exact.ground_state(exact.heisenberg_sparse(N, [(i, (i + 1) % N) for i in range(N)]))
    C, sweeps = 1024, 4
    n = C * sweeps
    plan = crbm.Plan(0, N, 1, M, n, crbm.PLAN_DENSE_S)
    psi = crbm.RBM.empty(N, M)
    crbm.init_rbm(psi, 7, 0.01)
    spins = torch.zeros(C, N, dtype=torch.int8, device="cuda")
    crbm.init_chains(plan, spins, 8, True)
    samples = torch.zeros(sweeps, C, N, dtype=torch.int8, device="cuda")
    energies = []
    for it in range(300):
        crbm.sample(plan, psi, spins, sweeps, crbm.EXCHANGE, 9, step_offset=it * sweeps * N, samples_out=samples)
        stats, _ = _energy_step_gpu(plan, psi, samples.view(n, N), 0.1, 1e-3, crbm.CG_DENSE, crbm.BF16,
                                    tol=1e-6, maxit=300)
        energies.append(float(np_of(stats)[1]))
    tail = np.mean(energies[-20:])
    print("E0", E0, "E first", energies[0], "E last 20", tail)
    assert energies[0] > E0 + 1.0
    assert abs(tail - E0) < 0.01 * abs(E0)
