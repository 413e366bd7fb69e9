"""The allocation-free fidelity gradient (crbm_fidelity_grad_noalloc, static device scratch) against the
plan-based crbm_fidelity_grad, both called through the C ABI: two calls in a row, the second with a smaller
input (fewer samples, fewer sites and hidden units), so that the second runs on scratch the first left
behind.  Both use the same kernels and the same sample chunks, so the gradient and the loss must be
bit-identical (stronger than the 1e-5 bound of the gradient against the oracle)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()


def _inputs(seed, kind, Lx, Ly, M, n):
    N = Lx * (Ly if kind == crbm.SQUARE else 1)
    r = np.random.default_rng(seed)
    sig = synth.random_spins(seed, n, N, True)
    T = (r.normal(0, 0.7, (n, M)) + 1j * r.normal(0, 0.7, (n, M))).astype(np.complex64)
    R = (1.0 + 0.3 * r.normal(size=n) + 0.3j * r.normal(size=n)).astype(np.complex64)
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return N, d(sig), d(T), d(R)


def _both(kind, Lx, Ly, M, n, seed):
    N, sig, T, R = _inputs(seed, kind, Lx, Ly, M, n)
    P = N + M + N * M
    plan = crbm.Plan(kind, Lx, Ly, M, n)
    g_plan = torch.zeros(P, dtype=torch.complex128, device="cuda")
    l_plan = torch.zeros(1, dtype=torch.float64, device="cuda")
    fit = crbm.RBM.empty(N, M)   # parameters are not read by the gradient of frozen samples
    crbm.fidelity_grad(plan, fit, sig, T, R, g_plan, l_plan)
    g_na = torch.full((P,), float("nan"), dtype=torch.complex128, device="cuda")
    l_na = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    L = crbm.lib()
    rc = L.crbm_fidelity_grad_noalloc(N, M, ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                      ctypes.c_void_p(R.data_ptr()), n, ctypes.c_void_p(g_na.data_ptr()),
                                      ctypes.c_void_p(l_na.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == crbm.CRBM_OK, L.crbm_last_error()
    torch.cuda.synchronize()
    plan.close()
    return (g_plan.cpu().numpy(), l_plan.cpu().numpy()), (g_na.cpu().numpy(), l_na.cpu().numpy())


def test_noalloc_gradient_equals_plan_gradient_twice():
    # the 16 x 16 lattice with M = 512 (the gradient workload's shape), then a smaller 6 x 6 input
    for kind, Lx, Ly, M, n, seed in [(crbm.SQUARE, 16, 16, 512, 8192, 91), (crbm.SQUARE, 6, 6, 40, 777, 92)]:
        (g0, l0), (g1, l1) = _both(kind, Lx, Ly, M, n, seed)
        assert np.all(np.isfinite(g1)) and np.isfinite(l1[0])
        assert np.array_equal(g0, g1), np.max(np.abs(g0 - g1))
        assert np.array_equal(l0, l1)
        print(f"{Lx}x{Ly} M={M} n={n}: |grad| {np.linalg.norm(g1):.4e}, loss {l1[0]:.6f}, bit-identical")


def test_noalloc_rejects_oversized_input():
    L = crbm.lib()
    dummy = ctypes.c_void_p(1)
    rc = L.crbm_fidelity_grad_noalloc(256, 512, dummy, dummy, dummy, 1 << 20, dummy, None, None)
    assert rc == crbm.CRBM_ENOMEM
    assert b"static scratch" in L.crbm_last_error()
