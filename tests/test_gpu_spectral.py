"""GPU parity of the moment-correction path (Sec. IV), the Lanczos continued fraction (Sec. V) and
the Jackson-damped reconstruction (Eq. Aw) against the FP64 oracle.

Tolerances.  G and H come from FP32 per-sample ratios accumulated in double: 1e-5 of max|G|, max|H|,
or, for large models, the bound of the binary32 log amplitudes behind each ratio (ratio_gram_tol).
The small dense kernels run in double on double inputs: corrected moments within 1e-9 mu_0 (the
recursion multiplies rounding by the conditioning of G, which these cases keep moderate), spectra
within 1e-9 of their maximum, and the exactness pins (Krylov basis, cyclic space) as in the oracle
tests."""
import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth
from gpu_util import log_amp_scale, np_of, ratio_gram_tol, to_device_rbm, to_oracle_rbm
from oracle import exact, spectral

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


# ------------------------------------------------------------------ G and H
MM_CASES = [
    # kind, Lx, Ly, M, n_max, n_samples (None = enumeration), q
    (0, 10, 1, 10, 4, None, (np.pi, 0.0)),
    (1, 4, 4, 16, 6, 777, (np.pi, np.pi)),
    (0, 8, 1, 4, 40, 333, (np.pi / 2, 0.0)),
    # the benchmarked shape (10 x 10, alpha = 4, K = 21) on 128 samples the oracle sums in seconds
    (1, 10, 10, 400, 20, 128, (np.pi, np.pi)),
]


@pytest.mark.parametrize("kind,Lx,Ly,M,n_max,n,q", MM_CASES)
def test_moment_matrices(orc, kind, Lx, Ly, M, n_max, n, q):
    N = Lx * Ly
    lat = orc.Lattice(kind, Lx, Ly)
    gs_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(90 + N, N, M, 0.1, std_im=0.05)))
    gs = to_oracle_rbm(orc, gs_d)
    tvec = [orc.RBM(*synth.random_rbm_arrays(91 + N + t, N, M, 0.1, std_im=0.05)).vector() for t in range(n_max)]
    tp = _dev(np.stack(tvec).astype(np.complex64), torch.complex64)
    ts = [orc.RBM.from_vector(np_of(tp[t]).astype(np.complex128), N, M) for t in range(n_max)]
    r = np.random.default_rng(N)
    betas = r.normal(size=n_max) + 1j * r.normal(size=n_max)
    sig = orc.enumerate_configs(N) if n is None else synth.random_spins(92, n, N, True)
    ns = sig.shape[0]
    w = orc.enum_weights(orc.logpsi(gs, sig)) if n is None else None
    K = n_max + 1
    plan = crbm.Plan(kind, Lx, Ly, M, ns, crbm.PLAN_BASIS, basis_k_max=K)
    G = torch.zeros(K, K, dtype=torch.complex128, device="cuda")
    H = torch.zeros_like(G)
    sig_d = _dev(sig, torch.int8)
    w_d = None if w is None else _dev(w, torch.float64)
    crbm.moment_matrices(plan, gs_d, tp, _dev(betas, torch.complex128), q, sig_d, G, H, weights=w_d)
    mu = torch.zeros(1, K, dtype=torch.complex128, device="cuda")
    crbm.chebyshev_moment(plan, gs_d, tp, _dev(betas, torch.complex128), [q], sig_d, mu, weights=w_d)
    torch.cuda.synchronize()
    G_ref, H_ref = orc.moment_matrices(gs, ts, betas, q, lat, sig, weights=w)
    eg = np.max(np.abs(np_of(G) - G_ref)) / np.max(np.abs(G_ref))
    eh = np.max(np.abs(np_of(H) - H_ref)) / np.max(np.abs(H_ref))
    tol = ratio_gram_tol(max(log_amp_scale(t, sig) for t in ts), log_amp_scale(gs, sig))
    print("K", K, "G err", eg, "H err", eh, "tolerance", tol)
    assert eg < tol and eh < tol
    # row 0 of G is the moment estimator on the same samples
    assert np.max(np.abs(np_of(G)[0] - np_of(mu)[0])) < 1e-5 * np.max(np.abs(G_ref[0]))


# ------------------------------------------------------------------ small dense kernels
def _random_krylov(dim=40, seed=3, K=8):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.normal(size=(dim, dim)) + 1j * r.normal(size=(dim, dim)))
    ev = np.sort(r.uniform(-2.0, 3.0, dim))
    Hf = (Q * ev) @ Q.conj().T
    Hf = 0.5 * (Hf + Hf.conj().T)
    t0 = r.normal(size=dim) + 1j * r.normal(size=dim)
    t0 /= np.linalg.norm(t0)
    E_c, W_scale = 0.5, 2.7
    Hp = (Hf - E_c * np.eye(dim)) / W_scale
    ts = [t0, Hp @ t0]
    for n in range(1, 4 * K):
        ts.append(2.0 * Hp @ ts[n] - ts[n - 1])
    mu = np.array([np.vdot(t0, t) for t in ts]).real
    T = np.stack(ts[:K], axis=1)
    return T.conj().T @ T, T.conj().T @ (Hf @ T), E_c, W_scale, mu


def _oracle_rbm_matrices(orc):
    N, M, n_max = 10, 10, 5
    lat = orc.Lattice(0, N)
    gs = orc.RBM(*synth.random_rbm_arrays(120, N, M, 0.1, std_im=0.05))
    ts = [orc.RBM(*synth.random_rbm_arrays(121 + t, N, M, 0.1, std_im=0.05)) for t in range(n_max)]
    sig = orc.enumerate_configs(N)
    G, H = orc.moment_matrices(gs, ts, np.ones(n_max), (np.pi, 0.0), lat, sig,
                               weights=orc.enum_weights(orc.logpsi(gs, sig)))
    E0 = exact.ground_state(exact.heisenberg_sparse(N, lat.bonds()))[0]
    E_c, W_scale = exact.rescaling(E0)
    return G, H, E_c, W_scale, E0


def test_corrected_moments_krylov_exact():
    K = 8
    G, H, E_c, W_scale, mu_ex = _random_krylov(K=K)
    plan = crbm.Plan(0, 4, 1, 1, 1)
    n_out = 3 * K
    mu = torch.zeros(n_out, dtype=torch.float64, device="cuda")
    info = torch.zeros(3, dtype=torch.float64, device="cuda")
    crbm.corrected_moments(plan, _dev(G, torch.complex128), _dev(H, torch.complex128), E_c, W_scale, mu, info)
    torch.cuda.synchronize()
    got = np_of(mu)
    assert int(np_of(info)[0]) == 0
    assert np.allclose(got[:2 * K], mu_ex[:2 * K], rtol=0, atol=1e-10)
    ref = spectral.corrected_moments(G, H, E_c, W_scale, n_out)
    assert np.max(np.abs(got - ref)) < 1e-9 * abs(ref[0])


def test_corrected_moments_rbm_basis(orc):
    G, H, E_c, W_scale, _ = _oracle_rbm_matrices(orc)
    K = G.shape[0]
    plan = crbm.Plan(0, 4, 1, 1, 1)
    n_out = 64
    mu = torch.zeros(n_out, dtype=torch.float64, device="cuda")
    info = torch.zeros(3, dtype=torch.float64, device="cuda")
    crbm.corrected_moments(plan, _dev(G, torch.complex128), _dev(H, torch.complex128), E_c, W_scale, mu, info)
    torch.cuda.synchronize()
    ref = spectral.corrected_moments(G, H, E_c, W_scale, n_out)
    inf = np_of(info)
    print("cond(G)", np.linalg.cond(G), "info", inf)
    assert int(inf[0]) == 0
    assert inf[1] <= 1.0 + 1e-9                 # an exact projection keeps |mu_n| <= mu_0
    assert np.max(np.abs(np_of(mu) - ref)) < 1e-9 * abs(ref[0])


def test_corrected_moments_rejects_indefinite_overlap():
    G = np.diag([1.0, -1.0, 2.0]).astype(np.complex128)
    H = np.eye(3, dtype=np.complex128)
    plan = crbm.Plan(0, 4, 1, 1, 1)
    mu = torch.full((5,), 7.0, dtype=torch.float64, device="cuda")
    info = torch.zeros(3, dtype=torch.float64, device="cuda")
    crbm.corrected_moments(plan, _dev(G, torch.complex128), _dev(H, torch.complex128), 0.0, 1.0, mu, info)
    torch.cuda.synchronize()
    assert int(np_of(info)[0]) == crbm.FLAG_CHOLESKY_FAIL
    assert np.all(np_of(mu) == 0.0)


def _cf_gpu(plan, G, H, E0, eta, omega, n_steps=None):
    K = G.shape[0]
    m = n_steps or K
    a = torch.zeros(m, dtype=torch.float64, device="cuda")
    b2 = torch.zeros(m, dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.float64, device="cuda")
    crbm.lanczos(plan, _dev(G, torch.complex128), _dev(H, torch.complex128), a, b2, info)
    torch.cuda.synchronize()
    inf = np_of(info)
    assert int(inf[0]) == 0
    done = int(inf[1])
    A = torch.zeros(len(omega), dtype=torch.float64, device="cuda")
    crbm.spectrum_cf(a, b2, done, E0, eta, _dev(omega, torch.float64), A)
    torch.cuda.synchronize()
    return np_of(A), done


@pytest.mark.parametrize("src", ["krylov", "rbm"])
def test_lanczos_continued_fraction(orc, src):
    if src == "krylov":
        G, H, _, _, _ = _random_krylov(K=8)
        E0 = -2.0
    else:
        G, H, _, _, E0 = _oracle_rbm_matrices(orc)
    plan = crbm.Plan(0, 4, 1, 1, 1)
    omega = np.linspace(-1.0, 8.0, 1001)
    eta = 0.1
    A, done = _cf_gpu(plan, G, H, E0, eta, omega)
    ref = spectral.cf_spectrum(G, H, E0, eta, omega)
    assert done == G.shape[0]
    assert np.max(np.abs(A - ref)) < 1e-9 * np.max(ref)


def test_continued_fraction_exact_on_cyclic_space():
    """Heisenberg 8-site ring: the Chebyshev vectors spanning the cyclic space of S^z_pi psi_0 give
    the exact Lorentzian-broadened spectrum, and Lanczos stops at the invariant subspace."""
    N = 8
    Hs = exact.heisenberg_sparse(N, [(i, (i + 1) % N) for i in range(N)])
    E0, psi = exact.ground_state(Hs)
    E_c, W_scale = exact.rescaling(E0)
    f = exact.sz_q_diag(N, exact.positions_of(0, N, 1, N), (np.pi, 0.0))
    _, ts = exact.chebyshev_moments_exact(Hs, psi, f, E_c, W_scale, 10)
    Hd = Hs.toarray()
    ev, V = np.linalg.eigh(Hd)
    amp = np.abs(V.conj().T @ ts[0]) ** 2
    levels = []
    for e, a in zip(ev, amp):
        if a > 1e-14:
            if levels and abs(e - levels[-1][0]) < 1e-9:
                levels[-1][1] += a
            else:
                levels.append([e, a])
    K = len(levels)
    T = np.stack(ts[:K], axis=1)
    plan = crbm.Plan(0, 4, 1, 1, 1)
    omega = np.linspace(-0.5, 6.0, 501)
    eta = 0.1
    A, done = _cf_gpu(plan, T.conj().T @ T, T.conj().T @ (Hd @ T), E0, eta, omega, n_steps=K + 3)
    ref = sum(a * eta / ((omega + E0 - e) ** 2 + eta ** 2) for e, a in levels) / np.pi
    assert done == K
    assert np.allclose(A, ref, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("jackson", [True, False])
def test_kpm_spectrum(jackson):
    N = 8
    Hs = exact.heisenberg_sparse(N, [(i, (i + 1) % N) for i in range(N)])
    E0, psi = exact.ground_state(Hs)
    E_c, W_scale = exact.rescaling(E0)
    f = exact.sz_q_diag(N, exact.positions_of(0, N, 1, N), (np.pi, 0.0))
    mu, _ = exact.chebyshev_moments_exact(Hs, psi, f, E_c, W_scale, 99)
    omega = np.linspace(-1.0, 2 * W_scale, 2001)       # crosses both ends of the expansion interval
    A = torch.zeros(len(omega), dtype=torch.float64, device="cuda")
    crbm.spectrum_kpm(_dev(mu.real, torch.float64), E0, E_c, W_scale, _dev(omega, torch.float64), A, jackson=jackson)
    torch.cuda.synchronize()
    ref = spectral.kpm_spectrum(mu, E0, E_c, W_scale, omega, damping=jackson)
    assert np.max(np.abs(np_of(A) - ref)) < 1e-9 * np.max(np.abs(ref))


def test_moment_matrices_first_call_under_graph_capture(orc):
    """With the basis workspace reserved at plan creation, the very first crbm_moment_matrices call on a plan
    (and crbm_corrected_moments after it) can be captured in a graph: nothing allocates or synchronises.
    Each of three replays, with eager work of the program between them, equals an eager run on a second
    plan bit for bit."""
    N, M, n_max, n = 8, 8, 4, 700
    K = n_max + 1
    lat = orc.Lattice(0, N)
    gs_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(95, N, M, 0.1, std_im=0.05)))
    tp = _dev(np.stack([orc.RBM(*synth.random_rbm_arrays(96 + t, N, M, 0.1, std_im=0.05)).vector()
                        for t in range(n_max)]).astype(np.complex64), torch.complex64)
    betas = _dev(np.linspace(0.5, 1.5, n_max) + 0.1j, torch.complex128)
    sig = _dev(synth.random_spins(97, n, N, True), torch.int8)
    q = (np.pi, 0.0)
    E0 = -3.6510934089371783   # any scale: the same on both sides
    E_c, W_scale = E0 + 0.9875 * 1.5 * abs(E0), 1.5 * abs(E0)

    def run(plan, G, H, mu, info):
        crbm.moment_matrices(plan, gs_d, tp, betas, q, sig, G, H)
        crbm.corrected_moments(plan, G, H, E_c, W_scale, mu, info)

    def bufs():
        G = torch.zeros(K, K, dtype=torch.complex128, device="cuda")
        return G, torch.zeros_like(G), torch.zeros(12, dtype=torch.float64, device="cuda"), \
            torch.zeros(3, dtype=torch.float64, device="cuda")

    eager_plan = crbm.Plan(0, N, 1, M, n, crbm.PLAN_BASIS, basis_k_max=K)
    ref = bufs()
    run(eager_plan, *ref)
    plan = crbm.Plan(0, N, 1, M, n, crbm.PLAN_BASIS, basis_k_max=K)
    out = bufs()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run(plan, *out)           # the plan's first call
    for rep in range(3):
        for t in out:
            t.fill_(-7.0)         # the program's own eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), rep
    # without the reservation the call refuses instead of allocating
    bare = crbm.Plan(0, N, 1, M, n)
    with pytest.raises(crbm.CrbmError) as ei:
        crbm.moment_matrices(bare, gs_d, tp, betas, q, sig, *bufs()[:2])
    assert ei.value.code == crbm.CRBM_ENOMEM
    for p in (plan, eager_plan, bare):
        p.close()
