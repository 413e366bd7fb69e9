"""GPU parity of the symmetry-projected moment-correction matrices (App. A, crbm_sym_matrices)
against the FP64 oracle: G^(k) and H^(k) for every lattice momentum, with and without rotations,
in one chunk and split into several chunks of samples (ragged last chunk).

Tolerance: FP32 per-image ratios and local energies, FP32 momentum sums, double Gram sums:
1e-5 of the largest |G^(k)| (|H^(k)|) over all k, or, for large models, the bound of the binary32 log
amplitudes behind each ratio (ratio_gram_tol)."""
import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth
from gpu_util import lattice_images, log_amp_scale, np_of, ratio_gram_tol, to_device_rbm, to_oracle_rbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()


CASES = [
    # kind, Lx, Ly, M, n_max, n (None = enumeration), rotations, samples per chunk (None = all)
    (1, 3, 3, 4, 2, None, True, None),
    (1, 3, 3, 4, 2, None, True, 100),
    (1, 4, 4, 8, 3, 333, True, None),
    (1, 4, 4, 8, 3, 333, False, 77),
    (0, 8, 1, 6, 3, 97, False, None),
    # the benchmarked shape (6 x 6, alpha = 2, 144 images, K = 21) on 64 samples
    (1, 6, 6, 72, 20, 64, True, None),
]


@pytest.mark.parametrize("kind,Lx,Ly,M,n_max,n,rot,chunk", CASES)
def test_sym_matrices(orc, kind, Lx, Ly, M, n_max, n, rot, chunk):
    lat = orc.Lattice(kind, Lx, Ly)
    N = lat.N
    gs_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(60 + N, N, M, 0.15, std_im=0.05)))
    gs = to_oracle_rbm(orc, gs_d)
    tv = np.stack([orc.RBM(*synth.random_rbm_arrays(61 + N + t, N, M, 0.15, std_im=0.05)).vector()
                   for t in range(n_max)]).astype(np.complex64)
    ts = [orc.RBM.from_vector(tv[t].astype(np.complex128), N, M) for t in range(n_max)]
    r = np.random.default_rng(N)
    betas = r.normal(size=n_max) + 1j * r.normal(size=n_max)
    sig = orc.enumerate_configs(N) if n is None else synth.random_spins(62, n, N, N % 2 == 0)
    ns = sig.shape[0]
    w = orc.enum_weights(orc.logpsi(gs, sig)) if n is None else None
    ng = N * (4 if rot else 1)
    K = n_max + 1
    plan = crbm.Plan(kind, Lx, Ly, M, ng * (chunk or ns), crbm.PLAN_SYM_BASIS, basis_k_max=K)
    G = torch.zeros(N, K, K, dtype=torch.complex128, device="cuda")
    H = torch.zeros_like(G)
    crbm.sym_matrices(plan, gs_d, torch.from_numpy(tv).cuda(), torch.from_numpy(betas).cuda(),
                      torch.from_numpy(sig).cuda(), G, H, rotations=rot,
                      weights=None if w is None else torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    G_ref, H_ref = orc.sym_matrices(gs, ts, betas, lat, sig, rotations=rot, weights=w)
    eg = np.max(np.abs(np_of(G) - G_ref)) / np.max(np.abs(G_ref))
    eh = np.max(np.abs(np_of(H) - H_ref)) / np.max(np.abs(H_ref))
    img = lattice_images(sig, Lx, Ly, rot)
    tol = ratio_gram_tol(max([log_amp_scale(t, img) for t in ts] + [log_amp_scale(gs, img)]), log_amp_scale(gs, sig))
    print("G err", eg, "H err", eh, "tolerance", tol)
    assert eg < tol and eh < tol


def test_sym_matrices_rejects_bad_shapes(orc):
    plan = crbm.Plan(1, 4, 2, 4, 1000, crbm.PLAN_SYM_BASIS, basis_k_max=1)
    gs = crbm.RBM.empty(8, 4)
    crbm.init_rbm(gs, 1, 0.01)
    sig = torch.ones(3, 8, dtype=torch.int8, device="cuda")
    G = torch.zeros(8, 1, 1, dtype=torch.complex128, device="cuda")
    with pytest.raises(crbm.CrbmError):                  # rotations need L x L
        crbm.sym_matrices(plan, gs, None, None, sig, G, G.clone(), rotations=True)
    small = crbm.Plan(1, 4, 4, 4, 10, crbm.PLAN_SYM_BASIS, basis_k_max=1)
    gs16 = crbm.RBM.empty(16, 4)
    crbm.init_rbm(gs16, 1, 0.01)
    G16 = torch.zeros(16, 1, 1, dtype=torch.complex128, device="cuda")
    with pytest.raises(crbm.CrbmError):                  # 64 images do not fit max_samples = 10
        crbm.sym_matrices(small, gs16, None, None, torch.ones(2, 16, dtype=torch.int8, device="cuda"), G16,
                          G16.clone(), rotations=True)
