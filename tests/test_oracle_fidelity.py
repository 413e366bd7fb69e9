"""Pin for the fidelity-surrogate gradient: central finite differences in FP64.

L(alpha) = (1/n) sum_s |1 - R(s; alpha)|^2 on a frozen sample set, with R the
Chebyshev target ratio; grad = dL/dRe(alpha) + i dL/dIm(alpha).
"""
import numpy as np

import synth


def test_fidelity_gradient_finite_differences(orc):
    N, M = 6, 4
    lat = orc.Lattice(0, N)
    fit = orc.RBM(*synth.random_rbm_arrays(60, N, M, 0.3))
    psn = orc.RBM(*synth.random_rbm_arrays(61, N, M, 0.3))
    psm = orc.RBM(*synth.random_rbm_arrays(62, N, M, 0.3))
    sig = synth.random_spins(63, 64, N, True)
    args = dict(lat=lat, sig=sig, order=2, E_c=-1.3, W_scale=2.5, beta_n=0.9, beta_nm1=1.1)

    def loss(rbm):
        R = orc.target_ratio(rbm, psn, psm, **args)
        return orc.fidelity_grad(rbm, sig, R)

    L0, g = loss(fit)
    v0 = fit.vector()
    r = np.random.default_rng(0)

    def central(k, h):
        fd = []
        for d in (1.0, 1j):
            vp, vm = v0.copy(), v0.copy()
            vp[k] += h * d
            vm[k] -= h * d
            Lp, _ = loss(orc.RBM.from_vector(vp, N, M))
            Lm, _ = loss(orc.RBM.from_vector(vm, N, M))
            fd.append((Lp - Lm) / (2 * h))
        return complex(fd[0], fd[1])

    for k in range(fit.P):
        scale = max(1.0, abs(g[k]))
        # h = 1e-3: truncation error O(h^2) relative to the third derivative
        assert abs(central(k, 1e-3) - g[k]) < 1e-4 * scale, k
        # Richardson extrapolation of h and h/2 removes the h^2 term
        d1, d2 = central(k, 1e-3), central(k, 5e-4)
        assert abs((4 * d2 - d1) / 3 - g[k]) < 1e-8 * scale, k
    h = 1e-4
    # random directions
    for _ in range(4):
        dvec = r.normal(size=fit.P) + 1j * r.normal(size=fit.P)
        dvec /= np.linalg.norm(dvec)
        Lp, _ = loss(orc.RBM.from_vector(v0 + h * dvec, N, M))
        Lm, _ = loss(orc.RBM.from_vector(v0 - h * dvec, N, M))
        dd = (Lp - Lm) / (2 * h)
        assert abs(dd - np.sum((g.conj() * dvec).real)) < 1e-6 * max(1.0, np.abs(g).max())


def test_fidelity_grad_entries_match_the_full_gradient(orc):
    """The entry-by-entry gradient (for models whose O does not fit in memory) equals the full one on
    scrambled and repeated indices of all three parameter kinds."""
    N, M = 7, 5
    lat = orc.Lattice(0, N)
    fit = orc.RBM(*synth.random_rbm_arrays(70, N, M, 0.3))
    psn = orc.RBM(*synth.random_rbm_arrays(71, N, M, 0.3))
    psm = orc.RBM(*synth.random_rbm_arrays(72, N, M, 0.3))
    sig = synth.random_spins(73, 200, N, False)
    R = orc.target_ratio(fit, psn, psm, lat, sig, 2, -1.3, 2.5, 0.9, 1.1)
    L, g = orc.fidelity_grad(fit, sig, R)
    ks = np.array([46, 0, 6, 7, 11, 12, 30, 7, 3], np.int64)            # P = 7 + 5 + 35 = 47
    Le, ge = orc.fidelity_grad_entries(fit, sig, R, ks)
    assert abs(Le - L) < 1e-14 * max(1.0, L)
    assert np.max(np.abs(ge - g[ks])) < 1e-13 * max(1.0, np.abs(g).max())
