"""Pins for the natural-gradient step (Sec. III).

* In enumeration mode the shifted system (S + eps I) dalpha = F is the normal
  equation of the weighted ridge least-squares problem
      min_x sum_s p_s |sum_k x_k (O_k(s) - <O_k>) - D(s)|^2 + eps |x|^2,
  D = dgamma gamma cot(gamma) (R/<R> - 1), so numpy's lstsq on the stacked
  system must reproduce dalpha (pins S, F, the solve and the update).
* The rotation has norm <|D|^2> = (dgamma gamma)^2 (the paper's
  <dpsi|dpsi> = (dgamma gamma)^2 <psi|psi>), which pins gamma and gamma cot gamma.
* R identically equal to a constant c gives gamma = 0, beta = c, F = 0.
* S equals the weighted covariance computed by numpy, is Hermitian and PSD.
"""
import numpy as np

import synth


def _setup(orc, N=6, M=6, seed=5):
    rbm = orc.RBM(*synth.random_rbm_arrays(seed, N, M, 0.3))
    sig = orc.enumerate_configs(N)
    p = orc.enum_weights(orc.logpsi(rbm, sig))
    r = np.random.default_rng(seed + 1)
    R = 1.0 + 0.4 * r.normal(size=sig.shape[0]) + 0.3j * r.normal(size=sig.shape[0])
    return rbm, sig, p, R


def test_sr_step_is_ridge_least_squares(orc):
    rbm, sig, p, R = _setup(orc)
    dgamma, eps = 0.1, 1e-3
    new, info = orc.sr_step(rbm, sig, R, dgamma, eps, weights=p, want_S=True)
    assert info["rc"] == 0
    O = orc.logderiv(rbm, sig)
    Ot = O - p @ O
    Rm = np.sum(p * R)
    gamma = np.arccos(min(1.0, abs(Rm) / np.sqrt(np.sum(p * abs(R) ** 2))))
    D = dgamma * gamma / np.tan(gamma) * (R / Rm - 1.0)
    A = np.vstack([np.sqrt(p)[:, None] * Ot, np.sqrt(eps) * np.eye(rbm.P)])
    y = np.concatenate([np.sqrt(p) * D, np.zeros(rbm.P)])
    x, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert np.allclose(info["dalpha"], x, rtol=1e-8, atol=1e-10)
    assert np.allclose(new.vector(), rbm.vector() + x, rtol=1e-8, atol=1e-10)
    # beta = <R>
    assert abs(info["beta"] - Rm) < 1e-13
    # rotation norm identity
    assert abs(np.sum(p * abs(D) ** 2) - (dgamma * info["gamma"]) ** 2) < 1e-12


def test_sr_covariance_matches_numpy(orc):
    rbm, sig, p, R = _setup(orc, N=5, M=4, seed=9)
    _, info = orc.sr_step(rbm, sig, R, 0.1, 1e-3, weights=p, want_S=True)
    O = orc.logderiv(rbm, sig)
    C = np.cov(O.T, aweights=p, bias=True)       # C_kk' = <(O_k-<O_k>)(O_k'-<O_k'>)^*>
    S = info["S"]
    assert np.allclose(S, C.T, rtol=1e-10, atol=1e-12)
    assert np.allclose(S, S.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(S).min() > -1e-12


def test_sr_constant_ratio(orc):
    rbm, sig, p, _ = _setup(orc, N=6, M=3, seed=2)
    c = 0.7 - 0.2j
    R = np.full(sig.shape[0], c)
    new, info = orc.sr_step(rbm, sig, R, 0.1, 1e-3, weights=p)
    assert info["gamma"] < 1e-7
    assert abs(info["beta"] - c) < 1e-13
    assert info["Fnorm"] < 1e-12
    assert np.allclose(new.vector(), rbm.vector(), atol=1e-12)


def test_sr_uniform_weights_equal_explicit(orc):
    rbm, _, _, _ = _setup(orc, N=6, M=3, seed=4)
    sig = synth.random_spins(8, 200, 6, True)
    r = np.random.default_rng(3)
    R = 1 + 0.2 * r.normal(size=200) + 0.1j * r.normal(size=200)
    n1, i1 = orc.sr_step(rbm, sig, R, 0.2, 1e-2)
    n2, i2 = orc.sr_step(rbm, sig, R, 0.2, 1e-2, weights=np.full(200, 1 / 200))
    assert np.allclose(i1["dalpha"], i2["dalpha"], rtol=1e-12, atol=1e-14)


def test_sr_entries_match_the_full_step(orc):
    """The entry-by-entry form (for models too large for the full O) equals the full step's S, F,
    gamma and beta on the chosen indices: weighted (enumeration) and uniform (MC) sums, indices of
    all three parameter kinds in scrambled order and repeated."""
    rbm, sig, p, R = _setup(orc, N=7, M=5, seed=9)
    ks = np.array([34, 0, 6, 7, 11, 12, 13, 40, 20, 7, 3], np.int64)      # P = 7 + 5 + 35 = 47
    for w in (p, None):
        _, info = orc.sr_step(rbm, sig, R, 0.2, 1e-3, weights=w, want_S=True)
        e = orc.sr_entries(rbm, sig, R, 0.2, ks, weights=w)
        assert np.max(np.abs(e["S"] - info["S"][np.ix_(ks, ks)])) < 1e-13
        assert np.max(np.abs(e["F"] - info["F"][ks])) < 1e-13
        assert abs(e["gamma"] - info["gamma"]) < 1e-14 and abs(e["beta"] - info["beta"]) < 1e-14
        O = orc.logderiv(rbm, sig)
        wt = np.full(sig.shape[0], 1.0 / sig.shape[0]) if w is None else w
        assert np.max(np.abs(e["Om"] - wt @ O[:, ks])) < 1e-13


def test_sr_diagonal_matches_the_full_step(orc):
    """The diagonal-only form equals the full step's diagonal of S and the means of O, weighted and
    uniform, including a model whose b puts |<tanh theta>| far above its spread (the diagonal of the b
    rows is then small against |<O>|^2)."""
    rbm, sig, p, R = _setup(orc, N=7, M=5, seed=9)
    biased = orc.RBM(rbm.a, rbm.b + 2.5, rbm.W)
    for model in (rbm, biased):
        for w in (p, None):
            _, info = orc.sr_step(model, sig, R, 0.2, 1e-3, weights=w, want_S=True)
            d, Om = orc.sr_diagonal(model, sig, weights=w)
            assert np.max(np.abs(d - np.real(np.diag(info["S"])))) < 1e-13
            O = orc.logderiv(model, sig)
            wt = np.full(sig.shape[0], 1.0 / sig.shape[0]) if w is None else w
            assert np.max(np.abs(Om - wt @ O)) < 1e-13
            assert np.all(d >= -1e-15)
    # the biased b rows: spread of tanh far below its mean
    d, Om = orc.sr_diagonal(biased, sig)
    assert np.all(d[7:12] < 0.05 * np.abs(Om[7:12]) ** 2)
