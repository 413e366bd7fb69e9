"""Pins for the oracle's Metropolis sampler (Sec. III: s ~ |psi_s|^2 / <psi|psi>).

* the empirical distribution of thinned samples matches the exact Born
  weights (total-variation distance and a chi-square test on well-populated
  configurations), for single flips over all 2^N configurations and for pair
  exchanges within the S^z = 0 sector;
* all-zero parameters accept every non-null proposal;
* replaying the sampler's own decisions reproduces the trajectory with no
  mismatch, while a decision stream with planted disagreements is flagged.
"""
import numpy as np
from scipy import stats

import synth




def _histogram_test(orc, rbm, N, proposal, C, sweeps, burn, thin):
    spins = orc.init_chains(N, C, 77, 1 if proposal == 1 else 0)
    samples, nacc, _, _ = orc.metropolis(rbm, spins, sweeps, proposal, seed=123)
    keep = samples[burn::thin].reshape(-1, N)
    idx = ((keep > 0).astype(np.int64) << np.arange(N)).sum(axis=1)
    counts = np.bincount(idx, minlength=1 << N)
    sig = orc.enumerate_configs(N)
    lp = orc.logpsi(rbm, sig)
    if proposal == 1:
        mask = sig.sum(axis=1) == 0
        lp = np.where(mask, lp, -np.inf + 0j)
        lp[~mask] = -1e300
    p = orc.enum_weights(lp)
    if proposal == 1:
        p[~mask] = 0.0
        p /= p.sum()
    emp = counts / counts.sum()
    tv = 0.5 * np.abs(emp - p).sum()
    return tv, counts, p


def test_single_flip_distribution(orc):
    N, M = 6, 4
    rbm = orc.RBM(*synth.random_rbm_arrays(12, N, M, 0.5))
    tv, counts, p = _histogram_test(orc, rbm, N, 0, C=512, sweeps=120, burn=20, thin=4)
    assert tv < 0.03, tv
    exp = p * counts.sum()
    sel = exp > 20
    chi2 = np.sum((counts[sel] - exp[sel]) ** 2 / exp[sel])
    # thinned samples are nearly independent; allow a generous inflation factor
    assert stats.chi2.sf(chi2 / 2.0, sel.sum() - 1) > 1e-4, chi2


def test_pair_exchange_distribution(orc):
    N, M = 8, 5
    rbm = orc.RBM(*synth.random_rbm_arrays(13, N, M, 0.5))
    tv, counts, p = _histogram_test(orc, rbm, N, 1, C=512, sweeps=120, burn=20, thin=4)
    assert tv < 0.04, tv
    # pair exchanges conserve total S^z
    assert counts[p == 0].sum() == 0


def test_zero_parameters_accept_everything(orc):
    N = 10
    rbm = orc.RBM(np.zeros(N), np.zeros(3), np.zeros((N, 3)))
    spins = orc.init_chains(N, 8, 1, 0)
    _, nacc, _, _ = orc.metropolis(rbm, spins, 5, 0, seed=9)
    assert np.all(nacc == 5 * N)


def test_replay_flags_planted_disagreement(orc):
    N, M = 8, 4
    rbm = orc.RBM(*synth.random_rbm_arrays(14, N, M, 0.6))
    s0 = orc.init_chains(N, 4, 3, 1)
    sweeps = 6
    words = (sweeps * N + 31) // 32
    # an all-reject decision stream: every proposal the oracle accepts with a
    # clear margin becomes a flagged mismatch, and the replay stays frozen
    trace = np.zeros((4, words), np.uint32)
    s = s0.copy()
    samples, nacc, amb, mis = orc.metropolis(rbm, s, sweeps, 1, seed=5, trace=trace)
    assert mis > 0
    assert np.all(nacc == 0)
    assert np.array_equal(s, s0)
    # a stream that agrees with the oracle everywhere (all-accept at zero
    # parameters, where every ratio is exactly 1 and u < 1) shows no mismatch
    z = orc.RBM(np.zeros(N), np.zeros(M), np.zeros((N, M)))
    s = s0.copy()
    ones = np.full((4, words), 0xFFFFFFFF, np.uint32)
    _, nacc, amb, mis = orc.metropolis(z, s, sweeps, 0, seed=5, trace=ones)
    assert mis == 0 and amb == 0


def test_chain_ids_select_the_stream(orc):
    """Rows run under explicit chain indices reproduce those chains of a run over all of them, so a
    few chains of a large launch can be replayed alone."""
    N, M, C = 12, 6, 40
    rbm = orc.RBM(*synth.random_rbm_arrays(5, N, M, 0.3, std_im=0.05))
    spins = orc.init_chains(N, C, 91, 1)
    start = spins.copy()
    smp, nacc, _, _ = orc.metropolis(rbm, spins, 7, 1, seed=17, step_offset=300)
    ids = np.array([0, 13, 39], np.int32)
    sub = np.ascontiguousarray(start[ids])
    smp_sub, nacc_sub, _, _ = orc.metropolis(rbm, sub, 7, 1, seed=17, step_offset=300, chain_ids=ids)
    assert np.array_equal(smp_sub, smp[:, ids])
    assert np.array_equal(nacc_sub, nacc[ids])
    assert np.array_equal(sub, spins[ids])
    # the same rows under the default indices 0, 1, 2 follow other streams
    sub2 = np.ascontiguousarray(start[ids])
    smp_def, _, _, _ = orc.metropolis(rbm, sub2, 7, 1, seed=17, step_offset=300)
    assert not np.array_equal(smp_def[:, 1:], smp[:, ids[1:]])
