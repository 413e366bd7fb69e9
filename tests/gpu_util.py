"""Helpers for the GPU parity tests: moving RBMs between the oracle and the device."""
import numpy as np
import torch

import paper_2103_08804_amd as crbm


def to_device_rbm(orc_rbm):
    """complex64 device copy of an oracle RBM (parameters rounded to binary32)."""
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.complex64)).cuda()
    return crbm.RBM(t(orc_rbm.a), t(orc_rbm.b), t(orc_rbm.W))


def to_oracle_rbm(orc, dev_rbm):
    """The exact binary32 parameters of a device RBM, widened to double for the oracle."""
    n = lambda x: x.detach().cpu().numpy().astype(np.complex128)
    return orc.RBM(n(dev_rbm.a), n(dev_rbm.b), n(dev_rbm.W))


def np_of(t):
    return t.detach().cpu().numpy()


def wrapped(d):
    return np.angle(np.exp(1j * d))


def rel_err(got, want, floor=1e-30):
    got, want = np.asarray(got), np.asarray(want)
    return np.max(np.abs(got - want)) / max(np.max(np.abs(want)), floor)


EPS32 = 2.0 ** -24


def logpsi_rounding_bound(rbm, sig, c=16.0):
    """First-order bound on the FP32 error of log psi caused by rounding theta:
    |d log psi| <= sum_k |tanh theta_k| |d theta_k|, |d theta_k| <= c eps (|b_k| + sum_i |W_ik|).
    Large where theta_k approaches a zero of cosh (the amplitude itself nearly vanishes).
    c = 16 for N <= 16 sites: theta = b + sigma W comes from three v_mfma_f32_32x32x16_bf16 products
    (the exact BF16 parts of W), each adding a 16-term dot product to the FP32 accumulator, so at most
    1 + log2(16) = 5 roundings per part (the dot product's pairwise levels and the accumulation),
    15 for the three parts, and one more for b."""
    sig = np.asarray(sig, np.float64)
    th = rbm.b[None, :] + sig @ rbm.W
    scale = np.abs(rbm.b) + np.abs(rbm.W).sum(axis=0)
    return c * EPS32 * (np.abs(np.tanh(th)) * scale[None, :]).sum(axis=1) + c * EPS32 * np.abs(rbm.a).sum()


def eloc_rounding_bound(rbm, bonds, sig, J=1.0):
    """Bound on the FP32 error of E_loc propagated from the log-amplitude bounds of sigma and of each
    bond-swapped configuration: (J/2) sum_b |rho_b| (bound(sigma^b) + bound(sigma))."""
    sig = np.asarray(sig, np.int8)
    base = logpsi_rounding_bound(rbm, sig)
    th = rbm.b[None, :] + sig.astype(np.float64) @ rbm.W
    lc = lambda z: np.log(2 * np.cosh(z))
    lp0 = sig.astype(np.float64) @ rbm.a + lc(th).sum(axis=1)
    out = np.zeros(sig.shape[0])
    for (i, j) in bonds:
        anti = sig[:, i] != sig[:, j]
        if not anti.any():
            continue
        s2 = sig[anti].copy()
        s2[:, [i, j]] = s2[:, [j, i]]
        th2 = rbm.b[None, :] + s2.astype(np.float64) @ rbm.W
        lp2 = s2.astype(np.float64) @ rbm.a + lc(th2).sum(axis=1)
        rho = np.abs(np.exp(lp2 - lp0[anti]))
        out[anti] += 0.5 * J * rho * (logpsi_rounding_bound(rbm, s2) + base[anti])
    return out


def log_amp_scale(rbm, sig):
    """max over the rows of sig of sum_j |theta_j| + |a . sigma|: the size of the terms whose binary32
    sums make log psi (theta = b + sigma W)."""
    s = np.asarray(sig, np.float64)
    th = rbm.b[None, :] + s @ rbm.W
    return float(np.max(np.abs(th).sum(axis=1) + np.abs(s @ rbm.a)))


def lattice_images(sig, Lx, Ly, rotations):
    """Every translation (and, with rotations, every rotation by a multiple of pi/2) of each row of sig
    on the Lx x Ly torus, stacked: the configurations the symmetry projection evaluates."""
    g = np.asarray(sig).reshape(-1, Ly, Lx)
    out = []
    for r in range(4 if rotations else 1):
        gr = np.rot90(g, r, axes=(1, 2))
        for dy in range(Ly):
            for dx in range(Lx):
                out.append(np.roll(np.roll(gr, dy, axis=1), dx, axis=2).reshape(g.shape[0], -1))
    return np.concatenate(out)


def ratio_gram_tol(L_states, L_gs, floor=1e-5):
    """Tolerance of G and H (relative to their largest entry) for basis ratios r = t / psi_gs formed from
    binary32 log amplitudes.  Each log psi is a binary32 tree sum of depth at most 8 (two units per lane,
    six lane levels, the log of the product factor) of terms of total size L, so |d log psi| <= 8 u L
    (u = 2^-24); a ratio carries two of them and a Gram entry <r_k^* r_k'> two ratios, and by
    Cauchy-Schwarz |<r_k^* r_k'>| <= max|G|: 16 u (L_t + L_gs), L_t the largest over the states."""
    return max(floor, 16.0 * EPS32 * (L_states + L_gs))
