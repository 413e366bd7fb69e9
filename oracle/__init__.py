"""FP64 CPU oracle for the Chebyshev-RBM hot path (arXiv:2103.08804).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the GPU library or its
Python binding.  It shares no code with the HIP path.

The numerics live in ``oracle.c`` (plain C, double precision, every quantity
from its definition).  This module only marshals numpy arrays into it.
``exact`` holds the exact-vector references (Heisenberg matrix over all 2^N
configurations, exact Chebyshev recursion); ``spectral`` the FP64 post-processing
of moments (Jackson reconstruction, moment correction, continued-fraction spectrum).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c = ctypes
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _ChebArgs(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("E_c", ctypes.c_double), ("W_scale", ctypes.c_double),
                ("beta_n", ctypes.c_double * 2), ("beta_nm1", ctypes.c_double * 2),
                ("q", ctypes.c_double * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_init_rbm.argtypes = [_c.c_int, _c.c_int, _c.c_uint64, _c.c_double, _c128p, _c128p, _c128p]
        L.orc_init_chains.argtypes = [_c.c_int, _c.c_int, _c.c_uint64, _c.c_int, _i8p]
        L.orc_lattice_bonds.argtypes = [_c.c_int, _c.c_int, _c.c_int, _i32p]
        L.orc_lattice_bonds.restype = _c.c_int
        L.orc_logpsi.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _i8p, _c.c_long, _c128p]
        L.orc_enumerate.argtypes = [_c.c_int, _i8p]
        L.orc_enum_weights.argtypes = [_c.c_long, _c128p, _f64p]
        L.orc_fq.argtypes = [_c.c_int, _c.c_int, _c.c_int, _f64p, _i8p, _c.c_long, _c128p]
        L.orc_local_energy.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _c.c_int, _c.c_int,
                                       _c.c_int, _c.c_double, _i8p, _c.c_long, _c128p]
        L.orc_logderiv.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _i8p, _c.c_long, _c128p]
        L.orc_target_ratio.argtypes = [_c.c_int, _c.c_int] + [_c.c_void_p] * 9 + [
            _c.POINTER(_ChebArgs), _c.c_int, _c.c_int, _c.c_int, _c.c_double, _i8p, _c.c_long,
            _c128p, _c.c_void_p]
        L.orc_metropolis.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _i8p, _c.c_int, _c.c_int,
                                     _c.c_int, _c.c_uint64, _c.c_uint64, _c.c_void_p, _c.c_void_p,
                                     _c.c_void_p, _c.c_long, _c.c_double,
                                     _c.POINTER(_c.c_long), _c.POINTER(_c.c_long), _c.c_void_p]
        L.orc_sr_entries.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _i8p, _c.c_void_p, _c128p, _c.c_long,
                                     _c.c_double, _c.c_void_p, _c.c_int, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                     _c.c_void_p]
        L.orc_sr_diagonal.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _i8p, _c.c_void_p, _c.c_long,
                                      _f64p, _c128p]
        L.orc_sr_diagonal.restype = None
        L.orc_sr_step.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _i8p, _c.c_void_p, _c128p,
                                  _c.c_long, _c.c_double, _c.c_double, _f64p, _c.c_void_p, _c.c_void_p,
                                  _c.c_void_p]
        L.orc_sr_step.restype = _c.c_int
        L.orc_moments.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _c128p, _c128p, _c.c_int,
                                  _f64p, _c.c_int, _c.c_int, _c.c_int, _i8p, _c.c_void_p, _c.c_long,
                                  _c128p]
        L.orc_moment_matrices.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _c128p, _c128p, _c.c_int,
                                          _f64p, _c.c_int, _c.c_int, _c.c_int, _c.c_double, _i8p, _c.c_void_p,
                                          _c.c_long, _c128p, _c128p]
        L.orc_moment_matrices.restype = None
        L.orc_sym_matrices.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _c128p, _c128p, _c.c_int,
                                       _c.c_int, _c.c_int, _c.c_int, _c.c_double, _c.c_int, _i8p, _c.c_void_p,
                                       _c.c_long, _c128p, _c128p]
        L.orc_sym_matrices.restype = None
        L.orc_fidelity_grad.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _i8p, _c128p, _c.c_long,
                                        _c.c_void_p]
        L.orc_fidelity_grad.restype = _c.c_double
        L.orc_fidelity_grad_entries.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _i8p, _c128p, _c.c_long,
                                                _c.c_void_p, _c.c_int, _c.c_void_p]
        L.orc_fidelity_grad_entries.restype = _c.c_double
        L.orc_sr_energy_step.argtypes = L.orc_sr_step.argtypes
        L.orc_sr_energy_step.restype = _c.c_int
        _i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        L.orc_batched_moments.argtypes = [_c.c_int, _c.c_int, _c128p, _c128p, _c128p, _c128p, _c128p, _f64p, _i64p,
                                          _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_uint64, _c.c_int, _c.c_int,
                                          _c.c_double, _c128p, _c.POINTER(_c.c_long), _c.c_void_p, _c.c_long,
                                          _c.POINTER(_c.c_long)]
        _lib = L
    return _lib


# --------------------------------------------------------------------------- helpers
def _c128(x):
    return np.ascontiguousarray(x, dtype=np.complex128)


def _i8(x):
    return np.ascontiguousarray(x, dtype=np.int8)


def _ptr(x):
    return None if x is None else x.ctypes.data_as(ctypes.c_void_p)


class RBM:
    """Complex RBM parameters a[N], b[M], W[N][M] (complex128 on the oracle side)."""

    def __init__(self, a, b, W):
        self.a = _c128(a)
        self.b = _c128(b)
        self.W = _c128(W)

    @property
    def N(self):
        return self.a.shape[0]

    @property
    def M(self):
        return self.b.shape[0]

    @property
    def P(self):
        return self.N + self.M + self.N * self.M

    def vector(self):
        return np.concatenate([self.a, self.b, self.W.ravel()])

    @classmethod
    def from_vector(cls, v, N, M):
        v = _c128(v)
        return cls(v[:N], v[N:N + M], v[N + M:].reshape(N, M))

    def copy(self):
        return RBM(self.a.copy(), self.b.copy(), self.W.copy())


class Lattice:
    """kind 0: periodic chain of Lx sites; kind 1: periodic Lx x Ly square lattice."""

    def __init__(self, kind, Lx, Ly=1, J=1.0):
        self.kind, self.Lx, self.Ly, self.J = int(kind), int(Lx), int(Ly if kind == 1 else 1), float(J)

    @property
    def N(self):
        return self.Lx * self.Ly

    def bonds(self):
        out = np.zeros(4 * self.N, dtype=np.int32)
        nb = lib().orc_lattice_bonds(self.kind, self.Lx, self.Ly, out)
        return out[:2 * nb].reshape(nb, 2)


# --------------------------------------------------------------------------- wrappers
def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def init_rbm(N, M, seed, stddev):
    a = np.zeros(N, np.complex128)
    b = np.zeros(M, np.complex128)
    W = np.zeros((N, M), np.complex128)
    lib().orc_init_rbm(N, M, seed, stddev, a, b, W)
    return RBM(a, b, W)


def init_chains(N, C, seed, mode):
    s = np.zeros((C, N), np.int8)
    lib().orc_init_chains(N, C, seed, mode, s)
    return s


def enumerate_configs(N):
    s = np.zeros((1 << N, N), np.int8)
    lib().orc_enumerate(N, s)
    return s


def logpsi(rbm, sig):
    sig = _i8(sig)
    out = np.zeros(sig.shape[0], np.complex128)
    lib().orc_logpsi(rbm.N, rbm.M, rbm.a, rbm.b, rbm.W, sig, sig.shape[0], out)
    return out


def enum_weights(lp):
    lp = _c128(lp)
    p = np.zeros(lp.shape[0], np.float64)
    lib().orc_enum_weights(lp.shape[0], lp, p)
    return p


def fq(lat, q, sig):
    sig = _i8(sig)
    out = np.zeros(sig.shape[0], np.complex128)
    lib().orc_fq(lat.kind, lat.Lx, lat.N, np.asarray(q, np.float64), sig, sig.shape[0], out)
    return out


def local_energy(rbm, lat, sig):
    sig = _i8(sig)
    out = np.zeros(sig.shape[0], np.complex128)
    lib().orc_local_energy(rbm.N, rbm.M, rbm.a, rbm.b, rbm.W, lat.kind, lat.Lx, lat.Ly, lat.J, sig,
                           sig.shape[0], out)
    return out


def logderiv(rbm, sig):
    sig = _i8(sig)
    out = np.zeros((sig.shape[0], rbm.P), np.complex128)
    lib().orc_logderiv(rbm.N, rbm.M, rbm.b, rbm.W, sig, sig.shape[0], out)
    return out


def target_ratio(fit, psi_n, psi_nm1, lat, sig, order, E_c, W_scale, beta_n=1.0, beta_nm1=1.0,
                 q=(0.0, 0.0), return_hpsi=False):
    """R(sigma) = phi(sigma) / psi_{n+1}(sigma) for the Chebyshev target of the given order."""
    sig = _i8(sig)
    ch = _ChebArgs()
    ch.order, ch.E_c, ch.W_scale = int(order), float(E_c), float(W_scale)
    bn, bm = complex(beta_n), complex(beta_nm1)
    ch.beta_n[0], ch.beta_n[1] = bn.real, bn.imag
    ch.beta_nm1[0], ch.beta_nm1[1] = bm.real, bm.imag
    ch.q[0], ch.q[1] = float(q[0]), float(q[1])
    R = np.zeros(sig.shape[0], np.complex128)
    hp = np.zeros(sig.shape[0], np.complex128)
    pm = psi_nm1
    args = [fit.a, fit.b, fit.W, psi_n.a, psi_n.b, psi_n.W]
    args += [pm.a, pm.b, pm.W] if pm is not None else [None, None, None]
    lib().orc_target_ratio(fit.N, fit.M, *[_ptr(x) for x in args], ctypes.byref(ch), lat.kind, lat.Lx,
                           lat.Ly, lat.J, sig, sig.shape[0], R, _ptr(hp))
    return (R, hp) if return_hpsi else R


def metropolis(rbm, spins, n_sweeps, proposal, seed, step_offset=0, trace=None, margin=1e-4, chain_ids=None):
    """Run the Metropolis chains in place on ``spins`` [C][N].

    Returns (samples [n_sweeps][C][N], n_accept [C], n_ambiguous, n_mismatch).
    ``trace`` ([C][words] uint32) replays another implementation's decisions.
    ``chain_ids`` ([C] int) gives the chain index of each row (its random stream); default 0 .. C-1.
    """
    C, N = spins.shape
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    samples = np.zeros((n_sweeps, C, N), np.int8)
    nacc = np.zeros(C, np.uint32)
    amb, mis = ctypes.c_long(0), ctypes.c_long(0)
    words = 0
    if trace is not None:
        trace = np.ascontiguousarray(trace, dtype=np.uint32)
        words = trace.shape[1]
    ids = None
    if chain_ids is not None:
        ids = np.ascontiguousarray(chain_ids, dtype=np.int32)
        assert ids.shape == (C,)
    lib().orc_metropolis(N, rbm.M, rbm.a, rbm.b, rbm.W, spins, C, n_sweeps, proposal, seed, step_offset,
                         _ptr(samples), _ptr(nacc), _ptr(trace), words, margin, ctypes.byref(amb),
                         ctypes.byref(mis), _ptr(ids))
    return samples, nacc, amb.value, mis.value


def sr_step(rbm, sig, R, dgamma, eps, weights=None, want_S=False):
    """One natural-gradient step; updates a copy of ``rbm`` and returns (new_rbm, info)."""
    sig = _i8(sig)
    R = _c128(R)
    n = sig.shape[0]
    new = rbm.copy()
    stats = np.zeros(4, np.float64)
    S = np.zeros((rbm.P, rbm.P), np.complex128) if want_S else None
    F = np.zeros(rbm.P, np.complex128)
    dx = np.zeros(rbm.P, np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    rc = lib().orc_sr_step(rbm.N, rbm.M, new.a, new.b, new.W, sig, _ptr(w), R, n, dgamma, eps, stats,
                           _ptr(S), _ptr(F), _ptr(dx))
    info = dict(rc=rc, gamma=stats[0], beta=complex(stats[1], stats[2]), Fnorm=stats[3], F=F, dalpha=dx, S=S)
    return new, info


def sr_entries(rbm, sig, R, dgamma, ks, weights=None):
    """S and F of the natural-gradient step restricted to the parameter indices ``ks``, with <O_k>,
    gamma and beta: dict(S [len(ks)][len(ks)], F [len(ks)], Om [len(ks)], gamma, beta).  Each O_k(s)
    is formed per sample, so the model may be too large for the full O."""
    sig = _i8(sig)
    R = _c128(R)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    nk = ks.shape[0]
    S = np.zeros((nk, nk), np.complex128)
    F = np.zeros(nk, np.complex128)
    Om = np.zeros(nk, np.complex128)
    stats = np.zeros(3, np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    lib().orc_sr_entries(rbm.N, rbm.M, rbm.b, rbm.W, sig, _ptr(w), R, sig.shape[0], dgamma, _ptr(ks), nk,
                         _ptr(stats), _ptr(S), _ptr(F), _ptr(Om))
    return dict(S=S, F=F, Om=Om, gamma=stats[0], beta=complex(stats[1], stats[2]))


def sr_diagonal(rbm, sig, weights=None):
    """(S_kk for every parameter k, <O_k>) over the samples, without forming O [n][P]."""
    sig = _i8(sig)
    S = np.zeros(rbm.P, np.float64)
    Om = np.zeros(rbm.P, np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    lib().orc_sr_diagonal(rbm.N, rbm.M, rbm.b, rbm.W, sig, _ptr(w), sig.shape[0], S, Om)
    return S, Om


def sr_energy_step(rbm, sig, eloc, lr, eps, weights=None, want_S=False):
    """One ground-state natural-gradient step; returns (new_rbm, info) with info['E'], info['var']."""
    sig = _i8(sig)
    E = _c128(eloc)
    n = sig.shape[0]
    new = rbm.copy()
    stats = np.zeros(4, np.float64)
    S = np.zeros((rbm.P, rbm.P), np.complex128) if want_S else None
    F = np.zeros(rbm.P, np.complex128)
    dx = np.zeros(rbm.P, np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    rc = lib().orc_sr_energy_step(rbm.N, rbm.M, new.a, new.b, new.W, sig, _ptr(w), E, n, lr, eps, stats,
                                  _ptr(S), _ptr(F), _ptr(dx))
    info = dict(rc=rc, E=complex(stats[0], stats[1]), var=stats[2], Fnorm=stats[3], F=F, dalpha=dx, S=S)
    return new, info


def moments(psi_gs, ts, betas, qs, lat, sig, weights=None):
    """mu[q][n], n = 0 .. len(ts), per the Chebyshev-moment definition."""
    sig = _i8(sig)
    n_max = len(ts)
    tp = np.concatenate([t.vector() for t in ts]) if n_max else np.zeros(1, np.complex128)
    qs = np.ascontiguousarray(np.asarray(qs, np.float64).reshape(-1, 2))
    mu = np.zeros((qs.shape[0], n_max + 1), np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    lib().orc_moments(psi_gs.N, psi_gs.M, psi_gs.a, psi_gs.b, psi_gs.W, _c128(tp),
                      _c128(np.asarray(betas, np.complex128).reshape(-1) if n_max else np.zeros(1)),
                      n_max, qs, qs.shape[0], lat.kind, lat.Lx, sig, _ptr(w), sig.shape[0], mu)
    return mu


def moment_matrices(psi_gs, ts, betas, q, lat, sig, weights=None):
    """(G, H), K x K with K = len(ts) + 1: G_nm = <conj(B_n) B_m>, H_nm = <conj(B_n) (H t_m)/psi_gs>."""
    sig = _i8(sig)
    n_max = len(ts)
    K = n_max + 1
    tp = np.concatenate([t.vector() for t in ts]) if n_max else np.zeros(1, np.complex128)
    G = np.zeros((K, K), np.complex128)
    H = np.zeros((K, K), np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    lib().orc_moment_matrices(psi_gs.N, psi_gs.M, psi_gs.a, psi_gs.b, psi_gs.W, _c128(tp),
                              _c128(np.asarray(betas, np.complex128).reshape(-1) if n_max else np.zeros(1)),
                              n_max, np.ascontiguousarray(np.asarray(q, np.float64).reshape(2)), lat.kind, lat.Lx,
                              lat.Ly, lat.J, sig, _ptr(w), sig.shape[0], G, H)
    return G, H


def sym_matrices(psi_gs, ts, betas, lat, sig, rotations=True, weights=None):
    """(G, H), each [N][K][K] over the N lattice momenta k = k1 + Lx k2, of the symmetry-projected
    basis of App. A (t_000 = S^z_0 psi_gs, t_n00 = beta_n t~_n)."""
    sig = _i8(sig)
    n_max = len(ts)
    K = n_max + 1
    N = lat.N
    tp = np.concatenate([t.vector() for t in ts]) if n_max else np.zeros(1, np.complex128)
    G = np.zeros((N, K, K), np.complex128)
    H = np.zeros((N, K, K), np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, np.float64)
    lib().orc_sym_matrices(psi_gs.N, psi_gs.M, psi_gs.a, psi_gs.b, psi_gs.W, _c128(tp),
                           _c128(np.asarray(betas, np.complex128).reshape(-1) if n_max else np.zeros(1)),
                           n_max, lat.kind, lat.Lx, lat.Ly, lat.J, int(bool(rotations)), sig, _ptr(w),
                           sig.shape[0], G, H)
    return G, H


def fidelity_grad(rbm, sig, R):
    """(L, grad) with grad = dL/dRe(alpha) + i dL/dIm(alpha) on frozen samples."""
    sig = _i8(sig)
    R = _c128(R)
    g = np.zeros(rbm.P, np.complex128)
    L = lib().orc_fidelity_grad(rbm.N, rbm.M, rbm.b, rbm.W, sig, R, sig.shape[0], _ptr(g))
    return L, g


def fidelity_grad_entries(rbm, sig, R, ks):
    """(L, grad[ks]): the fidelity gradient on the parameter indices ``ks`` only, each O_k(s) formed
    per sample (for models whose O does not fit in memory)."""
    sig = _i8(sig)
    R = _c128(R)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    g = np.zeros(ks.shape[0], np.complex128)
    L = lib().orc_fidelity_grad_entries(rbm.N, rbm.M, rbm.b, rbm.W, sig, R, sig.shape[0], _ptr(ks), ks.shape[0],
                                        _ptr(g))
    return L, g


def batched_moments(psi_gs, t_params, betas, qs, offsets, lat, n_burn, n_sweeps, proposal, seed, margin=1e-4,
                    trace=None):
    """Per-instance (<|f_q|^2>, <conj(f_q) beta t~/psi_gs>), with (n_ambiguous, n_mismatch).

    ``offsets`` holds the global chain indices of the instances (chain g's random stream is g).
    Without ``trace``, n_ambiguous counts the steps within the margin of the threshold and n_mismatch
    is 0.  With ``trace`` (uint32 [offsets[-1] - offsets[0]][words], row g - offsets[0]) the chains
    replay another implementation's decisions as in metropolis()."""
    t_params = _c128(np.asarray(t_params).reshape(len(betas), -1))
    out = np.zeros((len(betas), 2), np.complex128)
    amb, mis = ctypes.c_long(0), ctypes.c_long(0)
    words = 0
    if trace is not None:
        trace = np.ascontiguousarray(trace, dtype=np.uint32)
        words = trace.shape[1]
    lib().orc_batched_moments(psi_gs.N, psi_gs.M, psi_gs.a, psi_gs.b, psi_gs.W, t_params, _c128(betas),
                              np.ascontiguousarray(np.asarray(qs, np.float64).reshape(-1, 2)),
                              np.ascontiguousarray(offsets, np.int64), len(betas), n_burn, n_sweeps, proposal, seed,
                              lat.kind, lat.Lx, margin, out, ctypes.byref(amb), _ptr(trace), words,
                              ctypes.byref(mis))
    return out, amb.value, mis.value
