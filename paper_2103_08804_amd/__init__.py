"""Python binding of libchebrbm (the gfx950 Chebyshev-RBM hot path).

Argument marshalling only: every function checks dtype / device / shape of
the torch tensors it is given, passes their device pointers and the current
HIP stream to the C ABI declared in ``include/chebrbm.h``, and raises on a
non-zero status.  All arithmetic runs in the HIP kernels of the library.
Importing this module never falls back to anything else: if the library is
missing, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchebrbm.so")

CRBM_OK, CRBM_EINVAL, CRBM_EUNSUPPORTED, CRBM_EHIP, CRBM_ENOMEM = 0, -1, -2, -3, -4
FLAG_NOT_CONVERGED, FLAG_NONFINITE, FLAG_CHOLESKY_FAIL = 1, 2, 4
CHAIN, SQUARE = 0, 1
FLIP, EXCHANGE = 0, 1
CG_DENSE, CG_MATFREE, CHOLESKY = 0, 1, 2
FP32, BF16 = 0, 1
PLAN_DENSE_S, PLAN_CHOLESKY, PLAN_BASIS, PLAN_SYM_BASIS = 1, 2, 4, 8
BUF_F, BUF_DALPHA, BUF_OMEAN, BUF_S, BUF_WAVE_CLOCKS = 0, 1, 2, 3, 4
MAX_CLOCK_WAVES = 16384

# names declared in include/chebrbm.h
EXPORTS = ("crbm_plan_create", "crbm_plan_create_ex", "crbm_plan_destroy", "crbm_plan_buffer", "crbm_last_error", "crbm_plan_profile",
           "crbm_plan_profile_read", "crbm_init_rbm", "crbm_init_chains", "crbm_sample", "crbm_local_estimators",
           "crbm_sr_step", "crbm_sr_energy_step", "crbm_chebyshev_moment", "crbm_fidelity_grad", "crbm_batched_moments",
           "crbm_batched_autotune", "crbm_batched_set_shape", "crbm_batched_lds_rows", "crbm_plan_set_sbuild_tile", "crbm_sbuild_autotune", "crbm_moment_matrices", "crbm_corrected_moments", "crbm_lanczos",
           "crbm_spectrum_kpm", "crbm_spectrum_cf", "crbm_probe_mfma", "crbm_probe_hbm", "crbm_probe_logcosh", "crbm_probe_gather",
           "crbm_sym_matrices", "crbm_fit_stats", "crbm_enum_weights",
           "crbm_fidelity_grad_noalloc")
PROF_NAMES = ("sample", "theta", "local", "ot", "sbuild", "cg", "moment", "pack", "cholesky", "batched", "gram", "sborder")


class CrbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"chebrbm error {code}: {msg}")
        self.code = code


class _Rbm(ctypes.Structure):
    _fields_ = [("n_visible", ctypes.c_int), ("n_hidden", ctypes.c_int), ("a", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("W", ctypes.c_void_p)]


class _Lattice(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("J", ctypes.c_double)]


class _Cheb(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("E_c", ctypes.c_double), ("W_scale", ctypes.c_double),
                ("beta_n", ctypes.c_double * 2), ("beta_nm1", ctypes.c_double * 2), ("q", ctypes.c_double * 2)]


_lib = None
_vp, _i, _l, _u64, _d, _f = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_uint64, ctypes.c_double, ctypes.c_float


def lib():
    """Load libchebrbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2103_08804_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.crbm_last_error.restype = ctypes.c_char_p
        L.crbm_plan_create.argtypes = [P(_vp), P(_Lattice), _i, _l, _i]
        L.crbm_plan_create_ex.argtypes = [P(_vp), P(_Lattice), _i, _l, _i, _i]
        L.crbm_plan_destroy.argtypes = [_vp]
        L.crbm_plan_buffer.argtypes = [_vp, _i, P(_vp), P(ctypes.c_size_t)]
        L.crbm_plan_profile.argtypes = [_vp, _i]
        L.crbm_plan_profile_read.argtypes = [_vp, _i, P(_i), P(_d)]
        L.crbm_init_rbm.argtypes = [P(_Rbm), _u64, _f, _vp]
        L.crbm_init_chains.argtypes = [_vp, _vp, _i, _u64, _i, _vp]
        L.crbm_sample.argtypes = [_vp, P(_Rbm), _vp, _vp, _vp, _i, _i, _i, _u64, _u64, _vp, _vp, _vp, _vp]
        L.crbm_local_estimators.argtypes = [_vp, P(_Rbm), P(_Rbm), P(_Rbm), P(_Cheb), _vp, _l, _vp, _vp, _vp, _vp,
                                            _vp, _vp]
        L.crbm_sr_step.argtypes = [_vp, P(_Rbm), _vp, _vp, _vp, _vp, _l, _d, _d, _i, _i, _d, _i, _vp, _vp]
        L.crbm_sr_energy_step.argtypes = L.crbm_sr_step.argtypes
        L.crbm_fit_stats.argtypes = [_vp, _vp, _vp, _l, _vp, _vp]
        L.crbm_enum_weights.argtypes = [_vp, _vp, _l, _vp, _vp]
        L.crbm_moment_matrices.argtypes = [_vp, P(_Rbm), _vp, _vp, _i, P(_d), _vp, _vp, _l, _vp, _vp, _vp]
        L.crbm_sym_matrices.argtypes = [_vp, P(_Rbm), _vp, _vp, _i, _i, _vp, _vp, _l, _vp, _vp, _vp]
        L.crbm_corrected_moments.argtypes = [_vp, _vp, _vp, _i, _d, _d, _i, _vp, _vp, _vp]
        L.crbm_lanczos.argtypes = [_vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp]
        L.crbm_spectrum_kpm.argtypes = [_vp, _i, _i, _d, _d, _d, _vp, _i, _vp, _vp]
        L.crbm_spectrum_cf.argtypes = [_vp, _vp, _i, _d, _d, _vp, _i, _vp, _vp]
        L.crbm_probe_mfma.argtypes = [P(_d), _vp]
        L.crbm_probe_hbm.argtypes = [ctypes.c_size_t, P(_d), _vp]
        L.crbm_probe_logcosh.argtypes = [P(_d), _vp]
        L.crbm_probe_gather.argtypes = [_i, _i, P(_d), _vp]
        L.crbm_chebyshev_moment.argtypes = [_vp, P(_Rbm), _vp, _vp, _i, P(_d), _i, _vp, _vp, _l, _vp, _vp]
        L.crbm_fidelity_grad.argtypes = [_vp, P(_Rbm), _vp, _vp, _vp, _l, _vp, _vp, _vp]
        L.crbm_fidelity_grad_noalloc.argtypes = [_i, _i, _vp, _vp, _vp, _l, _vp, _vp, _vp]
        L.crbm_batched_moments.argtypes = [_vp, P(_Rbm), _vp, _vp, _vp, _vp, _i, ctypes.c_int64, _i, _i, _i, _u64,
                                           _vp, _vp, _vp]
        L.crbm_batched_autotune.argtypes = [_vp, P(_Rbm), _vp, _vp, _vp, _vp, _i, ctypes.c_int64, _i, _i, _u64, _vp,
                                            P(_i), P(_i), P(_i), P(_d), _vp]
        L.crbm_batched_set_shape.argtypes = [_vp, _i, _i, _i]
        L.crbm_batched_lds_rows.argtypes = [_vp, _i, _i, P(_i)]
        L.crbm_plan_set_sbuild_tile.argtypes = [_vp, _i]
        L.crbm_sbuild_autotune.argtypes = [_vp, _vp, _vp, _l, P(_i), P(_d), _vp]
        for name in EXPORTS:
            if name != "crbm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != CRBM_OK:
        raise CrbmError(rc, lib().crbm_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class RBM:
    """Device parameters of one RBM: a[N], b[M], W[N][M] (torch.complex64, contiguous)."""
    a: torch.Tensor
    b: torch.Tensor
    W: torch.Tensor

    @property
    def N(self):
        return self.a.shape[0]

    @property
    def M(self):
        return self.b.shape[0]

    @classmethod
    def empty(cls, N, M, device="cuda"):
        z = lambda *s: torch.zeros(*s, dtype=torch.complex64, device=device)
        return cls(z(N), z(M), z(N, M))

    @classmethod
    def from_packed(cls, v, N, M):
        """Views into one packed [a | b | W] vector (complex64, length N + M + N*M)."""
        return cls(v[:N], v[N:N + M], v[N + M:].view(N, M))

    def struct(self):
        N, M = self.N, self.M
        return _Rbm(N, M, _ptr(self.a, torch.complex64, (N,), "a"), _ptr(self.b, torch.complex64, (M,), "b"),
                    _ptr(self.W, torch.complex64, (N, M), "W"))


class Plan:
    """Lattice + hidden width + workspace (see crbm_plan_create / crbm_plan_create_ex: basis_k_max with
    PLAN_BASIS or PLAN_SYM_BASIS reserves the moment-correction workspace)."""

    def __init__(self, kind, Lx, Ly=1, M=1, max_samples=1, flags=0, J=1.0, basis_k_max=0):
        self.kind, self.Lx, self.Ly, self.M, self.J = kind, Lx, (Ly if kind == SQUARE else 1), M, J
        self.N = self.Lx * self.Ly
        self.P = self.N + M + self.N * M
        self.max_samples = max_samples
        self._h = ctypes.c_void_p()
        lat = _Lattice(kind, Lx, Ly, J)
        _check(lib().crbm_plan_create_ex(ctypes.byref(self._h), ctypes.byref(lat), M, max_samples, flags,
                                         basis_k_max))

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("plan is closed")
        return self._h

    def close(self):
        if self._h:
            _check(lib().crbm_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool):
        """Start (True) or stop (False) recording kernel-group timings; discards earlier records."""
        _check(lib().crbm_plan_profile(self.handle, int(enable)))

    def profile_read(self):
        """{group name: (count, total_ms)} of the recorded kernel groups (waits for their events)."""
        out = {}
        for gid, name in enumerate(PROF_NAMES):
            c, t = ctypes.c_int(), ctypes.c_double()
            _check(lib().crbm_plan_profile_read(self.handle, gid, ctypes.byref(c), ctypes.byref(t)))
            if c.value:
                out[name] = (c.value, t.value)
        return out

    def buffer_ptr(self, which):
        """(device pointer, bytes) of a workspace buffer (CRBM_BUF_*)."""
        p, n = ctypes.c_void_p(), ctypes.c_size_t()
        _check(lib().crbm_plan_buffer(self.handle, which, ctypes.byref(p), ctypes.byref(n)))
        return p.value, n.value


def copy_plan_buffer(plan, which, out):
    """Copy a workspace buffer into the tensor ``out`` (same byte size) on the current stream."""
    ptr, nbytes = plan.buffer_ptr(which)
    if out.numel() * out.element_size() != nbytes:
        raise ValueError(f"buffer has {nbytes} bytes, out has {out.numel() * out.element_size()}")
    src = torch.cuda.current_stream()
    hip = _hip_runtime()
    rc = hip.hipMemcpyAsync(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes),
                            ctypes.c_int(3), ctypes.c_void_p(src.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed with {rc}")
    return out


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    return _hip


# --------------------------------------------------------------------------- entry points
def init_rbm(rbm: RBM, seed: int, stddev: float, stream=None):
    s = rbm.struct()
    _check(lib().crbm_init_rbm(ctypes.byref(s), seed, stddev, _stream(stream)))


def init_chains(plan: Plan, spins, seed: int, zero_magnetisation: bool, stream=None):
    C = spins.shape[0]
    p = _ptr(spins, torch.int8, (C, plan.N), "spins")
    _check(lib().crbm_init_chains(plan.handle, p, C, seed, int(zero_magnetisation), _stream(stream)))


def sample(plan: Plan, psi: RBM, spins, n_sweeps: int, proposal: int, seed: int, step_offset: int = 0,
           theta_out=None, logpsi_out=None, samples_out=None, n_accept=None, trace=None, stream=None):
    C = spins.shape[0]
    N, M = plan.N, plan.M
    words = (n_sweeps * N + 31) // 32
    s = psi.struct()
    _check(lib().crbm_sample(
        plan.handle, ctypes.byref(s), _ptr(spins, torch.int8, (C, N), "spins"),
        _ptr(theta_out, torch.complex64, (C, M), "theta_out"), _ptr(logpsi_out, torch.complex64, (C,), "logpsi_out"),
        C, n_sweeps, proposal, seed, step_offset,
        _ptr(samples_out, torch.int8, (n_sweeps, C, N), "samples_out"),
        _ptr(n_accept, torch.int32, (C,), "n_accept"), _ptr(trace, torch.int32, (C, words), "trace"),
        _stream(stream)))


def make_cheb(order, E_c, W_scale, beta_n=1.0, beta_nm1=1.0, q=(0.0, 0.0)):
    c = _Cheb()
    c.order, c.E_c, c.W_scale = int(order), float(E_c), float(W_scale)
    bn, bm = complex(beta_n), complex(beta_nm1)
    c.beta_n[0], c.beta_n[1] = bn.real, bn.imag
    c.beta_nm1[0], c.beta_nm1[1] = bm.real, bm.imag
    c.q[0], c.q[1] = float(q[0]), float(q[1])
    return c


def local_estimators(plan: Plan, fit: RBM, samples, psi_n: RBM | None = None, psi_nm1: RBM | None = None,
                     cheb=None, logpsi_out=None, eloc_out=None, R_out=None, tanh_out=None, O_out=None, stream=None):
    n = samples.shape[0]
    N, M, P = plan.N, plan.M, plan.P
    f = fit.struct()
    pn = psi_n.struct() if psi_n is not None else None
    pm = psi_nm1.struct() if psi_nm1 is not None else None
    _check(lib().crbm_local_estimators(
        plan.handle, ctypes.byref(f), ctypes.byref(pn) if pn is not None else None,
        ctypes.byref(pm) if pm is not None else None, ctypes.byref(cheb) if cheb is not None else None,
        _ptr(samples, torch.int8, (n, N), "samples"), n,
        _ptr(logpsi_out, torch.complex64, (n,), "logpsi_out"), _ptr(eloc_out, torch.complex64, (n,), "eloc_out"),
        _ptr(R_out, torch.complex64, (n,), "R_out"), _ptr(tanh_out, torch.complex64, (n, M), "tanh_out"),
        _ptr(O_out, torch.complex64, (n, P), "O_out"), _stream(stream)))


def sr_step(plan: Plan, fit: RBM, samples, tanh_theta, R, dgamma: float, diag_shift: float, solver: int,
            precision: int, cg_tol: float, cg_maxit: int, stats_out, weights=None, stream=None):
    n = samples.shape[0]
    N, M = plan.N, plan.M
    f = fit.struct()
    _check(lib().crbm_sr_step(
        plan.handle, ctypes.byref(f), _ptr(samples, torch.int8, (n, N), "samples"),
        _ptr(weights, torch.float64, (n,), "weights"), _ptr(tanh_theta, torch.complex64, (n, M), "tanh_theta"),
        _ptr(R, torch.complex64, (n,), "R"), n, dgamma, diag_shift, solver, precision, cg_tol, cg_maxit,
        _ptr(stats_out, torch.float64, (8,), "stats_out"), _stream(stream)))


def sr_energy_step(plan: Plan, psi: RBM, samples, tanh_theta, eloc, lr: float, diag_shift: float, solver: int,
                   precision: int, cg_tol: float, cg_maxit: int, stats_out, weights=None, stream=None):
    n = samples.shape[0]
    N, M = plan.N, plan.M
    f = psi.struct()
    _check(lib().crbm_sr_energy_step(
        plan.handle, ctypes.byref(f), _ptr(samples, torch.int8, (n, N), "samples"),
        _ptr(weights, torch.float64, (n,), "weights"), _ptr(tanh_theta, torch.complex64, (n, M), "tanh_theta"),
        _ptr(eloc, torch.complex64, (n,), "eloc"), n, lr, diag_shift, solver, precision, cg_tol, cg_maxit,
        _ptr(stats_out, torch.float64, (8,), "stats_out"), _stream(stream)))


def fit_stats(plan: Plan, R, stats_out, weights=None, stream=None):
    """stats_out (float64 [5]) = {gamma, Re beta, Im beta, <|R|^2>, flags} of the ratios R (complex64 [n])."""
    n = R.shape[0]
    _check(lib().crbm_fit_stats(plan.handle, _ptr(R, torch.complex64, (n,), "R"),
                                _ptr(weights, torch.float64, (n,), "weights"), n,
                                _ptr(stats_out, torch.float64, (5,), "stats_out"), _stream(stream)))


def enum_weights(plan: Plan, logpsi, weights_out, stream=None):
    """weights_out (float64 [n]) = |psi_s|^2 / sum |psi|^2 from logpsi (complex64 [n]), all configurations listed once."""
    n = logpsi.shape[0]
    _check(lib().crbm_enum_weights(plan.handle, _ptr(logpsi, torch.complex64, (n,), "logpsi"), n,
                                   _ptr(weights_out, torch.float64, (n,), "weights_out"), _stream(stream)))


def chebyshev_moment(plan: Plan, psi_gs: RBM, t_params, betas, qs, samples, mu_out, weights=None, stream=None):
    n = samples.shape[0]
    N, P = plan.N, plan.P
    n_max = 0 if t_params is None else t_params.shape[0]
    qflat = [float(v) for q in qs for v in (q[0], q[1])]
    n_q = len(qflat) // 2
    qarr = (ctypes.c_double * len(qflat))(*qflat)
    g = psi_gs.struct()
    _check(lib().crbm_chebyshev_moment(
        plan.handle, ctypes.byref(g),
        _ptr(t_params, torch.complex64, (n_max, P), "t_params") if n_max else None,
        _ptr(betas, torch.complex128, (n_max,), "betas") if n_max else None, n_max,
        qarr, n_q, _ptr(samples, torch.int8, (n, N), "samples"), _ptr(weights, torch.float64, (n,), "weights"), n,
        _ptr(mu_out, torch.complex128, (n_q, n_max + 1), "mu_out"), _stream(stream)))


def fidelity_grad(plan: Plan, fit: RBM, samples, tanh_theta, R, grad_out, loss_out=None, stream=None):
    n = samples.shape[0]
    N, M, P = plan.N, plan.M, plan.P
    f = fit.struct()
    _check(lib().crbm_fidelity_grad(
        plan.handle, ctypes.byref(f), _ptr(samples, torch.int8, (n, N), "samples"),
        _ptr(tanh_theta, torch.complex64, (n, M), "tanh_theta"), _ptr(R, torch.complex64, (n,), "R"), n,
        _ptr(grad_out, torch.complex128, (P,), "grad_out") if grad_out is not None else None,
        _ptr(loss_out, torch.float64, (1,), "loss_out"),
        _stream(stream)))


def fidelity_grad_noalloc(N: int, M: int, samples, tanh_theta, R, grad_out, loss_out=None, stream=None):
    """crbm_fidelity_grad without a plan or any allocation (static device scratch of 48 MiB)."""
    n = samples.shape[0]
    P = N + M + N * M
    _check(lib().crbm_fidelity_grad_noalloc(
        N, M, _ptr(samples, torch.int8, (n, N), "samples"), _ptr(tanh_theta, torch.complex64, (n, M), "tanh_theta"),
        _ptr(R, torch.complex64, (n,), "R"), n,
        _ptr(grad_out, torch.complex128, (P,), "grad_out") if grad_out is not None else None,
        _ptr(loss_out, torch.float64, (1,), "loss_out"), _stream(stream)))


def moment_matrices(plan: Plan, psi_gs: RBM, t_params, betas, q, samples, G_out, H_out, weights=None, stream=None):
    """G_nm = <conj(B_n) B_m>, H_nm = <conj(B_n) (H t_m)/psi_gs> over samples of |psi_gs|^2, K = n_max + 1."""
    n = samples.shape[0]
    N, P = plan.N, plan.P
    n_max = 0 if t_params is None else t_params.shape[0]
    K = n_max + 1
    qarr = (ctypes.c_double * 2)(float(q[0]), float(q[1]))
    g = psi_gs.struct()
    _check(lib().crbm_moment_matrices(
        plan.handle, ctypes.byref(g),
        _ptr(t_params, torch.complex64, (n_max, P), "t_params") if n_max else None,
        _ptr(betas, torch.complex128, (n_max,), "betas") if n_max else None, n_max, qarr,
        _ptr(samples, torch.int8, (n, N), "samples"), _ptr(weights, torch.float64, (n,), "weights"), n,
        _ptr(G_out, torch.complex128, (K, K), "G_out"), _ptr(H_out, torch.complex128, (K, K), "H_out"),
        _stream(stream)))


def sym_matrices(plan: Plan, psi_gs: RBM, t_params, betas, samples, G_out, H_out, rotations: bool = True,
                 weights=None, stream=None):
    """G^(k), H^(k) [N][K][K] of the symmetry-projected basis (local S^z_0 RBMs) for all N momenta."""
    n = samples.shape[0]
    N, P = plan.N, plan.P
    n_max = 0 if t_params is None else t_params.shape[0]
    K = n_max + 1
    g = psi_gs.struct()
    _check(lib().crbm_sym_matrices(
        plan.handle, ctypes.byref(g),
        _ptr(t_params, torch.complex64, (n_max, P), "t_params") if n_max else None,
        _ptr(betas, torch.complex128, (n_max,), "betas") if n_max else None, n_max, int(bool(rotations)),
        _ptr(samples, torch.int8, (n, N), "samples"), _ptr(weights, torch.float64, (n,), "weights"), n,
        _ptr(G_out, torch.complex128, (N, K, K), "G_out"), _ptr(H_out, torch.complex128, (N, K, K), "H_out"),
        _stream(stream)))


def corrected_moments(plan: Plan, G, H, E_c: float, W_scale: float, mu_out, info_out, stream=None):
    K = G.shape[0]
    n_out = mu_out.shape[0]
    _check(lib().crbm_corrected_moments(
        plan.handle, _ptr(G, torch.complex128, (K, K), "G"), _ptr(H, torch.complex128, (K, K), "H"), K, E_c, W_scale,
        n_out, _ptr(mu_out, torch.float64, (n_out,), "mu_out"), _ptr(info_out, torch.float64, (3,), "info_out"),
        _stream(stream)))


def lanczos(plan: Plan, G, H, a_out, b2_out, info_out, stream=None):
    K = G.shape[0]
    m = a_out.shape[0]
    _check(lib().crbm_lanczos(
        plan.handle, _ptr(G, torch.complex128, (K, K), "G"), _ptr(H, torch.complex128, (K, K), "H"), K, m,
        _ptr(a_out, torch.float64, (m,), "a_out"), _ptr(b2_out, torch.float64, (m,), "b2_out"),
        _ptr(info_out, torch.float64, (2,), "info_out"), _stream(stream)))


def spectrum_kpm(mu, E0: float, E_c: float, W_scale: float, omega, A_out, jackson: bool = True, stream=None):
    n_mom = mu.shape[0]
    n_w = omega.shape[0]
    _check(lib().crbm_spectrum_kpm(
        _ptr(mu, torch.float64, (n_mom,), "mu"), n_mom, int(bool(jackson)), E0, E_c, W_scale,
        _ptr(omega, torch.float64, (n_w,), "omega"), n_w, _ptr(A_out, torch.float64, (n_w,), "A_out"),
        _stream(stream)))


def spectrum_cf(a, b2, m: int, E0: float, eta: float, omega, A_out, stream=None):
    n_w = omega.shape[0]
    if not 1 <= m <= min(a.shape[0], b2.shape[0]):
        raise ValueError(f"m = {m} levels but a has {a.shape[0]} and b2 {b2.shape[0]} entries")
    _check(lib().crbm_spectrum_cf(
        _ptr(a, torch.float64, (a.shape[0],), "a"), _ptr(b2, torch.float64, (b2.shape[0],), "b2"), m, E0, eta,
        _ptr(omega, torch.float64, (n_w,), "omega"), n_w, _ptr(A_out, torch.float64, (n_w,), "A_out"),
        _stream(stream)))


def probe_mfma(stream=None) -> float:
    """Sustained BF16 matrix-core TFLOP/s of the current device (synchronises)."""
    v = ctypes.c_double()
    _check(lib().crbm_probe_mfma(ctypes.byref(v), _stream(stream)))
    return v.value


def probe_hbm(nbytes: int = 1 << 30, stream=None) -> float:
    """Copy bandwidth (read + write) in GB/s of the current device (synchronises)."""
    v = ctypes.c_double()
    _check(lib().crbm_probe_hbm(nbytes, ctypes.byref(v), _stream(stream)))
    return v.value


def probe_logcosh(stream=None) -> float:
    """Re log(2 cosh z) evaluations per second in the sweep's form on the current device (synchronises)."""
    v = ctypes.c_double()
    _check(lib().crbm_probe_logcosh(ctypes.byref(v), _stream(stream)))
    return v.value


def probe_gather(n_rows: int, row_elems: int, stream=None) -> float:
    """GB/s of whole-row reads of an n_rows x row_elems complex64 table at random rows (synchronises)."""
    v = ctypes.c_double()
    _check(lib().crbm_probe_gather(n_rows, row_elems, ctypes.byref(v), _stream(stream)))
    return v.value


def batched_moments(plan: Plan, psi_gs: RBM, t_params, betas, q, chain_offsets, n_burn: int, n_sweeps: int,
                    proposal: int, seed: int, mu_out, total_chains: int | None = None, trace=None, stream=None):
    """Per-instance (<|f_q|^2>, <f_q^* beta t~/psi_gs>) for all instances in one persistent launch.

    total_chains (= chain_offsets[-1]) must be given under graph capture, where reading it back from
    the device is not allowed.  trace (int32 [total_chains][ceil((n_burn + n_sweeps) N / 32)]) receives
    the accept bit of every proposal."""
    n_inst, P = t_params.shape
    total = int(chain_offsets[-1].item()) if total_chains is None else int(total_chains)
    words = ((n_burn + n_sweeps) * plan.N + 31) // 32
    tr = None if trace is None else _ptr(trace, torch.int32, (total, words), "trace")
    g = psi_gs.struct()
    _check(lib().crbm_batched_moments(
        plan.handle, ctypes.byref(g), _ptr(t_params, torch.complex64, (n_inst, plan.P), "t_params"),
        _ptr(betas, torch.complex128, (n_inst,), "betas"), _ptr(q, torch.float64, (n_inst, 2), "q"),
        _ptr(chain_offsets, torch.int64, (n_inst + 1,), "chain_offsets"), n_inst, total, n_burn, n_sweeps, proposal,
        seed, _ptr(mu_out, torch.complex128, (n_inst, 2), "mu_out"), tr, _stream(stream)))


def batched_autotune(plan: Plan, psi_gs: RBM, t_params, betas, q, chain_offsets, n_sweeps_probe: int,
                     proposal: int, seed: int, stream=None):
    """Pick the launch shape of the batched kernel (host-synchronising).
    Returns (waves_per_block, blocks, lanes_per_chain, ms)."""
    n_inst = t_params.shape[0]
    total = int(chain_offsets[-1].item())
    scratch = torch.empty(n_inst, 2, dtype=torch.complex128, device=t_params.device)
    g = psi_gs.struct()
    w, b, ln, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().crbm_batched_autotune(
        plan.handle, ctypes.byref(g), _ptr(t_params, torch.complex64, (n_inst, plan.P), "t_params"),
        _ptr(betas, torch.complex128, (n_inst,), "betas"), _ptr(q, torch.float64, (n_inst, 2), "q"),
        _ptr(chain_offsets, torch.int64, (n_inst + 1,), "chain_offsets"), n_inst, total, n_sweeps_probe, proposal,
        seed, _ptr(scratch), ctypes.byref(w), ctypes.byref(b), ctypes.byref(ln), ctypes.byref(ms), _stream(stream)))
    return w.value, b.value, ln.value, ms.value


def batched_set_shape(plan: Plan, waves_per_block: int, blocks: int, lanes_per_chain: int):
    """Fix the launch shape of crbm_batched_moments (lanes per chain 64, 32 or 16)."""
    _check(lib().crbm_batched_set_shape(plan.handle, waves_per_block, blocks, lanes_per_chain))


def batched_lds_rows(plan: Plan, proposal: int, waves_per_block: int) -> bool:
    """Whether the 64-lane batched kernel reads psi_gs's rows from its copy in LDS at this shape."""
    u = ctypes.c_int()
    _check(lib().crbm_batched_lds_rows(plan.handle, proposal, waves_per_block, ctypes.byref(u)))
    return bool(u.value)


def set_sbuild_tile(plan: Plan, k_tile: int):
    """K tile (64 or 128 samples) of the plan's BF16 S contraction; every tile gives the same S."""
    _check(lib().crbm_plan_set_sbuild_tile(plan.handle, k_tile))


def sbuild_autotune(plan: Plan, samples, tanh_theta, stream=None):
    """Time the BF16 S contraction with each K tile on these operands, keep the faster in the plan
    (host-synchronising; overwrites the plan's S).  Returns (k_tile, ms)."""
    n = samples.shape[0]
    kt, ms = ctypes.c_int(), ctypes.c_double()
    _check(lib().crbm_sbuild_autotune(plan.handle, _ptr(samples, torch.int8, (n, plan.N), "samples"),
                                      _ptr(tanh_theta, torch.complex64, (n, plan.M), "tanh_theta"), n,
                                      ctypes.byref(kt), ctypes.byref(ms), _stream(stream)))
    return kt.value, ms.value
