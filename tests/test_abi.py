"""The C-ABI library loads, exports every entry point of include/chebrbm.h, and rejects
bad arguments on the host with the documented status codes (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2103_08804_amd as crbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "chebrbm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(crbm_\w+)\s*\(", txt, re.M)))


def test_header_lists_binding_exports():
    assert _declared() == sorted(crbm.EXPORTS)


def test_library_exports_every_symbol():
    L = crbm.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_host_side_argument_errors():
    L = crbm.lib()
    # NULL rbm -> EINVAL, before any HIP call
    assert L.crbm_init_rbm(None, 1, 0.1, None) == crbm.CRBM_EINVAL
    assert b"NULL" in L.crbm_last_error()
    # unknown lattice kind -> EINVAL
    h = ctypes.c_void_p()
    lat = crbm._Lattice(7, 4, 4, 1.0)
    assert L.crbm_plan_create(ctypes.byref(h), ctypes.byref(lat), 4, 16, 0) == crbm.CRBM_EINVAL
    # too many sites / hidden units -> EUNSUPPORTED
    lat = crbm._Lattice(crbm.SQUARE, 20, 20, 1.0)
    assert L.crbm_plan_create(ctypes.byref(h), ctypes.byref(lat), 4, 16, 0) == crbm.CRBM_EUNSUPPORTED
    lat = crbm._Lattice(crbm.CHAIN, 10, 1, 1.0)
    assert L.crbm_plan_create(ctypes.byref(h), ctypes.byref(lat), 600, 16, 0) == crbm.CRBM_EUNSUPPORTED
    assert L.crbm_plan_create(ctypes.byref(h), ctypes.byref(lat), 4, 0, 0) == crbm.CRBM_EINVAL
    assert L.crbm_plan_create(ctypes.byref(h), ctypes.byref(lat), 4, 16, 0x100) == crbm.CRBM_EINVAL
    # NULL plan -> EINVAL
    assert L.crbm_plan_destroy(None) == crbm.CRBM_EINVAL
    assert L.crbm_sample(None, None, None, None, None, 1, 1, 0, 0, 0, None, None, None, None) == crbm.CRBM_EINVAL


def test_binding_rejects_cpu_tensors():
    import torch
    rbm = crbm.RBM(torch.zeros(4, dtype=torch.complex64), torch.zeros(3, dtype=torch.complex64),
                   torch.zeros(4, 3, dtype=torch.complex64))
    with pytest.raises(ValueError):
        rbm.struct()


def test_host_side_errors_of_the_spectral_calls():
    L = crbm.lib()
    dummy = ctypes.c_void_p(256)      # never dereferenced: every case below fails validation first
    assert L.crbm_spectrum_kpm(None, 4, 1, 0.0, 0.0, 1.0, dummy, 8, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_spectrum_kpm(dummy, 0, 1, 0.0, 0.0, 1.0, dummy, 8, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_spectrum_kpm(dummy, 4, 1, 0.0, 0.0, 0.0, dummy, 8, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_spectrum_kpm(dummy, 4, 1, 0.0, 0.0, float("inf"), dummy, 8, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_spectrum_kpm(dummy, 4, 1, 0.0, 0.0, 1.0, dummy, -1, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_spectrum_kpm(dummy, 4, 1, 0.0, 0.0, 1.0, dummy, 0, dummy, None) == crbm.CRBM_OK   # nothing to do
    assert L.crbm_spectrum_cf(dummy, dummy, 3, 0.0, 0.0, dummy, 8, dummy, None) == crbm.CRBM_EINVAL
    assert b"eta" in L.crbm_last_error()
    assert L.crbm_spectrum_cf(dummy, dummy, 0, 0.0, 0.1, dummy, 8, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_corrected_moments(None, dummy, dummy, 4, 0.0, 1.0, 8, dummy, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_lanczos(None, dummy, dummy, 4, 4, dummy, dummy, dummy, None) == crbm.CRBM_EINVAL
    assert L.crbm_moment_matrices(None, None, None, None, 0, None, None, None, 1, None, None, None) == crbm.CRBM_EINVAL
    assert L.crbm_sr_energy_step(None, None, None, None, None, None, 1, 0.1, 0.0, 0, 0, 1e-6, 10, None,
                                 None) == crbm.CRBM_EINVAL


def test_host_side_errors_of_the_probes():
    L = crbm.lib()
    v = ctypes.c_double()
    assert L.crbm_probe_mfma(None, None) == crbm.CRBM_EINVAL
    assert L.crbm_probe_hbm(1 << 30, None, None) == crbm.CRBM_EINVAL
    assert L.crbm_probe_hbm(1000, ctypes.byref(v), None) == crbm.CRBM_EINVAL
    assert L.crbm_probe_logcosh(None, None) == crbm.CRBM_EINVAL
    assert L.crbm_probe_gather(100, 400, None, None) == crbm.CRBM_EINVAL
    assert L.crbm_probe_gather(0, 400, ctypes.byref(v), None) == crbm.CRBM_EINVAL
    assert L.crbm_probe_gather(1 << 13, 1 << 12, ctypes.byref(v), None) == crbm.CRBM_EINVAL
    assert b"2^24" in L.crbm_last_error()


def test_noalloc_gradient_rejects_oversized_input_on_the_host():
    """crbm_fidelity_grad_noalloc checks its static scratch before any HIP call."""
    L = crbm.lib()
    dummy = ctypes.c_void_p(1)
    assert L.crbm_fidelity_grad_noalloc(256, 512, dummy, dummy, dummy, 1 << 20, dummy, None, None) == crbm.CRBM_ENOMEM
    assert b"static scratch" in L.crbm_last_error()
    assert L.crbm_fidelity_grad_noalloc(0, 4, dummy, dummy, dummy, 8, dummy, None, None) == crbm.CRBM_EINVAL
    assert L.crbm_fidelity_grad_noalloc(4, 4, dummy, dummy, dummy, 8, None, None, None) == crbm.CRBM_EINVAL
