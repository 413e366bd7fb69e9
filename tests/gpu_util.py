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
