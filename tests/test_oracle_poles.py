"""Pin for the oracle's log(2 cosh theta) and tanh theta near the zeros of cosh (Sec. I amplitude, Sec. III
log-derivatives), against 50-digit arithmetic (mpmath) on the same double-precision theta.

Complex RBMs place hidden units on (or within rounding of) the zeros theta = i pi (m + 1/2) of cosh to
represent nodes of the state.  There the textbook form s z + log(1 + exp(-2 s z)) cancels; the oracle uses
cosh theta = i (-1)^m sinh delta and tanh theta = coth delta with delta = theta - i pi (m + 1/2).  Every
case compares log psi and O of a one-site, one-unit RBM (a = 0, W = 0, b = theta) with mpmath evaluated on
the exact binary64 value of theta."""
import math

import mpmath
import numpy as np

mpmath.mp.dps = 50


def _cases():
    half_pi = math.pi / 2   # binary64 value, 6.12e-17 below pi/2
    ulp = math.ulp(half_pi)
    out = []
    for m in (-2, -1, 0, 1, 3):
        y0 = math.pi * (m + 0.5)
        for dx in (0.0, 3e-15, -2e-12, 1e-9, 0.2, -0.45):
            for k in (0, 1, -3, 1000, 10 ** 6):
                out.append(complex(dx, y0 + k * math.ulp(y0)))
    # far from the zeros: the textbook branch
    out += [complex(0.3, 0.1), complex(-2.0, 1.0), complex(5.0, -7.3), complex(0.7, half_pi + 0.6)]
    return out


def test_log2cosh_and_tanh_near_zeros_of_cosh(orc):
    sig = np.array([[1]], np.int8)
    worst_l, worst_t = 0.0, 0.0
    for z in _cases():
        rbm = orc.RBM(np.zeros(1), np.array([z]), np.zeros((1, 1)))
        lp = orc.logpsi(rbm, sig)[0]
        t = orc.logderiv(rbm, sig)[0, 1]
        zm = mpmath.mpc(z.real, z.imag)   # exactly the double theta
        l_ref = complex(mpmath.log(2 * mpmath.cosh(zm)))
        t_ref = complex(mpmath.tanh(zm))
        # Re log psi absolutely (it may be far below zero), Im modulo 2 pi, tanh relatively
        dl = abs(lp.real - l_ref.real) + abs(math.remainder(lp.imag - l_ref.imag, 2 * math.pi))
        dt = abs(t - t_ref) / abs(t_ref)
        worst_l, worst_t = max(worst_l, dl), max(worst_t, dt)
        assert dl < 1e-12, (z, lp, l_ref)
        assert dt < 1e-12, (z, t, t_ref)
    print("largest differences: log 2cosh", worst_l, "tanh (relative)", worst_t)
