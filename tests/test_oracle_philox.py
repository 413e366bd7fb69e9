"""Pins for the oracle's counter-based generator and its derived draws.

Philox4x32-10 is a build choice (the paper names no sampler); the oracle's
implementation, written from Salmon et al. (SC'11), is pinned against the
rocRAND engine compiled for the host from its public header.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("kat") / "philox_ref")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe], check=True,
                   capture_output=True)

    def run(cases):
        inp = "".join("%x %x %x %x %x %x\n" % (k[0], k[1], c[0], c[1], c[2], c[3]) for c, k in cases)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]
    return run


def test_philox_matches_rocrand(orc, rocrand_ref):
    r = np.random.default_rng(7)
    cases = [([0, 0, 0, 0], [0, 0]),
             ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
             ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0])]
    for _ in range(200):
        cases.append((list(r.integers(0, 2**32, 4, dtype=np.uint64)), list(r.integers(0, 2**32, 2, dtype=np.uint64))))
    # the stream layout used by the sampler: (chain, step lo, step hi, tag)
    for c in range(3):
        for t in (0, 1, 99, 2**32 + 5):
            cases.append(([c, t & 0xFFFFFFFF, t >> 32, 0], [1234, 0]))
    ref = rocrand_ref(cases)
    for (ctr, key), want in zip(cases, ref):
        got = orc.philox([int(x) for x in ctr], [int(x) for x in key])
        assert [int(x) for x in got] == want, (ctr, key)


def test_init_chains_zero_magnetisation(orc):
    s = orc.init_chains(40, 256, 99, 1)
    assert s.shape == (256, 40)
    assert np.all(s.sum(axis=1) == 0)
    assert set(np.unique(s)) == {-1, 1}
    # Fisher-Yates gives a uniform permutation: each site is up with probability 1/2
    frac = (s == 1).mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 0.15)
    s2 = orc.init_chains(40, 256, 99, 1)
    assert np.array_equal(s, s2)


def test_init_chains_random(orc):
    s = orc.init_chains(64, 512, 5, 0)
    assert set(np.unique(s)) == {-1, 1}
    assert abs((s == 1).mean() - 0.5) < 0.02


def test_init_rbm_statistics(orc):
    rbm = orc.init_rbm(30, 60, 11, 0.25)
    v = rbm.vector()
    assert v.shape == (30 + 60 + 1800,)
    # Re and Im each ~ N(0, 0.25^2)
    for part in (v.real, v.imag):
        assert abs(part.mean()) < 4 * 0.25 / np.sqrt(v.size)
        assert abs(part.std() / 0.25 - 1.0) < 0.06
    assert abs(np.corrcoef(v.real, v.imag)[0, 1]) < 0.08
