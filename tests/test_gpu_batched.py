"""Batched moments over (q, n) instances: parity with the oracle, graph capture and replay,
and independence of the result from the launch shape chosen by the autotuner."""
import numpy as np
import pytest
import torch

import paper_2103_08804_amd as crbm
import synth
from gpu_util import np_of, rel_err, to_device_rbm, to_oracle_rbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    crbm.lib()


def _instances(orc, kind, Lx, Ly, M, counts, seed=5):
    N = Lx * Ly
    gs_d = to_device_rbm(orc.RBM(*synth.random_rbm_arrays(seed, N, M, 0.1, std_im=0.02)))
    n_inst = len(counts)
    tv = np.stack([orc.RBM(*synth.random_rbm_arrays(seed + 1 + i, N, M, 0.1, std_im=0.02)).vector()
                   for i in range(n_inst)]).astype(np.complex64)
    r = np.random.default_rng(seed)
    betas = r.normal(size=n_inst) + 1j * r.normal(size=n_inst)
    qs = np.stack([r.uniform(0, 2 * np.pi, n_inst), r.uniform(0, 2 * np.pi, n_inst) if kind == 1 else
                   np.zeros(n_inst)], axis=1)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dev = dict(t=torch.from_numpy(tv).cuda(), b=torch.from_numpy(betas).cuda(), q=torch.from_numpy(qs).cuda(),
               o=torch.from_numpy(offsets).cuda())
    return gs_d, tv, betas, qs, offsets, dev


@pytest.mark.parametrize("kind,Lx,Ly,M,counts,proposal", [
    (1, 4, 4, 16, [3, 0, 5, 1, 7, 2], 1),
    (0, 12, 1, 24, [2, 4, 1], 0),
    (1, 4, 4, 64, [4, 1, 2], 1),       # M fills one 64-lane group exactly
    (1, 10, 10, 16, [2, 1, 2], 1),     # N > 64: spins and a spread over two lane slots
])
def test_batched_vs_oracle(orc, kind, Lx, Ly, M, counts, proposal):
    N = Lx * Ly
    gs_d, tv, betas, qs, offsets, dev = _instances(orc, kind, Lx, Ly, M, counts)
    plan = crbm.Plan(kind, Lx, Ly, M, int(offsets[-1]) + 1)
    mu = torch.zeros(len(counts), 2, dtype=torch.complex128, device="cuda")
    crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 2, 5, proposal, 99, mu)
    torch.cuda.synchronize()
    gs = to_oracle_rbm(orc, gs_d)
    lat = orc.Lattice(kind, Lx, Ly)
    ref, amb, _ = orc.batched_moments(gs, tv.astype(np.complex128), betas, qs, offsets, lat, 2, 5, proposal, 99)
    assert amb == 0          # no step close enough to the threshold for FP32 to take the other branch
    assert rel_err(np_of(mu), ref) < 1e-5


def test_batched_graph_replay_and_autotune(orc):
    kind, Lx, Ly, M = 1, 8, 8, 128
    r = np.random.default_rng(4)
    counts = r.integers(4, 33, 48)
    gs_d, tv, betas, qs, offsets, dev = _instances(orc, kind, Lx, Ly, M, counts, seed=8)
    plan = crbm.Plan(kind, Lx, Ly, M, int(offsets[-1]))
    eager = torch.zeros(len(counts), 2, dtype=torch.complex128, device="cuda")
    crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 3, 1, 7, eager)
    torch.cuda.synchronize()
    ref = eager.clone()
    # graph capture of the whole launch sequence, several replays with eager work in between
    out = torch.zeros_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 3, 1, 7, out,
                                 total_chains=int(offsets[-1]))
    torch.cuda.current_stream().wait_stream(s)
    for k in range(3):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k
        crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 3, 1, 7, eager)
        torch.cuda.synchronize()
        assert torch.equal(eager, ref)
    # a different launch shape gives the same bits
    w, b, ln, ms = crbm.batched_autotune(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 1, 7)
    assert w in (1, 2, 4, 8) and b >= 1 and ln in (16, 32, 64) and ms > 0
    crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 3, 1, 7, eager)
    torch.cuda.synchronize()
    assert torch.equal(eager, ref)


def test_batched_rejects_oversized_chains(orc):
    """More than 2^31 - 1 proposals per chain is refused on the host, before any launch."""
    kind, Lx, Ly, M = 1, 4, 4, 16
    gs_d, tv, betas, qs, offsets, dev = _instances(orc, kind, Lx, Ly, M, [2, 3])
    plan = crbm.Plan(kind, Lx, Ly, M, int(offsets[-1]))
    mu = torch.zeros(2, 2, dtype=torch.complex128, device="cuda")
    n_sweeps = (2 ** 31) // (Lx * Ly) + 1
    with pytest.raises(crbm.CrbmError):
        crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 0, n_sweeps, 1, 3, mu,
                             total_chains=int(offsets[-1]))


def test_batched_bad_offsets_give_nan(orc):
    """Offsets live on the device and are not checked on the host: an instance whose chain range is
    reversed or runs past total_chains gets NaN moments, the others are unaffected."""
    kind, Lx, Ly, M = 1, 4, 4, 16
    counts = [3, 2, 3]
    gs_d, tv, betas, qs, offsets, dev = _instances(orc, kind, Lx, Ly, M, counts)
    total = int(offsets[-1])
    plan = crbm.Plan(kind, Lx, Ly, M, total)
    good = torch.zeros(3, 2, dtype=torch.complex128, device="cuda")
    crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 3, 1, 5, good, total_chains=total)
    bad_off = torch.tensor([0, 3, 1, total + 4], dtype=torch.int64, device="cuda")   # [3, 1) reversed, [1, 12) past 8
    bad = torch.zeros_like(good)
    crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], bad_off, 1, 3, 1, 5, bad, total_chains=total)
    torch.cuda.synchronize()
    b = np_of(bad)
    assert np.all(np.isfinite(np_of(good)))
    assert np.all(np.isnan(b[1].real)) and np.all(np.isnan(b[1].imag))
    assert np.all(np.isnan(b[2].real)) and np.all(np.isnan(b[2].imag))
    # instance 0 owns chains 0..2 under both offset vectors: same chains, same sums
    assert np.array_equal(b[0], np_of(good)[0])


@pytest.mark.parametrize("kind,Lx,Ly,M,proposal", [(1, 4, 4, 16, 1), (0, 12, 1, 24, 0), (1, 4, 4, 100, 1),
                                                    (1, 8, 8, 128, 1), (0, 66, 1, 70, 1), (1, 4, 4, 300, 1)])
def test_batched_lanes_per_chain_bit_identical(orc, kind, Lx, Ly, M, proposal):
    """Chains on 64, 32 or 16 lanes (one, two or four chains per wave) and several grid shapes give the
    same moments and the same accept traces bit for bit: every sum runs in one fixed order.  Ragged M
    (units past M in the last slots), N > 64 (sites in a second slot), uneven chain counts, both
    proposals; 16 lanes only where M <= 128 and 32 where M <= 256, other lane counts are refused.  On
    64 lanes the rows of psi_gs come from its copy in LDS or from global memory depending on the
    occupancy at that block size: one wave per block keeps more blocks per compute unit without the
    copy whenever it is large, eight with it."""
    N = Lx * Ly
    r = np.random.default_rng(31)
    counts = r.integers(1, 13, 37)
    gs_d, tv, betas, qs, offsets, dev = _instances(orc, kind, Lx, Ly, M, counts, seed=9)
    total = int(offsets[-1])
    plan = crbm.Plan(kind, Lx, Ly, M, total)
    words = ((1 + 3) * N + 31) // 32
    res = {}
    for lanes in (64, 32, 16):
        if (lanes == 32 and M > 256) or (lanes == 16 and M > 128):
            with pytest.raises(crbm.CrbmError):
                crbm.batched_set_shape(plan, 4, 64, lanes)
            continue
        for waves, blocks in ((1, 3), (8, 512)):
            crbm.batched_set_shape(plan, waves, blocks, lanes)
            mu = torch.zeros(len(counts), 2, dtype=torch.complex128, device="cuda")
            tr = torch.zeros(total, words, dtype=torch.int32, device="cuda")
            crbm.batched_moments(plan, gs_d, dev["t"], dev["b"], dev["q"], dev["o"], 1, 3, proposal, 7, mu, trace=tr)
            torch.cuda.synchronize()
            res[(lanes, waves)] = (np_of(mu), np_of(tr))
    lds = {w: crbm.batched_lds_rows(plan, proposal, w) for w in (1, 8)}
    print("psi_gs rows from LDS at 1 and 8 waves per block:", lds)
    if (N, M) in ((64, 128), (66, 70)):
        assert lds == {1: False, 8: True}   # both paths are compared below
    if M > 256:
        assert lds == {1: False, 8: False}  # W is copied only for M <= 256
    ref_mu, ref_tr = res[(64, 1)]
    assert np.all(np.isfinite(ref_mu))
    for key, (m, t) in res.items():
        assert np.array_equal(m, ref_mu), key
        assert np.array_equal(t, ref_tr), key
    print("shapes compared", sorted(res))
