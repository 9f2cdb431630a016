"""Heterogeneous persistent launch (bysdf_eval_batched): parity with the
oracle, identity with the plain kernel across schedules, graph capture
with replays, and the full-size 4,096-type batch on sampled outputs."""
import numpy as np
import pytest

import oracle
from paper_2401_12724_amd import autotune, bysdf, workloads as W

from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _small_hetero(n_types=384, seed=13):
    counts = W.lognormal_counts(n_types, median=96, sigma=1.5, lo=1, hi=2000, seed=seed)
    counts[::37] = 0  # some types without queries
    return W.heterogeneous(n_types, seed, counts=counts)


def test_batched_parity_and_schedules(torch_cuda):
    torch = torch_cuda
    P, q, off = _small_hetero()
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    offd = torch.from_numpy(off).cuda()
    v0, f0 = bysdf.bysdf_eval_batched(T, offd, qd)
    torch.cuda.synchronize()
    g, gf = v0.cpu().numpy().T, f0.cpu().numpy().view(np.uint32)
    o, of = oracle.eval(P, q)
    rep = compare(g, gf, o[:, :12], of)
    print({k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep)
    # plain kernel on the same queries agrees to rounding
    pv, pf = bysdf.bysdf_eval(T, qd)
    torch.cuda.synchronize()
    assert np.array_equal(pf.cpu().numpy(), f0.cpu().numpy())
    assert np.allclose(pv.cpu().numpy(), v0.cpu().numpy(), rtol=1e-6, atol=1e-9)
    # schedules only move tiles between workgroups (and change the register
    # budget of the kernel): outputs are identical
    for sc in (dict(chunk=1, grid=64, use_lds=0), dict(chunk=8, grid=4096, use_lds=1),
               dict(chunk=3, grid=7, use_lds=1), dict(chunk=2, grid=512, use_lds=1, block=128),
               dict(chunk=4, grid=1024, use_lds=0, min_waves=1),
               dict(chunk=1, grid=300, use_lds=1, block=128, min_waves=1)):
        v1, f1 = bysdf.bysdf_eval_batched(T, offd, qd, sched=sc)
        torch.cuda.synchronize()
        assert torch.equal(v1, v0) and torch.equal(f1, f0), sc
    for bad, what in ((dict(chunk=1, grid=64, use_lds=0, block=100), "block"),
                      (dict(chunk=1, grid=64, use_lds=0, min_waves=3), "min_waves")):
        with pytest.raises(RuntimeError, match=what):
            bysdf.bysdf_eval_batched(T, offd, qd, sched=bad)


def test_batched_graph_replays(torch_cuda):
    """Capture the launch sequence in a graph, replay it with eager work in
    between, and check every replay against the eager result."""
    torch = torch_cuda
    P, q, off = _small_hetero(128, 21)
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    offd = torch.from_numpy(off).cuda()
    n = len(q["h"])
    out = bysdf.alloc_eval_out(n)
    ws = bysdf.alloc_workspace(bysdf.bysdf_batched_workspace_size(T.n_types))
    ref_v, ref_f = bysdf.bysdf_eval_batched(T, offd, qd)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bysdf.bysdf_eval_batched(T, offd, qd, out, None, ws)  # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bysdf.bysdf_eval_batched(T, offd, qd, out, None, ws)
    for r in range(4):
        out[0].zero_()
        out[1].zero_()
        bysdf.bysdf_eval(T, qd)  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref_v) and torch.equal(out[1], ref_f), r


def test_autotuner_picks_a_schedule(torch_cuda, tmp_path):
    torch = torch_cuda
    P, q, off = _small_hetero(256, 17)
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    offd = torch.from_numpy(off).cuda()
    cache = str(tmp_path / "tune.json")
    cands = [dict(chunk=c, grid=g, use_lds=1, block=b, min_waves=w) for c in (1, 4) for g in (256, 2048)
             for b in (128, 256) for w in (1, 2)]
    r = autotune.autotune_batched(T, offd, qd, off, candidates=cands, reps=2, cache_path=cache)
    assert r["schedule"] in cands and r["ms"] == min(t[1] for t in r["timings"])
    r2 = autotune.autotune_batched(T, offd, qd, off, candidates=cands, cache_path=cache)
    assert r2.get("cached") and r2["schedule"] == r["schedule"]
    open(cache, "w").write("{not json")
    r3 = autotune.autotune_batched(T, offd, qd, off, candidates=cands[:1], reps=1,
                                   cache_path=cache)
    assert r3["schedule"] == cands[0]


def test_full_size_heterogeneous_sampled(torch_cuda):
    """4,096 types (2..5 plies, 32..128 fibers), lognormal counts summing to
    ~2^26 queries, one persistent launch; 8,000 sampled outputs against the
    oracle."""
    torch = torch_cuda
    P, q, off = W.heterogeneous(4096, 3)
    n = len(q["h"])
    assert 0.8 * 2 ** 26 < n < 1.25 * 2 ** 26, n
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    offd = torch.from_numpy(off).cuda()
    v, f = bysdf.bysdf_eval_batched(T, offd, qd)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(5).choice(n, 8000, replace=False))
    sub = {k: (a[..., idx] if a is not None else None) for k, a in q.items()}
    o, of = oracle.eval(oracle.TypeSet(P), sub)
    rep = compare(v[:, idx].cpu().numpy().T, f[idx].cpu().numpy(), o[:, :12], of)
    print({k: v_ for k, v_ in rep.items() if k != "bad_idx"})
    assert_parity(rep)
