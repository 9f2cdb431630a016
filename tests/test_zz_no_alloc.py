"""bysdf_eval_batched_noalloc (the batched evaluation for callers that cannot
allocate) against bysdf_eval_batched with a caller workspace, through the C
ABI: two calls in a row, the second with fewer types and queries, so the
static workspace is reused with stale contents from the first; and a handle
beyond the workspace's type limit is refused."""
import numpy as np
import pytest

from paper_2401_12724_amd import bysdf, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _batch(n_types, seed, lo=256, hi=4096):
    P = W.heterogeneous_params(n_types, seed)
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi, n_types)
    counts[rng.integers(0, n_types)] = 0  # an empty type
    off = np.zeros(n_types + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    q = W.queries(int(off[-1]), seed + 50, type_ids=np.repeat(np.arange(n_types, dtype=np.int32), counts))
    return P, q, off


@pytest.mark.parametrize("sched", [None, dict(chunk=2, grid=512, use_lds=0)])
def test_noalloc_matches_workspace_call(torch_cuda, sched):
    torch = torch_cuda
    for n_types, seed in ((96, 70), (7, 71)):   # the second call is smaller
        P, q, off = _batch(n_types, seed)
        print("noalloc case: types", n_types, "queries", int(off[-1]), "sched", sched, flush=True)
        T = bysdf.bysdf_types_create(P)
        qd = bysdf.to_device(q)
        offd = torch.from_numpy(off).cuda()
        ref_v, ref_f = bysdf.bysdf_eval_batched(T, offd, qd, sched=sched)
        out = bysdf.alloc_eval_out(int(off[-1]))
        out[0].fill_(-7.0)
        out[1].fill_(-7)
        torch.cuda.synchronize()
        v, f = bysdf.bysdf_eval_batched_noalloc(T, offd, qd, out, sched=sched)
        torch.cuda.synchronize()
        # the same kernels on the same schedule: equal bit for bit
        assert torch.equal(v, ref_v) and torch.equal(f, ref_f)


def test_noalloc_refuses_too_many_types(torch_cuda):
    torch = torch_cuda
    limit = 16384
    P = [W.default_params()] * (limit + 1)
    T = bysdf.bysdf_types_create(P)
    off = torch.zeros(limit + 2, dtype=torch.int64, device="cuda")
    q = bysdf.to_device(W.queries(1, 72))
    out = bysdf.alloc_eval_out(1)
    with pytest.raises(RuntimeError, match="at most 16384 types"):
        bysdf.bysdf_eval_batched_noalloc(T, off, q, out)
