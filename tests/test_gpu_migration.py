"""GPU parity of fiber migration (Sec. 3.5.2) against the FP64 oracle: the
perturbed fiber tables, evaluation, sampling, the fused call, the furnace,
the batched kernel and the adjoint on types whose fiber tables switch and
blend along the ply."""
import numpy as np
import pytest

import oracle
from paper_2401_12724_amd import bysdf, workloads as W

from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _mig(**kw):
    return W.default_params(**dict(dict(mig_tables=4, mig_period=3.0, mig_blend=0.25,
                                        mig_spread=0.4, mig_seed=11), **kw))


def _mixed_types():
    return [_mig(), W.default_params(), _mig(mig_tables=2, mig_period=1.5, mig_blend=0.5, mig_seed=3),
            _mig(mig_tables=8, mig_spread=0.7, mig_blend=0.0, tex_size=256, fibers_per_ply=40),
            _mig(n_plies=5, ply_radius=W.packed_ply_radius(5), mig_seed=99, K=6)]


def test_migration_tables_match(torch_cuda):
    P = _mixed_types()
    T = bysdf.bysdf_types_create(P)
    for i, d in enumerate(P):
        g = bysdf.bysdf_types_table(T, i)
        o = oracle.table(d)
        assert g.shape == o.shape
        print("type", i, "tables", max(1, d["mig_tables"]), "max diff", np.abs(g - o).max(),
              "exact share", np.mean(g == o.astype(np.float32)))
        assert np.abs(g - o).max() <= 1e-6
        assert np.mean(g == o.astype(np.float32)) > 0.999


@pytest.mark.parametrize("case", ["single", "mixed"])
def test_migration_eval_sample(torch_cuda, case):
    torch = torch_cuda
    if case == "single":
        P = [_mig()]
        _, q = W.single_type(65536 + 19, 31, with_xi=True)
        q["v"] = (np.random.default_rng(32).random(len(q["h"])) * 40.0).astype(np.float32)
    else:
        P = _mixed_types()
        n = 2 * 65536 + 55
        q = W.queries(n, 33, n_types=len(P), with_xi=True, v_max=40.0)
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    ev, ef = bysdf.bysdf_eval(T, qd)
    sv, lobe, node, sf = bysdf.bysdf_sample_pdf(T, qd)
    fv, ff, gv, globe, gnode, gf = bysdf.bysdf_eval_sample(T, qd)
    torch.cuda.synchronize()
    o, of = oracle.eval(P, q)
    rep = compare(ev.cpu().numpy().T, ef.cpu().numpy(), o[:, :12], of)
    print(case, "eval", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.05)
    so, sof = oracle.sample(P, q)
    rep = compare(sv.cpu().numpy().T, sf.cpu().numpy(), so[:, :10], sof)
    print(case, "sample", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.05)
    ok = (sof & oracle.MARGIN_MASK) == 0
    assert np.array_equal(lobe.cpu().numpy()[ok], so[ok, 10].astype(np.int32))
    # the fused call computes the same values
    assert np.abs(fv.cpu().numpy() - ev.cpu().numpy()).max() <= 1e-5 * np.abs(ev.cpu().numpy()).max()
    assert np.abs(gv.cpu().numpy() - sv.cpu().numpy()).max() <= 1e-5 * np.abs(sv.cpu().numpy()).max()


def test_migration_furnace_and_batched(torch_cuda):
    torch = torch_cuda
    P = [_mig()]
    _, q = W.single_type(256 * 128, 34, with_xi=True)
    q["v"] = (np.random.default_rng(35).random(len(q["h"])) * 40.0).astype(np.float32)
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    mean, var = bysdf.bysdf_furnace_blocks(T, qd, 256)
    torch.cuda.synchronize()
    om, ov = oracle.furnace(P, q, 256)
    nb = len(om)
    qq = dict(q)
    for k in ("type", "h", "u", "v"):
        qq[k] = np.repeat(q[k][::256][:nb], 256)
    qq["wi"] = np.repeat(q["wi"][:, ::256][:, :nb], 256, axis=1)
    _, sf = oracle.sample(P, qq)
    blk = ((sf & oracle.MARGIN_MASK) == 0).reshape(nb, 256).all(1)
    assert blk.sum() > nb // 2
    gm = mean.cpu().numpy()
    assert np.all((np.abs(gm - om) <= 1e-4 * np.abs(om) + 1e-6)[blk])
    # batched kernel: types sorted by count, tables staged in LDS and not
    P2 = _mixed_types()
    counts = np.array([3000, 257, 9000, 1, 4100])
    off = np.zeros(len(P2) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    tid = np.repeat(np.arange(len(P2), dtype=np.int32), counts)
    q2 = W.queries(int(off[-1]), 36, type_ids=tid, v_max=40.0)
    T2 = bysdf.bysdf_types_create(P2)
    vals, flags = bysdf.bysdf_eval_batched(T2, torch.from_numpy(off).cuda(), bysdf.to_device(q2))
    torch.cuda.synchronize()
    o, of = oracle.eval(P2, q2)
    rep = compare(vals.cpu().numpy().T, flags.cpu().numpy(), o[:, :12], of)
    print("batched", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.05)


def test_migration_adjoint_matches_fd(torch_cuda):
    """Gradients through the blended tables (the blend weight moves with the
    ply arc length, which the ply twist changes)."""
    torch = torch_cuda
    P = [_mig(), _mig(mig_tables=3, mig_period=2.0, mig_blend=0.6, mig_seed=5)]
    per = 4096
    tid = np.repeat(np.arange(2, dtype=np.int32), per)
    q = W.queries(2 * per, 37, type_ids=tid, v_max=20.0)
    off = np.array([0, per, 2 * per], dtype=np.int64)
    gE = np.random.default_rng(38).normal(size=(2 * per, 3)).astype(np.float32)
    ts = oracle.TypeSet(P)
    _, a = oracle.grad_fd(ts, q, gE, 1e-7)
    _, b = oracle.grad_fd(ts, q, gE, 3e-8)
    _, fl = oracle.eval(ts, q)
    ok = np.all(np.abs(a - b) <= 1e-4 * np.maximum(np.abs(a), 1e-7) + 1e-9, axis=1)
    ok &= (fl & oracle.MARGIN_MASK) == 0
    assert ok.mean() > 0.85, ok.mean()
    T = bysdf.bysdf_types_create(P)
    _, pq = bysdf.bysdf_eval_backward(T, bysdf.to_device(q), torch.from_numpy(off).cuda(),
                                      torch.from_numpy(gE).cuda(), per_query=True)
    torch.cuda.synchronize()
    pq = pq.cpu().numpy()
    tol = 1e-3 * np.abs(a) + 1e-6 * np.abs(a).max(0)
    bad = (np.abs(pq - a) > tol) & ok[:, None]
    print("per-query bad", bad.sum(0), "of", ok.sum())
    assert not bad.any()
