"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sizes span many 256-query workgroups with ragged tails; the full-size
per-block workload (2^24 queries) is checked on a random sample of outputs
in the launch configuration the benchmark times.
"""
import numpy as np
import pytest

import oracle
from paper_2401_12724_amd import build as hip_build
from paper_2401_12724_amd import bysdf, workloads as W

from parity import assert_parity, compare, furnace_draws_clear

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    if not __import__("os").path.exists(hip_build.LIB):
        hip_build.build()
    return torch


def _eval_gpu(torch, P, q):
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    vals, flags = bysdf.bysdf_eval(T, qd)
    torch.cuda.synchronize()
    return vals.cpu().numpy().T, flags.cpu().numpy().view(np.uint32)


def _sample_gpu(torch, P, q):
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    vals, lobe, node, flags = bysdf.bysdf_sample_pdf(T, qd)
    torch.cuda.synchronize()
    return (vals.cpu().numpy().T, lobe.cpu().numpy(), node.cpu().numpy(),
            flags.cpu().numpy().view(np.uint32))


def test_fiber_tables_match(torch_cuda):
    """Device FP64 table build against the oracle's tables (both rounded to
    single precision texels)."""
    P = [W.default_params(fibers_per_ply=m, fiber_radius=r, tex_size=nu)
         for m, r, nu in [(64, 0.06, 512), (32, 0.06, 512), (128, 0.06, 512), (7, 0.2, 100)]]
    T = bysdf.bysdf_types_create(P)
    for i, d in enumerate(P):
        g = bysdf.bysdf_types_table(T, i)
        o = oracle.table(d)
        dif = np.abs(g - o)
        k = np.unravel_index(np.argmax(dif), dif.shape)
        print("table", i, "max diff", dif.max(), "at", k, g[k[0]], o[k[0]],
              "exact share", np.mean(g == o.astype(np.float32)))
        assert np.max(np.abs(g - o)) <= 1e-6
        assert np.mean(g == o.astype(np.float32)) > 0.999


@pytest.mark.parametrize("beta", [0.05, 0.15, 0.3])
def test_eval_single_type(torch_cuda, beta):
    P = [W.default_params(beta=beta)]
    _, q = W.single_type(65536, 0)
    g, gf = _eval_gpu(torch_cuda, P, q)
    o, of = oracle.eval(P, q)
    rep = compare(g, gf, o[:, :12], of)
    print("beta", beta, {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep)


def test_eval_heterogeneous_types_ragged(torch_cuda):
    """Many types (1..8 plies, 1..16 nodes, assorted fiber counts and table
    sizes, anisotropic roughness, lattice shifts) in one call with a ragged
    tail; exercises the global-memory table path."""
    rng = np.random.default_rng(42)
    P = []
    for t in range(24):
        npl = int(rng.integers(1, 9))
        rp = W.packed_ply_radius(npl)
        P.append(W.default_params(
            n_plies=npl, ply_radius=rp, ply_center_radius=1 - rp if npl > 1 else 0.0,
            fibers_per_ply=int(rng.integers(8, 160)), K=int(rng.integers(1, 17)),
            n_iter=int(rng.integers(0, 8)), tex_size=int(rng.choice([64, 256, 512, 1024])),
            ply_twist=float(rng.uniform(-0.7, 0.7)), fiber_twist=float(rng.uniform(-0.7, 0.7)),
            beta=float(rng.uniform(0.05, 0.5)), aniso=float(rng.uniform(0.5, 2.0)),
            B=float(rng.uniform(0, 1)), r=float(rng.uniform(0, 1)),
            sigma_t=float(rng.uniform(0, 2)), ply_density=float(rng.uniform(0, 1)),
            fiber_density=float(rng.uniform(0, 1)), eta=float(rng.uniform(1.2, 1.8))))
    n = 3 * 65536 + 123
    q = W.queries(n, 7, n_types=len(P), v_max=40.0)
    q["shift"] = np.random.default_rng(8).random((2, n)).astype(np.float32)
    g, gf = _eval_gpu(torch_cuda, P, q)
    o, of = oracle.eval(P, q)
    rep = compare(g, gf, o[:, :12], of)
    print({k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.05)


def test_sample_single_type(torch_cuda):
    P = [W.default_params()]
    _, q = W.single_type(65536 + 17, 5, with_xi=True)
    g, lobe, node, gf = _sample_gpu(torch_cuda, P, q)
    o, of = oracle.sample(P, q)
    rep = compare(g, gf, o[:, :10], of)
    print({k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.03)
    ok = (of & oracle.MARGIN_MASK) == 0
    assert np.array_equal(lobe[ok], o[ok, 10].astype(np.int32))
    fw = ok & ((lobe == 1) | (lobe == 3))
    assert np.array_equal(node[fw], o[fw, 11].astype(np.int32))


def _hetero_types(seed, n_types=24):
    rng = np.random.default_rng(seed)
    P = []
    for t in range(n_types):
        npl = int(rng.integers(1, 9))
        rp = W.packed_ply_radius(npl)
        P.append(W.default_params(
            n_plies=npl, ply_radius=rp, ply_center_radius=1 - rp if npl > 1 else 0.0,
            fibers_per_ply=int(rng.integers(8, 160)), K=int(rng.integers(1, 17)),
            n_iter=int(rng.integers(0, 8)), tex_size=int(rng.choice([64, 256, 512, 1024])),
            beta=float(rng.uniform(0.05, 0.5)), aniso=float(rng.uniform(0.5, 2.0)),
            B=float(rng.uniform(0, 1)), r=float(rng.uniform(0, 1)),
            sigma_t=float(rng.uniform(0, 2)), eta=float(rng.uniform(1.2, 1.8))))
    return P


@pytest.mark.parametrize("case", ["single", "hetero"])
def test_eval_sample_fused(torch_cuda, case):
    """bysdf_eval_sample: the eval half against the oracle's eval and the
    sample half against the oracle's sampler on the same queries, and both
    against the separate entry points (same model code, so equal up to the
    compiler's operation order).  Some wo are made invalid: only the eval
    half may flag them."""
    torch = torch_cuda
    if case == "single":
        P = [W.default_params()]
        _, q = W.single_type(65536 + 41, 13, with_xi=True)
    else:
        P = _hetero_types(43)
        n = 2 * 65536 + 77
        q = W.queries(n, 17, n_types=len(P), v_max=40.0)
        rng = np.random.default_rng(18)
        q["xi"] = np.minimum(rng.random((3, n)).astype(np.float32), np.float32(1.0 - 2.0 ** -24))
        q["shift"] = rng.random((2, n)).astype(np.float32)
    n = len(q["h"])
    q["wo"] = np.array(q["wo"], dtype=np.float32, copy=True)
    q["wo"][:, 5:n:997] = np.nan
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    ev, ef, sv, lobe, node, sf = bysdf.bysdf_eval_sample(T, qd)
    ev2, ef2 = bysdf.bysdf_eval(T, qd)
    sv2, lobe2, node2, sf2 = bysdf.bysdf_sample_pdf(T, qd)
    torch.cuda.synchronize()
    ev, ef, sv, sf = ev.cpu().numpy().T, ef.cpu().numpy().view(np.uint32), sv.cpu().numpy().T, \
        sf.cpu().numpy().view(np.uint32)
    lobe, node = lobe.cpu().numpy(), node.cpu().numpy()
    bad_wo = np.zeros(n, bool)
    bad_wo[5:n:997] = True
    assert np.all(ef[bad_wo] & oracle.BAD_INPUT)
    assert not np.any(sf[bad_wo] & oracle.BAD_INPUT)
    # against the separate entry points
    ev2, ef2 = ev2.cpu().numpy().T, ef2.cpu().numpy().view(np.uint32)
    sv2, sf2 = sv2.cpu().numpy().T, sf2.cpu().numpy().view(np.uint32)
    assert np.array_equal(ef, ef2) and np.array_equal(sf, sf2)
    assert np.array_equal(lobe, lobe2.cpu().numpy()) and np.array_equal(node, node2.cpu().numpy())
    for a, b, label in ((ev, ev2, "eval"), (sv, sv2, "sample")):
        rel = np.abs(a - b) / (np.abs(b) + 1e-6)
        print(case, label, "equal share", np.mean(a == b), "max rel", rel.max())
        assert rel.max() <= 1e-5, label
    # against the oracle
    o, of = oracle.eval(P, q)
    rep = compare(ev, ef, o[:, :12], of)
    print(case, "eval", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.05)
    so, sof = oracle.sample(P, q)
    rep = compare(sv, sf, so[:, :10], sof)
    print(case, "sample", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.05)
    ok = (sof & oracle.MARGIN_MASK) == 0
    assert np.array_equal(lobe[ok], so[ok, 10].astype(np.int32))


def test_furnace_blocks(torch_cuda):
    """Per-block white-furnace mean and variance (Sec. 4.3) against the
    oracle.  Draws whose direction sits on a margin get fresh uniforms on
    both sides; only blocks whose hit itself is flagged stay out."""
    P = [W.default_params()]
    nb = 512
    _, q = W.single_type(256 * nb, 9, with_xi=True)
    q, blk_ok = furnace_draws_clear(P, q, 256, nb, 900)
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    mean, var = bysdf.bysdf_furnace_blocks(T, qd, 256)
    torch_cuda.cuda.synchronize()
    gm, gv = mean.cpu().numpy(), var.cpu().numpy()
    om, ov = oracle.furnace(P, q, 256)
    assert blk_ok.mean() >= 0.95
    assert np.all((np.abs(gm - om) <= 1e-4 * np.abs(om) + 1e-6)[blk_ok])
    assert np.all((np.abs(gv - ov) <= 1e-4 * np.abs(ov) + 1e-6)[blk_ok])
    # bitwise reproducible
    mean2, var2 = bysdf.bysdf_furnace_blocks(T, qd, 256)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(mean2.cpu().numpy(), gm) and np.array_equal(var2.cpu().numpy(), gv)


@pytest.mark.parametrize("block", [64, 192, 512, 1024])
def test_furnace_block_sizes(torch_cuda, block):
    """Blocks of up to 256 draws run one wavefront per block (1-4 draws per
    lane, a partial last workgroup), larger ones one workgroup per block:
    both against the oracle on 37 blocks of a mixed-type batch."""
    P = [W.default_params(), W.default_params(beta=0.1, albedo=(0.9, 0.6, 0.3))]
    nb = 37
    q = W.queries(block * nb, 19, n_types=2, with_xi=True)
    # one type per block (the block's first query decides)
    q["type"] = np.repeat(q["type"][::block][:nb], block).astype(np.int32)
    q, blk_ok = furnace_draws_clear(P, q, block, nb, 901)
    T = bysdf.bysdf_types_create(P)
    mean, var = bysdf.bysdf_furnace_blocks(T, bysdf.to_device(q), block)
    torch_cuda.cuda.synchronize()
    gm, gv = mean.cpu().numpy(), var.cpu().numpy()
    om, ov = oracle.furnace(P, q, block)
    assert blk_ok.sum() >= nb - 1
    assert np.all((np.abs(gm - om) <= 1e-4 * np.abs(om) + 1e-6)[blk_ok])
    assert np.all((np.abs(gv - ov) <= 1e-4 * np.abs(ov) + 1e-6)[blk_ok])


def test_sampler_draws_its_own_uniforms(torch_cuda):
    """Without xi arrays the sampler and the furnace draw their uniforms
    from Philox4x32-10 keyed by the seed (counter = query index): the same
    as the oracle given those draws, generated on the host."""
    P = [W.default_params()]
    n = 256 * 64 + 77
    q = W.queries(n, 23)
    T = bysdf.bysdf_types_create(P)
    seed = 0x9E3779B97F4A7C15
    qd = bysdf.to_device(q)
    qd["seed"] = seed
    sv, lobe, node, sf = bysdf.bysdf_sample_pdf(T, qd)
    mean, var = bysdf.bysdf_furnace_blocks(T, qd, 256)
    torch_cuda.cuda.synchronize()
    qx = dict(q, xi=W.sampler_xi(n, seed))
    so, sof = oracle.sample(P, qx)
    rep = compare(sv.cpu().numpy().T, sf.cpu().numpy(), so[:, :10], sof)
    print("sample (own draws)", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.03)
    ok = (sof & oracle.MARGIN_MASK) == 0
    assert np.array_equal(lobe.cpu().numpy()[ok], so[ok, 10].astype(np.int32))
    om, ov = oracle.furnace(P, qx, 256)
    nb = n // 256
    qq = dict(qx)
    for k in ("type", "h", "u", "v"):
        qq[k] = np.repeat(qx[k][::256][:nb], 256)
    qq["wi"] = np.repeat(qx["wi"][:, ::256][:, :nb], 256, axis=1)
    qq["xi"] = qx["xi"][:, :nb * 256]
    _, bsf = oracle.sample(P, qq)
    blk = ((bsf & oracle.MARGIN_MASK) == 0).reshape(nb, 256).all(1)
    gm, gv = mean.cpu().numpy(), var.cpu().numpy()
    assert np.all((np.abs(gm - om) <= 1e-4 * np.abs(om) + 1e-6)[blk])
    assert np.all((np.abs(gv - ov) <= 1e-4 * np.abs(ov) + 1e-6)[blk])
    # every block, flagged draws included: the furnace's mean is the mean of
    # the sampler's weights at the block's hit under the same Philox draws,
    # and those weights follow the parity rule draw by draw
    qqd = bysdf.to_device({k: v for k, v in qq.items() if k != "xi"})
    qqd["seed"] = seed
    bv, _, _, bf = bysdf.bysdf_sample_pdf(T, qqd)
    torch_cuda.cuda.synchronize()
    bw = bv.cpu().numpy()[3:6].reshape(3, nb, 256).astype(np.float64)
    assert np.all(np.abs(gm - bw.mean(2).T) <= 2e-6 * np.abs(gm) + 1e-7)
    rep = compare(bv.cpu().numpy().T, bf.cpu().numpy(), oracle.sample(P, qq)[0][:, :10], bsf)
    assert_parity(rep, max_flagged=0.05)


def test_edge_cases(torch_cuda):
    torch = torch_cuda
    P = [W.default_params()]
    T = bysdf.bysdf_types_create(P)
    # n = 0 is a no-op
    q0 = bysdf.to_device(W.queries(0, 1))
    bysdf.bysdf_eval(T, q0)
    # bad inputs: NaN, |h| > 1, non-unit directions, axial incidence, bad type
    q = W.queries(8, 2, with_xi=True)
    q["h"][0] = np.nan
    q["h"][1] = 1.5
    q["wi"][:, 2] = [2.0, 0.0, 0.0]
    q["wo"][:, 3] = [np.inf, 0.0, 0.0]
    q["wi"][:, 4] = [0.0, 0.0, 1.0]
    q["type"][5] = 3
    q["h"][6] = 1.0
    q["h"][7] = -1.0
    g, gf = _eval_gpu(torch, P, q)
    o, of = oracle.eval(P, q)
    for i in (0, 1, 2, 3, 5):
        assert gf[i] & bysdf.FLAG_BAD_INPUT and np.all(g[i] == 0.0)
        assert of[i] & oracle.BAD_INPUT
    assert gf[4] & bysdf.FLAG_AXIAL and gf[4] & bysdf.FLAG_PASS_THROUGH and np.all(g[4] == 0)
    rep = compare(g[6:], gf[6:], o[6:, :12], of[6:])
    assert rep["n_bad"] == 0
    s, lobe, node, sf = _sample_gpu(torch, P, q)
    assert sf[4] & bysdf.FLAG_PASS_THROUGH and lobe[4] == 4
    assert np.allclose(s[4, :3], -q["wi"][:, 4]) and np.all(s[4, 3:6] == 1.0)
    for i in (0, 1, 2, 5):
        assert sf[i] & bysdf.FLAG_BAD_INPUT and lobe[i] == -1
    # long yarns: v of hundreds of yarn radii keeps its phase accuracy
    qv = W.queries(20000, 3, v_max=2000.0)
    g, gf = _eval_gpu(torch, P, qv)
    o, of = oracle.eval(P, qv)
    assert_parity(compare(g, gf, o[:, :12], of))


def test_deterministic(torch_cuda):
    P = [W.default_params()]
    _, q = W.single_type(50000, 11, with_xi=True)
    a = _eval_gpu(torch_cuda, P, q)
    b = _eval_gpu(torch_cuda, P, q)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_full_size_per_block_sampled(torch_cuda):
    """The benchmark workload in the benchmark's launches: 2^24 queries in
    65,536 parameter blocks of 256 (beta and albedo per block) through
    bysdf_eval_sample (value at wo, one sampled direction with weight and
    pdf) and bysdf_furnace_blocks, checked on a random sample of 12,000
    queries and 64 furnace blocks."""
    torch = torch_cuda
    P, q = W.per_block(65536, 256, seed=1)
    T = bysdf.bysdf_types_create(P)
    qd = bysdf.to_device(q)
    ev, ef, sv, lobe, node, sf = bysdf.bysdf_eval_sample(T, qd)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(0).choice(len(q["h"]), 12000, replace=False))
    sub = {k: (v[..., idx] if v is not None else None) for k, v in q.items()}
    ts = oracle.TypeSet(P)
    o, of = oracle.eval(ts, sub)
    rep = compare(ev[:, idx].cpu().numpy().T, ef[idx].cpu().numpy(), o[:, :12], of)
    print("eval", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep)
    so, sof = oracle.sample(ts, sub)
    rep = compare(sv[:, idx].cpu().numpy().T, sf[idx].cpu().numpy(), so[:, :10], sof)
    print("sample", {k: v for k, v in rep.items() if k != "bad_idx"})
    assert_parity(rep, max_flagged=0.03)
    # furnace blocks: the oracle on whole blocks gathered from the workload
    blocks = np.sort(np.random.default_rng(1).choice(65536, 64, replace=False))
    rows = (blocks[:, None] * 256 + np.arange(256)[None, :]).ravel()
    qb = {k: (v[..., rows] if v is not None else None) for k, v in q.items()}
    # draws whose direction sits on a margin get fresh uniforms on both
    # sides: the sampled blocks' uniforms are replaced in the full-size input
    # and the furnace is run again over all 65,536 blocks
    qb, blk_ok = furnace_draws_clear(ts, qb, 256, len(blocks), 902)
    assert blk_ok.mean() >= 0.95
    xi = q["xi"].copy()
    xi[:, rows] = qb["xi"]
    qd["xi"] = torch.from_numpy(np.ascontiguousarray(xi)).cuda()
    mean, var = bysdf.bysdf_furnace_blocks(T, qd, 256)
    torch.cuda.synchronize()
    om, ov = oracle.furnace(ts, qb, 256)
    gm, gv = mean.cpu().numpy()[blocks], var.cpu().numpy()[blocks]
    assert np.all((np.abs(gm - om) <= 1e-4 * np.abs(om) + 1e-6)[blk_ok])
    assert np.all((np.abs(gv - ov) <= 1e-4 * np.abs(ov) + 1e-6)[blk_ok])
