"""The oracle's single-query evaluation with FP64 inputs, and the test-side
check that tells an ill-conditioned query (its value moves beyond the parity
tolerance when h, u or v moves by a few FP64 ulps) from a real disagreement."""
import numpy as np

import oracle
from paper_2401_12724_amd import workloads as W

from parity import fp64_sensitive, fp64_sensitive_multi


def test_eval_query_is_the_batched_evaluation():
    d = W.default_params(n_plies=5, ply_radius=W.packed_ply_radius(5), K=6)
    tab = oracle.table(d)
    q = W.queries(64, 5, with_xi=True, v_max=40.0)
    o, of = oracle.eval([d], q)
    for i in range(64):
        r, fl = oracle.eval_query(d, tab, float(q["h"][i]), float(q["u"][i]), float(q["v"][i]),
                                  q["wi"][:, i], q["wo"][:, i])
        assert fl == of[i]
        assert np.array_equal(r[:12], o[i, :12])


def test_sensitivity_check():
    # a well-conditioned workload: no query is sensitive
    d = W.default_params()
    tab = oracle.table(d)
    q = W.queries(300, 6)
    o, of = oracle.eval([d], q)
    ok = np.nonzero((of & oracle.MARGIN_MASK) == 0)[0]
    assert not any(fp64_sensitive(d, tab, q["h"][i], q["u"][i], q["v"][i], q["wi"][:, i],
                                  q["wo"][:, i], o[i]) for i in ok)
    # 8 plies of 256 fibers, 16 fixed-point steps, 4,096 texels: a query at
    # grazing incidence (wi_z = -0.97, v = 39.8) whose forward body lobe moves
    # by 8e-4 (relative) when h moves by 1e-15
    rp8 = W.packed_ply_radius(8)
    d = W.default_params(n_plies=8, ply_radius=rp8, ply_center_radius=1 - rp8, fibers_per_ply=256,
                         fiber_radius=0.03, K=16, n_iter=16, tex_size=4096)
    tab = oracle.table(d)
    q = W.queries(65536 + 77, 90, n_types=2, with_xi=True, v_max=40.0)
    i = 35747
    assert q["type"][i] == 0
    h, u, v, wi, wo = float(q["h"][i]), float(q["u"][i]), float(q["v"][i]), q["wi"][:, i], q["wo"][:, i]
    r0, fl = oracle.eval_query(d, tab, h, u, v, wi, wo)
    r1, _ = oracle.eval_query(d, tab, h + 1e-15, u, v, wi, wo)
    assert abs(r1[8] - r0[8]) > 5e-4 * abs(r0[8])
    assert fp64_sensitive(d, tab, h, u, v, wi, wo, r0)
    # ILLCOND prices the amplification per texel of the table: this query's
    # A |kappa| = 3.2e4 times 4,096 / 512 texels exceeds the 1e5 limit
    assert fl & oracle.ILLCOND


def _largest():
    rp8 = W.packed_ply_radius(8)
    return [W.default_params(n_plies=8, ply_radius=rp8, ply_center_radius=1 - rp8, fibers_per_ply=256,
                             fiber_radius=0.03, K=16, n_iter=16, tex_size=4096),
            W.default_params(mig_tables=8, mig_period=2.0, mig_blend=1.0, mig_spread=0.9, mig_seed=7,
                             tex_size=2048, fibers_per_ply=128, K=16, n_iter=16)]


def test_unflagged_queries_are_fixed_by_fp64():
    """At the largest accepted yarn types no query that the oracle leaves
    unflagged moves beyond the parity tolerance when h, u or v moves by a
    few FP64 ulps: the margin flags cover every query whose value double
    precision does not fix (every fourth query of the GPU parity workloads
    of those types)."""
    P = _largest()
    tabs = [oracle.table(d) for d in P]
    q = W.queries(65536 + 77, 90, n_types=2, with_xi=True, v_max=40.0)
    o, of = oracle.eval(P, q)
    idx = np.nonzero((of & oracle.MARGIN_MASK) == 0)[0][::4]
    assert len(idx) > 15000
    sens = [i for i in idx if fp64_sensitive(P[q["type"][i]], tabs[q["type"][i]], q["h"][i], q["u"][i],
                                             q["v"][i], q["wi"][:, i], q["wo"][:, i], o[i])]
    assert sens == []
    qm = W.footprints(W.queries(16384 + 33, 93, n_types=2, with_xi=True, v_max=40.0), 94)
    om, ofm = oracle.eval_multi(P, qm, 16)
    idx = np.nonzero((ofm & oracle.MARGIN_MASK) == 0)[0][::4]
    sens = [i for i in idx if fp64_sensitive_multi(P[qm["type"][i]], tabs[qm["type"][i]], qm, i, 16, om[i])]
    assert sens == []


def test_eval_multi_query_is_the_batched_evaluation():
    d = W.default_params(n_plies=5, ply_radius=W.packed_ply_radius(5), K=6)
    tab = oracle.table(d)
    q = W.footprints(W.queries(48, 7, with_xi=True, v_max=40.0), 8)
    o, of = oracle.eval_multi([d], q, 8)
    for i in range(48):
        r, fl = oracle.eval_multi_query(d, tab, float(q["h"][i]), float(q["h1"][i]), float(q["h2"][i]),
                                        float(q["zeta"][i]), 8, float(q["u"][i]), float(q["v"][i]),
                                        q["wi"][:, i], q["wo"][:, i])
        assert fl == of[i]
        assert np.array_equal(r[:12], o[i, :12])
