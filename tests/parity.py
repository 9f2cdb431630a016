"""Parity rule shared by the GPU tests.

A query counts when the oracle sets none of its margin flags (the query sits
within the rounding margin of one of the method's discrete decisions, or
the ply fixed point amplifies double rounding beyond 1e5).  On those
queries every floating-point output must satisfy
    |gpu - oracle| <= 1e-4 |oracle| + 1e-6
and the structural flags (pass-through, axial, back-facing, sample failure,
bad input) must agree exactly.
"""
import numpy as np

import oracle

REL = 1e-4
ABS = 1e-6
STRUCT = (oracle.PASS_THROUGH | oracle.AXIAL | oracle.BACKFACING | oracle.SAMPLE_FAIL
          | oracle.BAD_INPUT)


def compare(gpu, gflags, ref, rflags, extra_ok=None):
    """gpu, ref: [n, m] arrays; flags uint32 [n].  Returns a report dict."""
    gflags = np.asarray(gflags).view(np.uint32)
    ok = (rflags & oracle.MARGIN_MASK) == 0
    if extra_ok is not None:
        ok &= extra_ok
    tol = REL * np.abs(ref) + ABS
    err = np.abs(gpu - ref)
    bad = (err > tol) & ok[:, None]
    fmis = ((gflags & STRUCT) != (rflags & STRUCT)) & ok
    rel = err / np.maximum(np.abs(ref), ABS / REL)
    return dict(n=len(ok), counted=int(ok.sum()), flagged_share=float(1 - ok.mean()),
                n_bad=int(bad.any(1).sum()), n_flag_mismatch=int(fmis.sum()),
                bad_idx=np.nonzero(bad.any(1) | fmis)[0][:20],
                max_rel=float(rel[ok].max()) if ok.any() else 0.0)


def assert_parity(rep, max_flagged=0.02):
    assert rep["n_bad"] == 0 and rep["n_flag_mismatch"] == 0, rep
    assert rep["flagged_share"] <= max_flagged, rep


def fp64_sensitive(d, tab, h, u, v, wi, wo, ref, ulps=4):
    """True when moving h, u or v by `ulps` FP64 ulps moves the oracle's
    evaluation beyond the parity tolerance.  Such a query's value is not
    fixed to the tolerance by double-precision arithmetic: the rounding of
    any FP64 evaluation of it, the oracle's included, lands anywhere in that
    spread.  Used on the few queries that fail the rule, to tell these from
    real disagreements."""
    for k, x in enumerate((float(h), float(u), float(v))):
        for s in (-1.0, 1.0):
            a = [float(h), float(u), float(v)]
            a[k] = x + s * ulps * float(np.spacing(abs(x) if x != 0.0 else 1e-300))
            o, _ = oracle.eval_query(d, tab, a[0], a[1], a[2], wi, wo)
            if np.any(np.abs(o[:12] - ref[:12]) > REL * np.abs(ref[:12]) + ABS):
                return True
    return False


def fp64_sensitive_multi(d, tab, q, i, n_max, ref, ulps=4):
    """fp64_sensitive for the multi-scale evaluation of query i of q: u or
    v moved by `ulps` FP64 ulps (the strata heights are single precision by
    construction, so the footprint itself stays put)."""
    a = dict(h0=float(q["h"][i]), h1=float(q["h1"][i]), h2=float(q["h2"][i]), zeta=float(q["zeta"][i]),
             u=float(q["u"][i]), v=float(q["v"][i]))
    for k in ("u", "v"):
        for s in (-1.0, 1.0):
            b = dict(a)
            b[k] = a[k] + s * ulps * float(np.spacing(abs(a[k]) if a[k] != 0.0 else 1e-300))
            o, _ = oracle.eval_multi_query(d, tab, b["h0"], b["h1"], b["h2"], b["zeta"], n_max, b["u"],
                                           b["v"], q["wi"][:, i], q["wo"][:, i])
            if np.any(np.abs(o[:12] - ref[:12]) > REL * np.abs(ref[:12]) + ABS):
                return True
    return False


def furnace_draws_clear(P, q, block, nb, seed, rounds=8):
    """Furnace inputs whose draws sit on no margin: block b's draws all use
    the hit of its first query, and a draw whose direction the oracle flags
    (a lobe edge, a refraction next to the critical angle) gets fresh
    uniforms from a seeded generator, on both sides alike.  Returns (the
    modified query dict, per-block mask of blocks whose draws are all clear
    -- a block stays out only when its hit itself is flagged)."""
    q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in q.items()}
    qq = dict(q)
    for k in ("type", "h", "u", "v"):
        qq[k] = np.repeat(q[k][::block][:nb], block)
    qq["wi"] = np.repeat(q["wi"][:, ::block][:, :nb], block, axis=1)
    rng = np.random.Generator(np.random.Philox(key=seed))
    n = nb * block
    for _ in range(rounds):
        qq["xi"] = q["xi"][:, :n]
        _, sf = oracle.sample(P, qq)
        bad = (sf & oracle.MARGIN_MASK) != 0
        if not bad.any():
            break
        fresh = rng.random((3, int(bad.sum()))).astype(np.float32)
        q["xi"][:, :n][:, bad] = np.minimum(fresh, np.float32(1.0 - 2.0 ** -24))
    qq["xi"] = q["xi"][:, :n]
    _, sf = oracle.sample(P, qq)
    return q, ((sf & oracle.MARGIN_MASK) == 0).reshape(nb, block).all(1)
