"""The precision split of the kernels' model, checked on the host.

libbysdf_audit runs the kernels' per-query model (the templates of
bysdf_model.hpp) on the CPU with a geometry scalar that can round chosen
stages to single precision (tests/precision_audit.py).

* With no stage rounded it is the kernels' formulation in double: on the
  queries the oracle leaves unflagged it must agree with the oracle to the
  parity tolerance, structural flags included (a CPU-side check of the
  formulation, independent of the device's arithmetic sequences).
* Every stage the kernels keep in double must fail the tolerance somewhere
  when computed in single precision: that is the evidence for keeping it
  there (Sec. 3.4 phases and fixed point, Sec. 3.5 fiber frames, Sec. 4.1
  chords, refraction and half vectors, Sec. 4.1.4 the ply horizon,
  Sec. 4.1.5 drawn directions).
"""
import numpy as np
import pytest

import oracle
import precision_audit as A
from paper_2401_12724_amd import build as hip_build


@pytest.fixture(scope="module")
def sets():
    if hip_build.stale():
        hip_build.build()
    out = []
    for name, P, q in A.workloads(extended=True):
        q = A.with_xi(q)
        ref, rf = oracle.eval(P, q)
        sref, sf = oracle.sample(P, q)
        out.append((name, P, q, ref, rf, sref, sf))
    return out


def test_formulation_matches_oracle_in_double(sets):
    for name, P, q, ref, rf, sref, sf in sets:
        g, gf = A.audit_eval(P, q, 0)
        e = A.report(g.T, gf, ref[:, :12], rf)
        s, ssf = A.audit_sample(P, q, 0)
        r = A.report(s.T, ssf, sref[:, :7], sf)
        assert e["worst"] <= 1.0 and e["flag_mismatch"] == 0, (name, e)
        assert r["worst"] <= 1.0 and r["flag_mismatch"] == 0, (name, r)
        assert e["counted"] > 0.9 * len(q["h"]), (name, e)


def test_rounding_engages_only_in_its_stage(sets):
    """The mask changes the arithmetic of the selected stage only: the
    drawn-direction stage leaves the evaluation bit-identical, and the
    fixed point in single precision moves it."""
    name, P, q = sets[0][:3]
    g0, _ = A.audit_eval(P, q, 0)
    gs, _ = A.audit_eval(P, q, A.mask_of("sample"))
    assert np.array_equal(g0, gs)
    gp, _ = A.audit_eval(P, q, A.mask_of("plies"))
    assert not np.array_equal(g0, gp)


@pytest.mark.parametrize("stage", ["plies", "frame", "shadow", "refract", "chord", "half_x", "exit", "sample"])
def test_double_precision_stages_need_it(sets, stage):
    worst = 0.0
    for name, P, q, ref, rf, sref, sf in sets:
        m = A.mask_of(stage)
        g, gf = A.audit_eval(P, q, m)
        s, ssf = A.audit_sample(P, q, m)
        worst = max(worst, A.report(g.T, gf, ref[:, :12], rf)["worst"],
                    A.report(s.T, ssf, sref[:, :7], sf)["worst"])
        if worst > 1.0:
            break
    assert worst > 1.0, (stage, worst)
