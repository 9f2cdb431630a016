"""Sampler pins (Sec. 4.1.5): the directions the sampler draws follow the
mixture pdf it reports (chi-square on sphere bins), its weights equal E/pdf,
and the pdf integrates to one minus the probability of a failed draw."""
import math

import numpy as np
import pytest

from paper_2401_12724_amd import workloads as W


def _rep(qi, n, wo=None, xi=None):
    q = dict(type=np.zeros(n, np.int32), h=np.full(n, qi["h"], np.float32),
             u=np.full(n, qi["u"], np.float32), v=np.full(n, qi["v"], np.float32),
             wi=np.repeat(qi["wi"][:, None], n, 1).astype(np.float32))
    if wo is not None:
        q["wo"] = np.ascontiguousarray(wo, dtype=np.float32)
    if xi is not None:
        q["xi"] = np.ascontiguousarray(xi, dtype=np.float32)
    return q


def _queries(oracle_mod, P, seed, k):
    _, q = W.single_type(300, seed)
    out, fl = oracle_mod.eval(P, q)
    idx = [i for i in range(300) if not fl[i] & (oracle_mod.PASS_THROUGH | oracle_mod.MARGIN_MASK
                                                 | oracle_mod.BACKFACING)]
    return [dict(h=q["h"][i], u=q["u"][i], v=q["v"][i], wi=q["wi"][:, i]) for i in idx[:k]]


def _chi2_quantile(dof, z=3.29):
    return dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3


@pytest.mark.parametrize("beta,seed", [(0.3, 21), (0.15, 22)])
def test_sampler_chi_square(oracle_mod, beta, seed):
    P = [W.default_params(beta=beta)]
    ts = oracle_mod.TypeSet(P)
    N = 200000
    nz, nph, sub = 32, 64, 6
    for qi in _queries(oracle_mod, P, seed, 2):
        rng = np.random.default_rng(seed)
        xi = np.minimum(rng.random((3, N)), 1 - 2 ** -24).astype(np.float32)
        so, sf = oracle_mod.sample(ts, _rep(qi, N, xi=xi))
        ok = (sf & oracle_mod.SAMPLE_FAIL) == 0
        wo = so[ok, :3]
        zi = np.minimum(((1 - wo[:, 2]) / 2 * nz).astype(int), nz - 1)
        pi_ = np.minimum(((np.arctan2(wo[:, 1], wo[:, 0]) % (2 * math.pi)) / (2 * math.pi) * nph)
                         .astype(int), nph - 1)
        obs = np.zeros((nz, nph))
        np.add.at(obs, (zi, pi_), 1)
        # expected counts: sub-quadrature of the reported pdf in each bin
        zz = 1 - 2 * (np.arange(nz * sub) + 0.5) / (nz * sub)
        pp = 2 * math.pi * (np.arange(nph * sub) + 0.5) / (nph * sub)
        Z, PH = np.meshgrid(zz, pp, indexing="ij")
        s = np.sqrt(1 - Z * Z)
        d = np.stack([s * np.cos(PH), s * np.sin(PH), Z]).reshape(3, -1)
        out, _ = oracle_mod.eval(ts, _rep(qi, d.shape[1], wo=d))
        pdf = out[:, 11].reshape(nz * sub, nph * sub)
        dw = (2.0 / (nz * sub)) * (2 * math.pi / (nph * sub))
        expb = pdf.reshape(nz, sub, nph, sub).sum((1, 3)) * dw * N
        total = pdf.sum() * dw
        # fail mass: the share of draws the sampler rejects
        fail = 1.0 - ok.mean()
        assert abs((1.0 - fail) - total) < 4e-3 + 4 * math.sqrt(fail * (1 - fail) / N)
        m = expb > 30
        chi2 = (((obs[m] - expb[m]) ** 2) / expb[m]).sum()
        dof = int(m.sum()) - 1
        assert chi2 < _chi2_quantile(dof), (chi2, dof)


def test_weight_is_value_over_pdf(oracle_mod):
    P = [W.default_params()]
    ts = oracle_mod.TypeSet(P)
    _, q = W.single_type(20000, 23, with_xi=True)
    so, sf = oracle_mod.sample(ts, q)
    ok = (sf & (oracle_mod.SAMPLE_FAIL | oracle_mod.PASS_THROUGH | oracle_mod.BAD_INPUT)) == 0
    qq = dict(q)
    qq["wo"] = np.ascontiguousarray(so[:, :3].T.astype(np.float32))
    e, ef = oracle_mod.eval(ts, qq)
    # wo rounds to FP32 on the way back into eval: compare where the value is
    # insensitive to that rounding
    good = ok & ((ef & oracle_mod.MARGIN_MASK) == 0)
    rel = np.abs(so[good, 3:6] * so[good, 6:7] - e[good, :3]) / np.maximum(e[good, :3], 1e-12)
    assert np.median(rel) < 1e-5
    assert np.all(so[good, 6] > 0)
    # pass-through draws continue straight through with unit weight
    ps = (sf & oracle_mod.PASS_THROUGH) != 0
    assert np.allclose(so[ps, :3], -q["wi"][:, ps].T, atol=1e-7)
    assert np.all(so[ps, 3:6] == 1.0) and np.all(so[ps, 10] == 4)


def test_furnace_blocks(oracle_mod):
    """Per-block furnace means stay below 1 + 3 sigma; with B = 1, no occlusion
    and albedo 1 every non-pass block integrates to exactly 1 (weights are
    constant up to the LS / Lambert mixture)."""
    P = [W.default_params()]
    _, q = W.single_type(256 * 64, 24, with_xi=True)
    mean, var = oracle_mod.furnace(P, q, 256)
    assert np.all(mean <= 1.0 + 3 * np.sqrt(var / 256) + 1e-12)
    P1 = [W.default_params(albedo=(1.0, 1.0, 1.0), B=1.0, ply_density=0.0, fiber_density=0.0)]
    m1, v1 = oracle_mod.furnace(P1, q, 256)
    assert np.all(np.abs(m1 - 1.0) <= 3 * np.sqrt(v1 / 256) + 1e-9)
