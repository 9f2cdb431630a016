"""Pins of the forward-specular lobe and of the energy bookkeeping, on the
oracle.

* Sec. 4.1.2, Eq. 3, smooth limit: as the roughness goes to zero the exit
  BTDF becomes a delta in Snell's direction that carries the Fresnel
  transmittance of the exit, so int E_yS d omega_o = (1 - B) k_S T att
  (1 - F_in) for one node, and the lobe is centred on the refracted
  direction.
* Sec. 4.1.1: each node's weight T_k is the Fresnel transmittance times the
  masking of the refracted direction by the normal that refracts omega_i
  into omega_t,k (the generalised half vector of Walter et al. 2007, which
  also obeys Snell's law).
* Sec. 4.3, at finite roughness: the cosine-weighted integral of a
  microfacet lobe over outgoing directions equals the mean, over the
  normals visible from the incident direction, of the Fresnel factor times
  the masking of the outgoing direction (the change of variables to the
  half vector; Walter et al. 2007, Heitz 2014).  Hence
  int E d omega_o = (1 - B) k_S [A_R + 1/K sum_k T_k att_k A_T,k] + B G_p G_f k
  with the reflection albedo A_R at x and the exit albedos A_T,k computed
  here in microfacet-normal space, independently of the oracle's
  direction-space lobes.
"""
import math

import numpy as np
import pytest

from paper_2401_12724_amd import workloads as W

import microfacet_ref as M


def _query(q, i, n=None):
    return {k: (v[..., i] if k != "type" else v[i]) for k, v in q.items()}


def _clear(orc, fl):
    return not fl & (orc.PASS_THROUGH | orc.MARGIN_MASK | orc.BACKFACING)


def _eval_dirs(orc, P, qi, dirs):
    """The oracle's outputs for one hit at many outgoing directions."""
    n = dirs.shape[1]
    qq = dict(type=np.zeros(n, np.int32), h=np.full(n, qi["h"], np.float32),
              u=np.full(n, qi["u"], np.float32), v=np.full(n, qi["v"], np.float32),
              wi=np.repeat(np.asarray(qi["wi"], np.float32).reshape(3, 1), n, 1),
              wo=np.ascontiguousarray(dirs, dtype=np.float32))
    return orc.eval(P, qq)[0]


def _sphere_grid(nt=900, npp=1800):
    mu = 1.0 - 2.0 * (np.arange(nt) + 0.5) / nt
    ph = 2 * math.pi * (np.arange(npp) + 0.5) / npp
    Mu, Ph = np.meshgrid(mu, ph, indexing="ij")
    s = np.sqrt(1 - Mu * Mu)
    d = np.stack([s * np.cos(Ph), s * np.sin(Ph), Mu]).reshape(3, -1)
    return d, (2.0 / nt) * (2 * math.pi / npp)


def test_primitives_match_oracle(oracle_mod):
    """The vectorised primitives the pins use are the oracle's (pinned by
    closed forms in test_oracle_closed_forms)."""
    rng = np.random.default_rng(40)
    for _ in range(200):
        c = rng.uniform(0, 1)
        for e in (1.55, 1 / 1.55):
            assert abs(M.fresnel(c, e) - oracle_mod.fresnel(c, e)) < 1e-14
        a = rng.uniform(0.01, 0.5)
        m = rng.normal(size=3)
        m[2] = abs(m[2])
        m /= np.linalg.norm(m)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        assert abs(M.ggx_D(m[2], m[0] ** 2 + m[1] ** 2, a) - oracle_mod.ggx_D(m, a, a)) < 1e-9 * M.ggx_D(
            m[2], m[0] ** 2 + m[1] ** 2, a) + 1e-14
        g = M.smith_G1(w.reshape(3, 1), m.reshape(3, 1), a)[0]
        assert abs(g - oracle_mod.smith_G1(w, m, a, a)) < 1e-14


@pytest.mark.parametrize("wz", [1.0, 0.6, 0.15, 0.03])
def test_visible_normals_normalised(wz):
    """int D_w(m) dm = 1 for Smith's G1 at any view, grazing included: the
    quadrature the identities below rely on resolves the visible normals."""
    w = np.array([math.sqrt(1 - wz * wz), 0.0, wz])
    for a in (0.05, 0.15, 0.3):
        _, tot = M.visible_normal_mean(w, a, lambda m: np.ones(m.shape[1]))
        assert abs(tot - 1.0) < 2e-5, (wz, a, tot)


def _exit_nodes(orc, d, q, n_want, min_ct=0.3):
    """(query, node row) pairs with a clear hit whose exit refraction is
    well inside the critical angle (transmitted cosine >= min_ct)."""
    ts = orc.TypeSet([d])
    _, fl = orc.eval([d], q)
    eta = d["eta"]
    found = []
    for i in range(len(fl)):
        if not _clear(orc, fl[i]):
            continue
        qi = _query(q, i)
        wi = np.asarray(qi["wi"], np.float64)
        nd, f2 = orc.nodes(d, ts.tables[0], qi["h"], qi["u"], qi["v"], wi)
        if f2 & orc.MARGIN_MASK or nd[0, 4] <= 0.0:
            continue
        c = float(nd[0, 5:8] @ nd[0, 11:14])  # wi'.n' with wi' = -wt, n' = -n_y
        s2 = eta * eta * (1 - c * c)
        if s2 >= 1.0 or math.sqrt(1 - s2) < min_ct:
            continue
        found.append((qi, nd[0]))
        if len(found) == n_want:
            break
    return found


def smooth_limit_errors(orc, n_nodes=5):
    """Relative error of int E_yS against T att (1 - F_in) and the angle
    between the lobe's centroid and Snell's direction, for one-node hits at
    roughness 1e-3 (B = 0: only the specular lobes)."""
    beta = 1e-3
    d = W.default_params(K=1, B=0.0, beta=beta)
    eta = d["eta"]
    _, q = W.single_type(400, 21)
    rows = []
    for qi, nd in _exit_nodes(orc, d, q, n_nodes):
        wt, ny, att, T = nd[5:8], nd[11:14], nd[3], nd[4]
        wip, nin = -wt, -ny
        c = float(wip @ nin)
        ct = math.sqrt(1 - eta * eta * (1 - c * c))
        snell = -eta * wip + (eta * c - ct) * nin
        # polar grid about Snell's direction, dense near it: theta = bs tan(pi s / 2)
        bs, ns, nph = 5 * beta, 3000, 720
        smax = (2 / math.pi) * math.atan(math.pi / bs)
        s = (np.arange(ns) + 0.5) / ns * smax
        th = bs * np.tan(math.pi * s / 2)
        dth = bs * (math.pi / 2) / np.cos(math.pi * s / 2) ** 2 * (smax / ns)
        ph = 2 * math.pi * (np.arange(nph) + 0.5) / nph
        TH, PH = np.meshgrid(th, ph, indexing="ij")
        loc = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)]).reshape(3, -1)
        dirs = M.local_frame(snell).T @ loc
        wgt = (np.sin(TH) * dth[:, None] * (2 * math.pi / nph)).reshape(-1)
        eys = _eval_dirs(orc, [d], qi, dirs)[:, 4]
        integ = float((eys * wgt).sum())
        expect = T * att * (1.0 - M.fresnel(c, 1.0 / eta))
        cen = (dirs * (eys * wgt)).sum(1)
        cen /= np.linalg.norm(cen)
        rows.append((integ / expect - 1.0, math.acos(min(1.0, float(cen @ snell)))))
    return rows


def test_exit_btdf_smooth_limit(oracle_mod):
    rows = smooth_limit_errors(oracle_mod)
    assert len(rows) == 5
    for rel, ang in rows:
        assert abs(rel) < 5e-4, rows
        assert ang < 2e-3, rows


def node_weight_errors(orc, n_queries=40):
    """Largest deviations of (T_k, Snell's law, visibility of the
    refracting normal) over the nodes of n_queries clear hits."""
    d = W.default_params(K=6)
    ts = orc.TypeSet([d])
    eta, a = d["eta"], d["beta"]
    _, q = W.single_type(600, 22)
    _, fl = orc.eval([d], q)
    worst_T = worst_snell = 0.0
    n = 0
    for i in range(len(fl)):
        if not _clear(orc, fl[i]):
            continue
        qi = _query(q, i)
        wi = np.asarray(qi["wi"], np.float64)
        fx, _ = orc.frame_x(d, ts.tables[0], qi["h"], qi["u"], qi["v"], wi)
        nf = fx[6:9]
        nd, _ = orc.nodes(d, ts.tables[0], qi["h"], qi["u"], qi["v"], wi)
        F = M.local_frame(nf)
        for k in range(d["K"]):
            wt, T = nd[k, 5:8], nd[k, 4]
            m = -(wi + eta * wt)
            m /= np.linalg.norm(m)
            if m @ nf < 0:
                m = -m
            assert wi @ m > 0.0  # a normal the incident direction sees
            # Snell: the tangential components match, |wi x m| = eta |wt x m|
            worst_snell = max(worst_snell, abs(np.linalg.norm(np.cross(wi, m)) -
                                                eta * np.linalg.norm(np.cross(wt, m))))
            Tk = (1.0 - M.fresnel(wi @ m, eta)) * M.smith_G1((F @ wt).reshape(3, 1), (F @ m).reshape(3, 1), a)[0]
            worst_T = max(worst_T, abs(Tk - T))
        n += 1
        if n == n_queries:
            break
    return worst_T, worst_snell


def test_forward_node_weights(oracle_mod):
    worst_T, worst_snell = node_weight_errors(oracle_mod)
    assert worst_T < 1e-12 and worst_snell < 1e-12


def energy_identity_errors(orc, n_queries=3, grid=(900, 1800)):
    """Per query: (int E_xS, (1-B) k_S A_R), (int E_yS, (1-B) k_S/K sum T att A_T),
    (int E_c, identity_c) for c = r, g, b."""
    d = W.default_params()
    ts = orc.TypeSet([d])
    a, eta, B, kS, K = d["beta"], d["eta"], d["B"], d["k_spec"], d["K"]
    _, q = W.single_type(400, 13)
    _, fl = orc.eval([d], q)
    sph, dw = _sphere_grid(*grid)
    rows = []
    for i in range(len(fl)):
        if not _clear(orc, fl[i]):
            continue
        qi = _query(q, i)
        wi = np.asarray(qi["wi"], np.float64)
        fx, _ = orc.frame_x(d, ts.tables[0], qi["h"], qi["u"], qi["v"], wi)
        nf, gp, gf = fx[6:9], fx[9], fx[10]
        nd, _ = orc.nodes(d, ts.tables[0], qi["h"], qi["u"], qi["v"], wi)
        A_R = M.reflection_albedo(M.local_frame(nf) @ wi, a, eta)
        ys = 0.0
        for k in range(K):
            wt, ny = nd[k, 5:8], nd[k, 11:14]
            ys += nd[k, 4] * nd[k, 3] * M.exit_albedo(M.local_frame(-ny) @ (-wt), a, eta)
        integ = _eval_dirs(orc, [d], qi, sph).sum(0) * dw
        xs_id = (1 - B) * kS * A_R
        ys_id = (1 - B) * kS * ys / K
        tot = [(integ[c], xs_id + ys_id + B * gp * gf * d["albedo"][c]) for c in range(3)]
        rows.append(((integ[3], xs_id), (integ[4], ys_id), tot))
        if len(rows) == n_queries:
            break
    return rows


def test_energy_identity(oracle_mod):
    rows = energy_identity_errors(oracle_mod)
    assert len(rows) == 3
    for xs, ys, tot in rows:
        assert abs(xs[0] - xs[1]) < 5e-6 + 1e-4 * xs[1], rows
        assert abs(ys[0] - ys[1]) < 5e-6 + 1e-4 * ys[1], rows
        for e, i in tot:
            assert abs(e - i) < 1e-5, rows
