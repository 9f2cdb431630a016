"""Brute-force pins of the oracle's geometry on tiny inputs.

The fiber table, the ply horizon, the implicit-ply hit and the forward chords
are checked against explicit geometry (discs and helices) probed by dense
marching and direct distance tests -- a different computation from the
oracle's closed-form ray/disc and interval arithmetic.
"""
import math

import numpy as np
import pytest

from paper_2401_12724_amd import workloads as W


def _vogel(M, rho):
    """Fiber centres of the ply cross-section (the arrangement the oracle
    documents: Vogel spiral inside radius 1 - rho)."""
    g = math.pi * (3 - math.sqrt(5))
    j = np.arange(M)
    r = (1 - rho) * np.sqrt((j + 0.5) / M)
    return np.stack([r * np.cos(j * g), r * np.sin(j * g)], 1)


def _first_inside(o, d, centres, rad, smax, step):
    """March o + s d; return (s, index) of the first point inside any disc,
    refined by bisection."""
    s = 0.0
    prev = 0.0
    while s <= smax:
        p = o + s * d
        dist = np.linalg.norm(centres - p, axis=1) - rad
        j = int(np.argmin(dist))
        if dist[j] <= 0:
            lo, hi = prev, s
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                if np.min(np.linalg.norm(centres - (o + mid * d), axis=1) - rad) <= 0:
                    hi = mid
                else:
                    lo = mid
            pp = o + hi * d
            j = int(np.argmin(np.linalg.norm(centres - pp, axis=1) - rad))
            return hi, j
        prev = s
        s += step
    return None, -1


def _blocked_fraction(q, normal, others, rad, n_dir=20001):
    """Cosine-weighted share of the hemisphere around `normal` at q whose
    rays pass within `rad` of some centre ahead of q."""
    th = (np.arange(n_dir) + 0.5) / n_dir * math.pi - 0.5 * math.pi
    base = math.atan2(normal[1], normal[0])
    dirs = np.stack([np.cos(base + th), np.sin(base + th)], 1)
    w = others - q  # (L, 2)
    proj = dirs @ w.T  # (n_dir, L)
    perp2 = (w * w).sum(1)[None, :] - proj ** 2
    blocked = ((proj > 0) & (perp2 <= rad * rad)).any(1)
    cosw = np.cos(th)
    return (cosw * blocked).sum() / cosw.sum()


@pytest.mark.parametrize("M,rho", [(64, 0.06), (32, 0.06), (12, 0.15)])
def test_fiber_table_bruteforce(oracle_mod, M, rho):
    d = W.default_params(fibers_per_ply=M, fiber_radius=rho, tex_size=256)
    tab = oracle_mod.table(d)
    C = _vogel(M, rho)
    rng = np.random.default_rng(M)
    for i in rng.choice(256, 24, replace=False):
        z = 2 * math.pi * (i + 0.5) / 256
        e = np.array([math.cos(z), math.sin(z)])
        s, j = _first_inside(1.0000001 * e, -e, C, rho, 2.0, rho / 50)
        if j < 0:
            assert tab[i, 1] == 0.0 and tab[i, 2] == 1.0 and tab[i, 0] == 0.0  # no fiber on the ray
            continue
        q = 1.0000001 * e - s * e
        n = (q - C[j]) / rho
        dn = math.atan2(e[0] * n[1] - e[1] * n[0], e @ n)
        assert abs(tab[i, 0] - dn) < 1e-5
        # texels are stored in single precision
        assert abs(tab[i, 1] - np.linalg.norm(C[j]) / (1 - rho)) < 1.2e-7
        others = np.delete(C, j, 0)
        gf = 1.0 - _blocked_fraction(q, n, others, rho)
        assert abs(tab[i, 2] - gf) < 2e-3


def test_ply_shadow_bruteforce(oracle_mod):
    for npl in (2, 3, 5):
        rp = W.packed_ply_radius(npl)
        d = W.default_params(n_plies=npl, ply_radius=rp, ply_center_radius=1 - rp)
        Rpc = 1 - rp
        C = np.array([[Rpc * math.cos(2 * math.pi * j / npl), Rpc * math.sin(2 * math.pi * j / npl)]
                      for j in range(npl)])
        rng = np.random.default_rng(npl)
        for _ in range(20):
            a = rng.uniform(-math.pi, math.pi)
            phi = rng.uniform(-1.4, 1.4)
            P = C[0] + rp * np.array([math.cos(a), math.sin(a)])
            nrm = np.array([math.cos(a), math.sin(a)])
            # directions in the window, blocked below the tangent line or by
            # another ply disc ahead
            th = phi + (np.arange(4001) + 0.5) / 4001 * 0.2 - 0.1
            base = a
            dirs = np.stack([np.cos(base + th), np.sin(base + th)], 1)
            below = (dirs @ nrm) < 0
            w = C[1:] - P
            proj = dirs @ w.T
            perp2 = (w * w).sum(1)[None, :] - proj ** 2
            blk = ((proj > 0) & (perp2 <= rp * rp)).any(1) | below
            bf = 1.0 - blk.mean()
            assert abs(oracle_mod.ply_shadow_raw(d, a, phi) - bf) < 2e-3


def _explicit_ply_hit(d, h, u, v, wi, step=2e-4):
    """First 3D point along the incident ray inside an explicit helical ply
    tube (horizontal cross-sections are discs of radius r_p around the helix
    centre at that height)."""
    rp, Rpc, N = d["ply_radius"], d["ply_center_radius"], d["n_plies"]
    wp = math.tan(d["ply_twist"]) / Rpc
    sxy = math.hypot(wi[0], wi[1])
    c = np.array([wi[0], wi[1]]) / sxy
    g = math.asin(h)
    x2 = np.array([c[0] * math.cos(g) - c[1] * math.sin(g), c[1] * math.cos(g) + c[0] * math.sin(g)])
    dxy = -np.array([wi[0], wi[1]])
    dz = -wi[2]
    best = None
    t = 0.0
    tmax = 2.0 / sxy
    prev_in = None
    while t <= tmax:
        p = x2 + t * dxy
        z = v + t * dz
        th = u + 2 * math.pi * np.arange(N) / N + wp * z
        cen = Rpc * np.stack([np.cos(th), np.sin(th)], 1)
        dist = np.linalg.norm(cen - p, axis=1)
        if (dist <= rp).any():
            return t * sxy, int(np.argmin(dist - rp))  # 2D distance from x2
        t += step
    return None, -1


def test_implicit_plies_match_explicit_for_steep_rays(oracle_mod):
    """For rays nearly perpendicular to the yarn axis the ellipse plane is
    the perpendicular cross-section, and the implicit ply hit must coincide
    with the explicit helix; the deviation grows with |kappa|."""
    d = W.default_params()
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(400):
        th = rng.uniform(0, 2 * math.pi)
        kz = rng.uniform(-0.02, 0.02)
        wi = np.array([math.cos(th), math.sin(th), kz])
        wi /= np.linalg.norm(wi)
        h, u, v = rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
        out, fl = oracle_mod.ply_hit(d, h, u, v, wi)
        s_ex, k_ex = _explicit_ply_hit(d, h, u, v, wi)
        if fl & oracle_mod.MARGIN_MASK:
            continue
        if out[0]:
            # a miss may only disagree when the explicit hit is a sliver
            assert k_ex < 0 or s_ex > 1.9 * math.sqrt(1 - h * h) - 0.05
            continue
        if k_ex < 0:
            continue
        checked += 1
        kappa = abs(wi[2]) / math.hypot(wi[0], wi[1])
        if int(out[1]) == k_ex:
            assert abs(out[2] - s_ex) < 2e-3 + 5 * kappa
    assert checked > 200


def test_straight_plies_reduce_to_circles(oracle_mod):
    """alpha_p = 0: ply centres do not move, the fixed point is trivial and
    the hit is the first 2D disc crossing."""
    d = W.default_params(ply_twist=0.0)
    rng = np.random.default_rng(6)
    Rpc, rp = d["ply_center_radius"], d["ply_radius"]
    for _ in range(200):
        wi = rng.normal(size=3)
        wi /= np.linalg.norm(wi)
        h, u, v = rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
        out, fl = oracle_mod.ply_hit(d, h, u, v, wi)
        if fl & (oracle_mod.MARGIN_MASK | oracle_mod.AXIAL):
            continue
        sxy = math.hypot(wi[0], wi[1])
        c = wi[:2] / sxy
        g = math.asin(h)
        x2 = np.array([c[0] * math.cos(g) - c[1] * math.sin(g), c[1] * math.cos(g) + c[0] * math.sin(g)])
        cen = np.array([[Rpc * math.cos(u + 2 * math.pi * k / 3), Rpc * math.sin(u + 2 * math.pi * k / 3)]
                        for k in range(3)])
        s, j = _first_inside(x2, -c, cen, rp, 2 * math.sqrt(1 - h * h), 1e-3)
        if out[0]:
            assert j < 0
        else:
            assert j == int(out[1]) and abs(s - out[2]) < 1e-9 + 1e-6
            assert abs(out[7] - (v + (-wi[2] / sxy) * out[2])) < 1e-12


def test_single_ply_is_the_yarn(oracle_mod):
    """N_p = 1 with r_p = 1, R_pc = 0: the ply is the yarn; the hit is the
    yarn hit and the ply normal is the yarn normal."""
    d = W.default_params(n_plies=1, ply_radius=1.0, ply_center_radius=0.0)
    rng = np.random.default_rng(8)
    for _ in range(100):
        wi = rng.normal(size=3)
        wi /= np.linalg.norm(wi)
        h = rng.uniform(-0.99, 0.99)
        out, fl = oracle_mod.ply_hit(d, h, 1.0, 2.0, wi)
        assert not out[0]
        assert abs(out[2]) < 1e-12
        sxy = math.hypot(wi[0], wi[1])
        g = math.asin(h)
        psi = math.atan2(wi[1], wi[0]) + g
        assert abs(out[5] - math.cos(psi)) < 1e-12 and abs(out[6] - math.sin(psi)) < 1e-12


def test_forward_chords_bruteforce(oracle_mod):
    """Node chords: the number of plies the refracted segment enters and the
    exit point, against dense sampling of the segment."""
    d = W.default_params()
    tab = oracle_mod.table(d)
    rng = np.random.default_rng(9)
    Rpc, rp = d["ply_center_radius"], d["ply_radius"]
    n_checked = 0
    for _ in range(300):
        wi = rng.normal(size=3)
        wi /= np.linalg.norm(wi)
        h, u, v = rng.uniform(-1, 1), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
        ph, fl = oracle_mod.ply_hit(d, h, u, v, wi)
        if ph[0] or fl & oracle_mod.MARGIN_MASK:
            continue
        nd, fl2 = oracle_mod.nodes(d, tab, h, u, v, wi)
        if fl2 & oracle_mod.MARGIN_MASK:
            continue
        th = ph[10:13]
        cen = Rpc * np.stack([np.cos(th), np.sin(th)], 1)
        for k in range(d["K"]):
            if nd[k, 0] != 0:
                continue
            p2 = nd[k, 14:16]
            e = nd[k, 5:7] / np.linalg.norm(nd[k, 5:7])
            # yarn boundary exit
            ts = np.linspace(1e-9, 2.0, 200001)
            pts = p2[None, :] + ts[:, None] * e[None, :]
            inside_yarn = (pts ** 2).sum(1) <= 1.0
            pts = pts[inside_yarn]
            ts = ts[inside_yarn]
            dist = np.linalg.norm(pts[:, None, :] - cen[None, :, :], axis=2) <= rp
            entered = dist.any(0)
            assert entered.sum() == int(nd[k, 1])
            last = np.nonzero(dist.any(1))[0][-1]
            s_exit = ts[last]
            ell2 = nd[k, 2] * np.linalg.norm(nd[k, 5:7])
            assert abs(s_exit - ell2) < 2e-5
            assert abs(nd[k, 3] - math.exp(-d["sigma_t"] * nd[k, 2] * nd[k, 1])) < 1e-12
            n_checked += 1
    assert n_checked > 100
