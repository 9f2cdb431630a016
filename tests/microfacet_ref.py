"""Vectorised textbook microfacet primitives for the oracle's pins, and
quadrature over visible microfacet normals.

The primitives (dielectric Fresnel, isotropic GGX D, Smith's uncorrelated
G1) are the published definitions (Walter et al. 2007; Heitz 2014).  The
tests check them against the oracle's own primitives at random points, which
are pinned by closed forms elsewhere; what the pins here test is how the
oracle assembles them into lobes.

Integrals over microfacet normals use a midpoint grid in the polar and
azimuthal angles of m (solid-angle weight sin(theta) dtheta dphi), fine
enough to resolve both the GGX peak and the kink of max(0, w.m) for grazing
views.
"""
import math

import numpy as np


def fresnel(c, e):
    """Unpolarised dielectric Fresnel reflectance for the cosine c >= 0 of
    the incident direction, relative index e = eta_transmitted / eta_incident;
    total internal reflection gives 1."""
    c = np.asarray(c, dtype=np.float64)
    s2 = (1.0 - c * c) / (e * e)
    tir = s2 >= 1.0
    ct = np.sqrt(np.maximum(0.0, 1.0 - s2))
    with np.errstate(invalid="ignore", divide="ignore"):
        rs = (c - e * ct) / (c + e * ct)
        rp = (e * c - ct) / (e * c + ct)
    return np.where(tir, 1.0, 0.5 * (rs * rs + rp * rp))


def ggx_D(mz, mxy2, a):
    """Isotropic GGX density of microfacet normals with local z = mz and
    squared tangential length mxy2 (mz > 0)."""
    t = mxy2 / (a * a) + mz * mz
    return np.where(mz > 0.0, 1.0 / (math.pi * a * a * t * t), 0.0)


def smith_G1(w, m, a):
    """Smith's uncorrelated masking of direction w (local, normal = z) by a
    microfacet m: chi+((w.m)(w.n)) 2 / (1 + sqrt(1 + a^2 tan^2 theta_w))."""
    wm = (w * m).sum(0)
    wz = w[2]
    t2 = (w[0] ** 2 + w[1] ** 2) / (wz * wz)
    g = 2.0 / (1.0 + np.sqrt(1.0 + a * a * t2))
    return np.where(wm * wz > 0.0, g, 0.0)


def normal_grid(nth=3000, nphi=2000):
    """Microfacet normals m (3, N) on the upper hemisphere and their
    solid-angle weights."""
    th = 0.5 * math.pi * (np.arange(nth) + 0.5) / nth
    ph = 2.0 * math.pi * (np.arange(nphi) + 0.5) / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    st = np.sin(T)
    m = np.stack([st * np.cos(P), st * np.sin(P), np.cos(T)]).reshape(3, -1)
    return m, (st * (0.5 * math.pi / nth) * (2.0 * math.pi / nphi)).reshape(-1)


def visible_normal_mean(w, a, integrand, nth=3000, nphi=2000):
    """Mean of integrand(m) over the distribution of normals visible from w
    (local, w.z > 0): D_w(m) = G1(w, m) max(0, w.m) D(m) / w.z.  Returns
    (mean, total visible weight); the weight is 1 for Smith's G1."""
    m, dw = normal_grid(nth, nphi)
    wv = np.asarray(w, dtype=np.float64).reshape(3, 1)
    wm = (wv * m).sum(0)
    D = ggx_D(m[2], m[0] ** 2 + m[1] ** 2, a)
    vis = smith_G1(np.broadcast_to(wv, m.shape), m, a) * np.maximum(wm, 0.0) * D / wv[2, 0] * dw
    return float((vis * integrand(m)).sum()), float(vis.sum())


def local_frame(n):
    """An orthonormal (t, b, n) with the given unit normal."""
    n = np.asarray(n, dtype=np.float64)
    h = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t = h - n * (h @ n)
    t /= np.linalg.norm(t)
    return np.stack([t, np.cross(n, t), n])


def reflection_albedo(wi_l, a, eta):
    """A_R: the share of light from wi (local at x) reflected once by the
    rough dielectric, int D_wi(m) F(wi.m) G1(wo(m), m) dm with wo the mirror
    direction about m."""
    def g(m):
        c = (wi_l.reshape(3, 1) * m).sum(0)
        wo = 2.0 * c * m - wi_l.reshape(3, 1)
        return fresnel(np.maximum(c, 0.0), eta) * smith_G1(wo, m, a)
    return visible_normal_mean(wi_l, a, g)[0]


def exit_albedo(wip_l, a, eta):
    """A_T at an exit point: light inside the yarn travelling towards the
    surface, seen from inside along wip (local, z = the inward normal,
    wip.z > 0), refracted out (index eta to 1) through a visible normal m:
    int D_wip(m) (1 - F_in(wip.m)) G1(wo(m), m) dm."""
    def g(m):
        c = np.maximum((wip_l.reshape(3, 1) * m).sum(0), 0.0)
        s2 = eta * eta * (1.0 - c * c)
        ok = s2 < 1.0
        ct = np.sqrt(np.maximum(0.0, 1.0 - s2))
        wo = -eta * wip_l.reshape(3, 1) + (eta * c - ct) * m
        return np.where(ok, (1.0 - fresnel(c, 1.0 / eta)) * smith_G1(wo, m, a), 0.0)
    return visible_normal_mean(wip_l, a, g)[0]
