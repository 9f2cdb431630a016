"""Pins of the explicit-ply reference of the cross-section study (Sec. 3.4,
the elliptical vs circular cross-section comparison): explicit helical
plies around a circular-arc yarn, marched in 3D.

* on a straight yarn it agrees with the independent Python marcher of the
  brute-force tests (same ply, same chord length to the hit);
* a vanishing curvature gives the straight yarn;
* the returned tangent is the derivative of the stated ply centre curve
  (central differences written here);
* at perpendicular incidence on a straight yarn the ellipse plane is the
  cross-section, and both implicit constructions (n_iter = 0 and 5) find the
  explicit hit."""
import math

import numpy as np

from paper_2401_12724_amd import workloads as W

from test_oracle_bruteforce import _explicit_ply_hit


def _ray(rng, elev_deg):
    phi = rng.uniform(0, 2 * math.pi)
    e = math.radians(elev_deg) * (1 if rng.random() < 0.5 else -1)
    return np.array([math.cos(phi) * math.cos(e), math.sin(phi) * math.cos(e), math.sin(e)])


def test_straight_reference_matches_python_marcher(oracle_mod):
    d = W.default_params()
    rng = np.random.default_rng(1)
    checked = 0
    for _ in range(120):
        wi = _ray(rng, rng.uniform(0, 50))
        h, u, v = rng.uniform(-0.9, 0.9), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
        ok, ref = oracle_mod.explicit_ply(d, 0.0, h, u, v, wi, step=5e-4)
        assert ok
        s_py, k_py = _explicit_ply_hit(d, h, u, v, wi, step=2e-4)
        assert (k_py < 0) == (ref[0] < 0)
        if k_py < 0:
            continue
        s_c = math.hypot(*(ref[1:3] - _x2(h, wi)))  # chord length in the cross-section
        assert int(ref[0]) == k_py
        assert abs(s_c - s_py) < 2e-3
        checked += 1
    assert checked > 60


def _x2(h, wi):
    sxy = math.hypot(wi[0], wi[1])
    c = wi[:2] / sxy
    g = math.asin(h)
    return np.array([c[0] * math.cos(g) - c[1] * math.sin(g), c[1] * math.cos(g) + c[0] * math.sin(g)])


def test_small_curvature_is_the_straight_yarn(oracle_mod):
    d = W.default_params()
    rng = np.random.default_rng(2)
    for _ in range(60):
        wi = _ray(rng, rng.uniform(0, 60))
        h, u, v = rng.uniform(-0.9, 0.9), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
        ok0, a = oracle_mod.explicit_ply(d, 0.0, h, u, v, wi)
        ok1, b = oracle_mod.explicit_ply(d, 1e-7, h, u, v, wi)
        assert ok0 == ok1 and a[0] == b[0]
        if a[0] >= 0:
            assert np.allclose(a[1:], b[1:], atol=1e-4)


def test_reference_tangent_is_the_centre_curve_derivative(oracle_mod):
    """The ply centre at arc length s: c(s) + R_pc (cos th N(s) + sin th B)
    with the arc c(s) = ((1 - cos ks)/k, 0, sin(ks)/k), N(s) = (cos ks, 0,
    -sin ks), B = y, th = u + 2 pi j / N_p + w_p (v + s)."""
    d = W.default_params()
    rng = np.random.default_rng(3)
    wp = math.tan(d["ply_twist"]) / d["ply_center_radius"]
    checked = 0
    for kappa in (0.0, 0.125, 0.25):
        for _ in range(40):
            wi = _ray(rng, rng.uniform(0, 50))
            h, u, v = rng.uniform(-0.9, 0.9), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
            ok, ref = oracle_mod.explicit_ply(d, kappa, h, u, v, wi)
            if not ok or ref[0] < 0:
                continue
            j = int(ref[0])
            q = ref[1:4]
            s = q[2] if kappa == 0 else math.atan2(q[2], 1 / kappa - q[0]) / kappa

            def centre(s):
                if kappa == 0:
                    c, N = np.array([0, 0, s]), np.array([1.0, 0, 0])
                else:
                    c = np.array([(1 - math.cos(kappa * s)) / kappa, 0, math.sin(kappa * s) / kappa])
                    N = np.array([math.cos(kappa * s), 0, -math.sin(kappa * s)])
                th = u + 2 * math.pi * j / d["n_plies"] + wp * (v + s)
                return c + d["ply_center_radius"] * (math.cos(th) * N + math.sin(th) * np.array([0, 1.0, 0]))

            eps = 1e-5
            t = (centre(s + eps) - centre(s - eps)) / (2 * eps)
            t /= np.linalg.norm(t)
            assert np.allclose(ref[4:7], t, atol=1e-6)
            checked += 1
    assert checked > 60


def test_perpendicular_view_implicit_equals_explicit(oracle_mod):
    d = W.default_params()
    rng = np.random.default_rng(4)
    checked = 0
    for _ in range(150):
        wi = _ray(rng, 0.0)
        h, u, v = rng.uniform(-0.9, 0.9), rng.uniform(0, 2 * math.pi), rng.uniform(0, 10)
        ok, ref = oracle_mod.explicit_ply(d, 0.0, h, u, v, wi, step=5e-4)
        if not ok or ref[0] < 0:
            continue
        for it in (0, 5):
            out, fl = oracle_mod.ply_frame(dict(d, n_iter=it), h, u, v, wi)
            if fl & oracle_mod.MARGIN_MASK:
                continue
            assert not out[0] and int(out[1]) == int(ref[0])
            assert np.linalg.norm(np.array([out[2], out[3], out[4] - v]) - ref[1:4]) < 1e-4
            assert np.allclose(out[5:8], ref[4:7], atol=1e-6)
        checked += 1
    assert checked > 80
