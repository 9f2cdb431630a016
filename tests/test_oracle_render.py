"""Pins of the CPU path tracer (render_oracle.c) that other tests compare the
GPU renderer with:

* a view that misses the scene shows the environment radiance exactly;
* a view into the light shows its radiance (first hit, no weighting);
* white furnace: with a lossless BYSDF (B = 1, unit albedo, no ply/fiber
  occlusion: the model then integrates to one, Sec. 4.3), no light and a
  unit environment, every pixel averages to one (within sampling error,
  less the rare paths still bouncing after the last allowed bounce);
* the image is a deterministic function of the seed.
"""
import numpy as np

import oracle
from paper_2401_12724_amd import workloads as W


def _settings(cam, crop, **kw):
    rs = dict(eye=cam["eye"], look_at=cam["look_at"], up=cam["up"], vfov=cam["vfov"],
              width=cam["width"], height=cam["height"], crop_x=crop[0], crop_y=crop[1],
              crop_w=crop[2], crop_h=crop[3], light_corner=(-5.0, -5.0, 30.0),
              light_u=(0.0, 10.0, 0.0), light_v=(10.0, 0.0, 0.0), light_radiance=(5.0, 5.0, 5.0),
              env_radiance=(0.2, 0.2, 0.2), spp=4, max_depth=8, lod_px=1.0, n_h=4, seed=7,
              ray_eps=1e-4)
    rs.update(kw)
    return rs


def _scene(n=8):
    ctrl, off, ty, ph = W.weave(n, n, 0.15, 0.05, 4)
    return oracle.Scene(ctrl, off), ty, ph


def test_sky_and_light():
    S, ty, ph = _scene()
    P = [W.default_params()]
    # looking up past the light: environment only
    cam = W.camera((20.0, 20.0, 1.0), (40.0, 40.0, 3.0), width=64, height=64)
    fb, _ = oracle.render(S, P, ty, ph, _settings(cam, (0, 0, 16, 16)))
    assert np.all(fb == np.float32(0.2))
    # looking straight at the light from below: its radiance
    cam = W.camera((0.0, 0.0, 25.0), (0.0, 0.0, 40.0), up=(0.0, 1.0, 0.0), vfov_deg=10.0,
                   width=32, height=32)
    fb, _ = oracle.render(S, P, ty, ph, _settings(cam, (0, 0, 8, 8)))
    assert np.all(fb == 5.0)


def test_white_furnace_image():
    S, ty, ph = _scene()
    P = [W.default_params(B=1.0, albedo=(1.0, 1.0, 1.0), ply_density=0.0, fiber_density=0.0)]
    cam = W.camera((0.0, -1.5, 0.8), (0.0, 0.0, 0.0), width=48, height=48)
    # the light is moved below the fabric, facing down, so that no path can
    # reach its emitting side (an opaque rectangle would absorb)
    rs = _settings(cam, (8, 8, 32, 32), light_radiance=(0.0, 0.0, 0.0), env_radiance=(1.0, 1.0, 1.0),
                   light_corner=(-5.0, -5.0, -30.0), spp=16, max_depth=32)
    fb, sq = oracle.render(S, P, ty, ph, rs)
    var = np.maximum(sq - fb * fb, 0.0)
    m = fb.mean()
    sigma = np.sqrt(var.mean() / (fb.size * rs["spp"] / 3))
    print("furnace mean", m, "sigma", sigma)
    assert abs(m - 1.0) < 4 * sigma + 2e-3
    assert fb.max() < 1.0 + 20 * np.sqrt(var.max() / rs["spp"]) + 1e-6


def test_deterministic():
    S, ty, ph = _scene()
    P = [W.default_params()]
    cam = W.camera((0.0, -3.0, 1.2), (0.0, 0.0, 0.0), width=64, height=36)
    rs = _settings(cam, (20, 10, 16, 16))
    a, _ = oracle.render(S, P, ty, ph, rs)
    b, _ = oracle.render(S, P, ty, ph, rs)
    assert np.array_equal(a, b)
    c, _ = oracle.render(S, P, ty, ph, dict(rs, seed=8))
    assert not np.array_equal(a, c)


def test_nee_and_bysdf_sampling_agree():
    """Direct light estimated with next-event estimation + MIS and with
    BYSDF sampling alone: two unbiased estimators of the same image (pins
    the light pdf and the power-heuristic weights).  A large light and no
    environment keep the sampling-only estimate from being too noisy."""
    S, ty, ph = _scene(6)
    P = [W.default_params()]
    cam = W.camera((0.0, -1.2, 0.9), (0.0, 0.0, 0.0), width=40, height=40)
    base = dict(env_radiance=(0.0, 0.0, 0.0), light_corner=(-3.0, -3.0, 2.0),
                light_u=(0.0, 6.0, 0.0), light_v=(6.0, 0.0, 0.0), light_radiance=(1.0, 1.0, 1.0),
                max_depth=3)
    a, a2 = oracle.render(S, P, ty, ph, _settings(cam, (4, 4, 32, 32), spp=32, seed=1, **base))
    b, b2 = oracle.render(S, P, ty, ph, _settings(cam, (4, 4, 32, 32), spp=256, seed=2, nee=0,
                                                  **base))
    va = np.maximum(a2 - a * a, 0).sum() / 32 / a.size ** 2
    vb = np.maximum(b2 - b * b, 0).sum() / 256 / b.size ** 2
    d = a.mean() - b.mean()
    print("nee", a.mean(), "bysdf only", b.mean(), "z", d / np.sqrt(va + vb))
    assert abs(d) < 4 * np.sqrt(va + vb)
