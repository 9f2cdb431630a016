"""GPU ray / yarn-tube intersection (yarn_scene_create, yarn_tube_intersect)
against the FP64 intersection oracle: a small weave with random rays (every
ray), the full 512-yarn weave with camera and random rays (sampled rays),
a non-planar yarn, scenes of 1 to 9 spans (wide BVH nodes with unused
slots), rays starting inside and just outside the tubes, and the edge cases (misses, t_max, origins inside a tube, end caps,
bad rays, empty batches)."""
import numpy as np
import pytest

import oracle
from paper_2401_12724_amd import bysdf, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _run(torch, scene, o, d, t_max, t_min=1e-4):
    od = torch.from_numpy(np.ascontiguousarray(o.T)).cuda()
    dd = torch.from_numpy(np.ascontiguousarray(d.T)).cuda()
    tm = torch.from_numpy(np.ascontiguousarray(t_max, np.float32)).cuda()
    h = bysdf.yarn_tube_intersect(scene, od, dd, tm, t_min)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in h.items()}


def _compare(g, r, phase, label, frame_tol=1e-6):
    """Misses and yarns equal; t, span parameter, h, v, frame to float
    rounding of the FP64 results (oracle margin flags left out)."""
    of = r[:, 12].astype(np.int64)
    ok = (of & oracle.HIT_MARGIN_MASK) == 0
    miss_o = (of & oracle.HIT_MISS) != 0
    miss_g = (g["flags"].astype(np.int64) & bysdf.HIT_MISS) != 0
    assert np.array_equal(miss_o[ok], miss_g[ok]), label
    both = ok & ~miss_o
    assert np.array_equal(g["yarn"][both], r[both, 1].astype(np.int32)), label
    t_ref = r[both, 0]
    assert np.all(np.abs(g["t"][both] - t_ref) <= 2e-7 * np.maximum(1.0, t_ref)), label
    # span parameter: spans meet at integer values of seg + s
    assert np.all(np.abs(g["seg"][both] + g["s"][both] - (r[both, 2] + r[both, 3])) < 1e-6), label
    assert np.all(np.abs(g["h"][both] - r[both, 4]) < 1e-6), label
    assert np.all(np.abs(g["v"][both] - r[both, 5]) <= 1e-6 + 2e-7 * np.abs(r[both, 5])), label
    assert np.all(np.abs(g["u"][both] - phase[r[both, 1].astype(int)]) == 0), label
    T = np.stack([g["tan_x"], g["tan_y"], g["tan_z"]], 1)[both]
    N = np.stack([g["nrm_x"], g["nrm_y"], g["nrm_z"]], 1)[both]
    assert np.abs(T - r[both, 6:9]).max() < 1e-6, label
    assert np.abs(N - r[both, 9:12]).max() < frame_tol, label
    cap_o = (of & oracle.HIT_CAP) != 0
    cap_g = (g["flags"].astype(np.int64) & bysdf.HIT_CAP) != 0
    assert np.array_equal(cap_o[both], cap_g[both]), label
    print(label, "rays", len(of), "hits", both.sum(), "margin", (~ok).sum())
    return both


def test_small_weave_every_ray(torch_cuda):
    torch = torch_cuda
    ctrl, off, ty, ph = W.weave(8, 8, 0.15, 0.05, 4)
    S = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    info = bysdf.yarn_scene_info(S)
    assert info["n_spans"] == 16 * (8 * 4) and info["depth"] <= 64
    half = 8 * 0.15 / 2
    o, d = W.random_rays(6000, 11, (-half, -half, 0.2), (half, half, 1.0), (-half, -half, -0.06),
                         (half, half, 0.06))
    # and rays from below and sideways, some starting between the yarns
    o2, d2 = W.random_rays(3000, 12, (-half, -half, -0.08), (half, half, 0.08))
    o, d = np.concatenate([o, o2]), np.concatenate([d, d2])
    tm = np.full(len(o), 100.0, np.float32)
    g = _run(torch, S, o, d, tm)
    r = oracle.intersect(oracle.Scene(ctrl, off), o, d, tm, 1e-4)
    both = _compare(g, r, ph, "small weave")
    assert both.sum() > 4000
    # bitwise reproducible
    g2 = _run(torch, S, o, d, tm)
    for k in g:
        assert np.array_equal(g[k], g2[k]), k


def test_full_weave_sampled(torch_cuda):
    """The 256 + 256 yarn weave (525,824 control points): 4,000 camera rays
    of the grazing 1920x1080 view and 2,000 random rays from above."""
    torch = torch_cuda
    ctrl, off, ty, ph = W.weave()
    S = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    info = bysdf.yarn_scene_info(S)
    assert info["n_spans"] == 512 * 1024 and info["depth"] <= 64
    rng = np.random.default_rng(3)
    o, d = W.pinhole_rays(W.weave_camera(), rng.integers(0, 1920, 4000), rng.integers(0, 1080, 4000))
    o2, d2 = W.random_rays(2000, 13, (-19, -19, 0.5), (19, 19, 3.0), (-19, -19, -0.06),
                           (19, 19, 0.06))
    o, d = np.concatenate([o, o2]), np.concatenate([d, d2])
    tm = np.full(len(o), 1e3, np.float32)
    g = _run(torch, S, o, d, tm)
    r = oracle.intersect(oracle.Scene(ctrl, off), o, d, tm, 1e-4)
    both = _compare(g, r, ph, "full weave")
    assert both.sum() > 3000


def test_scene_build_independent_of_threads(torch_cuda):
    """The full weave built on one host thread and on the default number
    gives the same scene and the same intersections, byte for byte."""
    torch = torch_cuda
    ctrl, off, ty, ph = W.weave()
    rng = np.random.default_rng(7)
    o, d = W.pinhole_rays(W.weave_camera(), rng.integers(0, 1920, 20000), rng.integers(0, 1080, 20000))
    tm = np.full(len(o), 1e3, np.float32)
    try:
        bysdf.yarn_scene_build_threads(1)
        S1 = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    finally:
        bysdf.yarn_scene_build_threads(0)
    S0 = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    assert bysdf.yarn_scene_info(S1) == bysdf.yarn_scene_info(S0)
    g1, g0 = _run(torch, S1, o, d, tm), _run(torch, S0, o, d, tm)
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k


def test_origins_inside_and_near_tubes(torch_cuda):
    """Rays in random directions from points at 0 to 1.2 R off a yarn's
    centreline on the small weave: inside the tube the point query excludes
    the yarn (and any other tube holding the point), just outside it does
    not.  The fractions stay clear of the exclusion limit R (1 - 1e-3), where
    rounding would decide."""
    torch = torch_cuda
    ctrl, off, ty, ph = W.weave(8, 8, 0.15, 0.05, 4)
    S = bysdf.yarn_scene_create(ctrl, off, ty, ph)
    sc = oracle.Scene(ctrl, off)
    rng = np.random.default_rng(21)
    fr = np.array([0.0, 0.3, 0.7, 0.95, 0.99, 1.01, 1.05, 1.2])
    o, d = [], []
    for i in range(4000):
        y = int(rng.integers(len(off) - 1))
        seg = int(rng.integers(off[y + 1] - off[y] - 3))
        f = sc.frame(y, seg, float(rng.random()))
        T, N, c = f[0:3], f[3:6], f[7:10]
        phi = 2.0 * np.pi * rng.random()
        rr = float(ctrl[off[y], 3]) * fr[i % len(fr)]
        o.append(c + rr * (np.cos(phi) * N + np.sin(phi) * np.cross(T, N)))
        v = rng.normal(size=3)
        d.append(v / np.linalg.norm(v))
    o, d = np.array(o, np.float32), np.array(d, np.float32)
    tm = np.full(len(o), 100.0, np.float32)
    g = _run(torch, S, o, d, tm)
    r = oracle.intersect(sc, o, d, tm, 1e-4)
    both = _compare(g, r, ph, "origins inside and near tubes")
    assert both.sum() > 1500


def test_non_planar_yarn(torch_cuda):
    """Control points on a helix: the frame is transported in 16 steps per
    span on the device and 64 in the oracle; both converge to the
    rotation-minimising frame (fourth-order steps); over 37 strongly
    twisting spans they part by about 1e-6, hence the 5e-6 bound."""
    torch = torch_cuda
    k = np.arange(40)
    ctrl = np.stack([np.cos(0.3 * k), np.sin(0.3 * k), 0.1 * k, np.full(40, 0.08)],
                    1).astype(np.float32)
    off = np.array([0, 40], np.int64)
    S = bysdf.yarn_scene_create(ctrl, off)
    o, d = W.random_rays(3000, 14, (-2, -2, -1), (2, 2, 5), (-1, -1, 0), (1, 1, 4))
    tm = np.full(len(o), 50.0, np.float32)
    g = _run(torch, S, o, d, tm)
    r = oracle.intersect(oracle.Scene(ctrl, off), o, d, tm, 1e-4)
    both = _compare(g, r, np.zeros(1, np.float32), "helix", frame_tol=5e-6)
    assert both.sum() > 100


@pytest.mark.parametrize("n_spans", [1, 2, 5, 9])
def test_tiny_scenes(torch_cuda, n_spans):
    """A single gently bent yarn of 1, 2, 5 or 9 spans: the root of the wide
    BVH has unused child slots (and a 1-span scene a root whose second
    binary child is empty), which must never be entered.  The bend is kept
    small: the frame's transport within a span (16 steps on the device, 64
    in the oracle) is checked on the helix above."""
    torch = torch_cuda
    n_cp = n_spans + 3
    x = np.linspace(-1.0, 1.0, n_cp)
    ctrl = np.stack([x, 0.02 * np.sin(3.0 * x), 0.01 * np.cos(2.0 * x), np.full(n_cp, 0.15)],
                    1).astype(np.float32)
    off = np.array([0, n_cp], np.int64)
    S = bysdf.yarn_scene_create(ctrl, off)
    assert bysdf.yarn_scene_info(S)["n_spans"] == n_spans
    o, d = W.random_rays(2000, 20 + n_spans, (-2, -2, -2), (2, 2, 2), (-1, -0.3, -0.3), (1, 0.3, 0.3))
    tm = np.full(len(o), 20.0, np.float32)
    g = _run(torch, S, o, d, tm)
    r = oracle.intersect(oracle.Scene(ctrl, off), o, d, tm, 1e-4)
    both = _compare(g, r, np.zeros(1, np.float32), "tiny %d" % n_spans)
    assert both.sum() > 200


def test_edge_cases(torch_cuda):
    torch = torch_cuda
    R = float(np.float32(0.2))
    x = -2.0 + 0.5 * np.arange(10)
    ctrl = np.stack([x, np.zeros(10), np.zeros(10), np.full(10, R)], 1).astype(np.float32)
    off = np.array([0, 10], np.int64)
    S = bysdf.yarn_scene_create(ctrl, off, yarn_phase=np.array([1.25], np.float32))
    o = np.array([[0.0, 0.0, 3.0],      # straight down onto the capsule
                  [0.0, 0.0, 3.0],      # same, t_max short of the surface
                  [0.0, 0.0, 0.0],      # origin on the axis: yarn skipped
                  [-5.0, 0.0, 0.0],     # along the axis into the end cap
                  [0.0, 5.0, 3.0],      # misses
                  [0.0, 0.0, 3.0]],     # zero direction
                 np.float32)
    d = np.array([[0, 0, -1], [0, 0, -1], [0, 0, 1], [1, 0, 0], [0, 0, -1], [0, 0, 0]], np.float32)
    tm = np.array([10, 2.5, 10, 10, 10, 10], np.float32)
    g = _run(torch, S, o, d, tm)
    f = g["flags"].astype(np.int64)
    assert f[0] == 0 and abs(g["t"][0] - (3.0 - R)) < 1e-6 and abs(g["h"][0]) < 1e-7
    assert abs(g["u"][0] - 1.25) == 0 and abs(g["v"][0] - 1.5) < 1e-6
    assert f[1] & bysdf.HIT_MISS and np.isinf(g["t"][1]) and g["yarn"][1] == -1
    assert f[2] & bysdf.HIT_MISS and f[2] & bysdf.HIT_EXCLUDED
    assert f[3] & bysdf.HIT_CAP and abs(g["t"][3] - (5.0 - 1.5 - R)) < 1e-6
    assert f[4] & bysdf.HIT_MISS
    assert f[5] & bysdf.HIT_BAD_INPUT and f[5] & bysdf.HIT_MISS
    # empty batch is a no-op
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda")
    bysdf.yarn_tube_intersect(S, e, e, torch.empty(0, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
