"""Seeded synthetic workloads for the BYSDF hot path.

This module only draws inputs: parameter records and query arrays.  It holds
none of the method's arithmetic, so both the HIP path and the test oracle can
consume what it produces.  Every array is generated once on the host from
``numpy.random.Generator(Philox(seed))`` and rounded to FP32.

The paper's datasets (yarn-level cloth, knit models, measured fibers) are not
available; these draws stand in for them with the shapes of the workloads:

* ``single_type``    -- 65,536 queries of one 3-ply yarn type (N_p=3, M=64,
                        ply twist 28 deg, fiber twist 15 deg, r_p=0.45,
                        r_f=0.06 r_p, eta=1.55, albedo (0.8,0.6,0.4), beta=0.15)
* ``per_block``      -- 2^24 queries in blocks of 256, beta and albedo drawn
                        per block, xi drawn per query for the sampler
* ``heterogeneous``  -- 4,096 yarn types, lognormal query counts (median 4,096,
                        clipped to 256..65,536), sorted by type
* ``fitting``        -- 64 types x 65,536 queries with hidden parameters
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0


def default_params(**over) -> dict:
    """Parameter record of the single-type workload (defaults of the build)."""
    p = dict(
        n_plies=3, fibers_per_ply=64, K=4, n_iter=5, tex_size=512,
        ply_radius=0.45, ply_center_radius=0.55, fiber_radius=0.06,
        ply_twist=28.0 * DEG, fiber_twist=15.0 * DEG, eta=1.55,
        albedo=(0.8, 0.6, 0.4), beta=0.15, aniso=1.0, k_spec=1.0,
        B=0.5, r=0.5, sigma_t=0.5, ply_density=1.0, fiber_density=1.0,
        shadow_halfwidth=0.1,
        # fiber migration (off with one table)
        mig_tables=1, mig_period=4.0, mig_blend=0.25, mig_spread=0.3, mig_seed=0,
    )
    p.update(over)
    if "ply_radius" in over and "ply_center_radius" not in over:
        p["ply_center_radius"] = 1.0 - p["ply_radius"]
    return as_f32(p)


INT_FIELDS = ("n_plies", "fibers_per_ply", "K", "n_iter", "tex_size", "mig_tables", "mig_seed")


def as_f32(p: dict) -> dict:
    """Round every real parameter to a single-precision value: parameter
    records are FP32 inputs of the library, and the oracle must see the same
    numbers."""
    q = dict(p)
    for k, v in p.items():
        if k in INT_FIELDS:
            q[k] = int(v)
        elif k == "albedo":
            q[k] = tuple(float(np.float32(a)) for a in v)
        else:
            q[k] = float(np.float32(v))
    return q


def packed_ply_radius(n_plies: int) -> float:
    """Ply radius (in yarn radii) of N_p equal discs packed tightly inside the
    yarn circle, each touching the boundary and its two neighbours."""
    if n_plies == 1:
        return 1.0
    s = math.sin(math.pi / n_plies)
    return s / (1.0 + s)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=seed))


def _sphere(rng, n):
    z = 1.0 - 2.0 * rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z]).astype(np.float32)


def sphere(n: int, rng) -> np.ndarray:
    """n directions uniform on S^2 from a numpy Generator, (3, n) float32."""
    return _sphere(rng, n)


def footprints(q: dict, seed: int, w_min: float = 2.0 ** -6, w_max: float = 2.0) -> dict:
    """Pixel footprints for the multi-scale model around each query's h: a
    width log-uniform in [w_min, w_max] (2 = a pixel covering the whole
    yarn), split at a uniform share to either side of h and cut at +-1;
    the strata offset zeta and the stratum draw xi_s uniform in [0, 1)."""
    rng = _rng(seed + 3000)
    n = len(q["h"])
    w = np.exp(rng.uniform(math.log(w_min), math.log(w_max), n))
    a = rng.random(n)
    h = q["h"].astype(np.float64)
    q["h1"] = np.maximum(h - a * w, -1.0).astype(np.float32)
    q["h2"] = np.minimum(h + (1.0 - a) * w, 1.0).astype(np.float32)
    # FP32 rounding keeps h1 <= h <= h2: both ends round towards h
    q["h1"] = np.minimum(q["h1"], q["h"])
    q["h2"] = np.maximum(q["h2"], q["h"])
    top = np.float32(1.0 - 2.0 ** -24)
    q["zeta"] = np.minimum(rng.random(n).astype(np.float32), top)
    q["xi_s"] = np.minimum(rng.random(n).astype(np.float32), top)
    return q


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) on arrays: ctr (4, n) and key (2,
    n) of uint32; ten rounds of the two 32 x 32 -> 64 multiplications, the
    Weyl key schedule between rounds.  Returns (4, n) uint32."""
    c = [np.asarray(x, np.uint64) & np.uint64(0xFFFFFFFF) for x in ctr]
    k0 = np.asarray(key[0], np.uint64) & np.uint64(0xFFFFFFFF)
    k1 = np.asarray(key[1], np.uint64) & np.uint64(0xFFFFFFFF)
    m32 = np.uint64(0xFFFFFFFF)
    for r in range(10):
        p0 = np.uint64(0xD2511F53) * c[0]
        p1 = np.uint64(0xCD9E8D57) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & m32, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & m32]
        if r < 9:
            k0 = (k0 + np.uint64(0x9E3779B9)) & m32
            k1 = (k1 + np.uint64(0xBB67AE85)) & m32
    return np.stack(c).astype(np.uint32)


def sampler_xi(n: int, seed: int) -> np.ndarray:
    """The three uniforms the library draws for sampler queries 0..n-1 when
    no xi arrays are given: Philox4x32-10 with counter (i mod 2^32, i >> 32,
    0, 0x53414d50), key (seed mod 2^32, seed >> 32), words 0..2 as
    (word >> 8) * 2^-24.  (3, n) float32."""
    i = np.arange(n, dtype=np.uint64)
    ctr = [i & np.uint64(0xFFFFFFFF), i >> np.uint64(32), np.zeros(n, np.uint64),
           np.full(n, 0x53414D50, np.uint64)]
    key = [np.full(n, seed & 0xFFFFFFFF, np.uint64), np.full(n, (seed >> 32) & 0xFFFFFFFF, np.uint64)]
    w = philox4x32_10(ctr, key)[:3]
    return ((w >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def queries(n: int, seed: int, n_types: int = 1, type_ids=None, with_xi: bool = False,
            v_max: float = 10.0) -> dict:
    """n queries: h~U[-1,1], u~U[0,2pi), v~U[0,v_max), wi, wo uniform on S^2."""
    rng = _rng(seed)
    if type_ids is None:
        type_ids = rng.integers(0, n_types, n) if n_types > 1 else np.zeros(n)
    q = dict(
        type=np.asarray(type_ids, dtype=np.int32),
        h=(2.0 * rng.random(n) - 1.0).astype(np.float32),
        u=(2.0 * math.pi * rng.random(n)).astype(np.float32),
        v=(v_max * rng.random(n)).astype(np.float32),
    )
    q["wi"] = np.ascontiguousarray(_sphere(rng, n))
    q["wo"] = np.ascontiguousarray(_sphere(rng, n))
    if with_xi:
        q["xi"] = np.ascontiguousarray(rng.random((3, n)).astype(np.float32))
        # keep xi strictly inside [0, 1) after rounding to FP32
        q["xi"] = np.minimum(q["xi"], np.float32(1.0 - 2.0 ** -24))
    return q


def single_type(n: int = 65536, seed: int = 0, with_xi: bool = False):
    """One 3-ply yarn type; returns (param list, queries)."""
    return [default_params()], queries(n, seed, with_xi=with_xi)


def per_block(n_blocks: int = 65536, block: int = 256, seed: int = 1):
    """Blocks of `block` queries sharing one parameter record whose beta ~
    U[0.05, 0.3] and albedo ~ U[0.3, 0.95]^3; xi per query for the sampler."""
    rng = _rng(seed + 1000)
    betas = rng.uniform(0.05, 0.3, n_blocks)
    albs = rng.uniform(0.3, 0.95, (n_blocks, 3))
    params = [default_params(beta=float(betas[b]), albedo=tuple(float(a) for a in albs[b]))
              for b in range(n_blocks)]
    tid = np.repeat(np.arange(n_blocks, dtype=np.int32), block)
    q = queries(n_blocks * block, seed, type_ids=tid, with_xi=True)
    return params, q


def heterogeneous_params(n_types: int = 4096, seed: int = 3):
    """Per-type records: plies 2..5 (tightly packed), fibers 32..128, twist
    angles U[10, 40] deg, beta U[0.05, 0.3], albedo U[0.2, 0.95]^3."""
    rng = _rng(seed + 2000)
    out = []
    for _ in range(n_types):
        npl = int(rng.integers(2, 6))
        rp = packed_ply_radius(npl)
        out.append(default_params(
            n_plies=npl, fibers_per_ply=int(rng.integers(32, 129)),
            ply_radius=rp, ply_center_radius=1.0 - rp,
            ply_twist=float(rng.uniform(10.0, 40.0)) * DEG,
            fiber_twist=float(rng.uniform(10.0, 40.0)) * DEG,
            beta=float(rng.uniform(0.05, 0.3)),
            albedo=tuple(float(a) for a in rng.uniform(0.2, 0.95, 3))))
    return out


def lognormal_counts(n_types: int = 4096, median: int = 4096, sigma: float = 2.49,
                     lo: int = 256, hi: int = 65536, seed: int = 3) -> np.ndarray:
    rng = _rng(seed + 3000)
    c = np.exp(np.log(median) + sigma * rng.standard_normal(n_types))
    return np.clip(np.rint(c), lo, hi).astype(np.int64)


def heterogeneous(n_types: int = 4096, seed: int = 3, counts=None):
    """Types with lognormal counts; queries sorted by type (CSR offsets)."""
    params = heterogeneous_params(n_types, seed)
    if counts is None:
        counts = lognormal_counts(n_types, seed=seed)
    offsets = np.zeros(n_types + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    tid = np.repeat(np.arange(n_types, dtype=np.int32), counts)
    q = queries(int(offsets[-1]), seed, type_ids=tid)
    return params, q, offsets


def fitting(n_types: int = 64, per_type: int = 65536, seed: int = 4):
    """Hidden parameters theta* per type (heterogeneous ranges, densities
    U[0.5, 1]) and the starting point theta0 = range midpoints."""
    rng = _rng(seed + 4000)
    hidden, start = [], []
    for _ in range(n_types):
        base = dict(n_plies=3, fibers_per_ply=64)
        hidden.append(default_params(
            **base,
            ply_twist=float(rng.uniform(10.0, 40.0)) * DEG,
            fiber_twist=float(rng.uniform(10.0, 40.0)) * DEG,
            beta=float(rng.uniform(0.05, 0.3)),
            albedo=tuple(float(a) for a in rng.uniform(0.2, 0.95, 3)),
            ply_density=float(rng.uniform(0.5, 1.0)),
            fiber_density=float(rng.uniform(0.5, 1.0))))
        start.append(default_params(
            **base, ply_twist=25.0 * DEG, fiber_twist=25.0 * DEG, beta=0.175,
            albedo=(0.575, 0.575, 0.575), ply_density=0.75, fiber_density=0.75))
    tid = np.repeat(np.arange(n_types, dtype=np.int32), per_type)
    q = queries(n_types * per_type, seed, type_ids=tid)
    return hidden, start, q


THETA_NAMES = ("albedo_r", "albedo_g", "albedo_b", "beta", "ply_twist", "fiber_twist",
               "ply_density", "fiber_density")


def theta_of(p: dict) -> np.ndarray:
    return np.array([p["albedo"][0], p["albedo"][1], p["albedo"][2], p["beta"], p["ply_twist"],
                     p["fiber_twist"], p["ply_density"], p["fiber_density"]], dtype=np.float64)


def with_theta(p: dict, th) -> dict:
    q = dict(p)
    q["albedo"] = (float(th[0]), float(th[1]), float(th[2]))
    q["beta"], q["ply_twist"], q["fiber_twist"] = float(th[3]), float(th[4]), float(th[5])
    q["ply_density"], q["fiber_density"] = float(th[6]), float(th[7])
    return as_f32(q)


# ---------------------------------------------------------------- yarn scenes

def weave(n_warp: int = 256, n_weft: int = 256, pitch: float = 0.15, radius: float = 0.05,
          cps_per_crossing: int = 4, seed: int = 2):
    """Plain weave of yarn centrelines as uniform cubic B-spline control
    points.  Warp yarn i runs along x at y_i, weft yarn j along y at x_j
    (pitch apart, the fabric centred on the origin); their heights follow
    +-radius/2 cos(pi (index coordinate) + pi (yarn index)), so the two
    yarns of a crossing sit one radius apart with alternating over/under.
    Control points are spaced pitch / cps_per_crossing along each yarn and
    extend half a pitch past the outermost crossings (plus one point for
    the spline's end spans).

    Returns (ctrl (n_cp, 4) float32 rows x, y, z, r; yarn_off (n_yarns+1)
    int64; yarn_type (n_yarns) int32; yarn_phase (n_yarns) float32, the
    ply-helix phase of each yarn drawn uniformly in [0, 2 pi))."""
    cw = (n_weft - 1) / 2.0
    cp = (n_warp - 1) / 2.0
    dx = pitch / cps_per_crossing
    n_cp = n_weft * cps_per_crossing + 3
    k = np.arange(n_cp, dtype=np.float64)
    ctrl, off = [], [0]
    # warp: along x
    xs = (-cw - 0.5) * pitch - dx + k * dx
    for i in range(n_warp):
        y = (i - cp) * pitch
        z = 0.5 * radius * np.cos(math.pi * (xs / pitch + cw) + math.pi * i)
        ctrl.append(np.stack([xs, np.full(n_cp, y), z, np.full(n_cp, radius)], 1))
        off.append(off[-1] + n_cp)
    n_cp2 = n_warp * cps_per_crossing + 3
    k2 = np.arange(n_cp2, dtype=np.float64)
    ys = (-cp - 0.5) * pitch - dx + k2 * dx
    for j in range(n_weft):
        x = (j - cw) * pitch
        z = -0.5 * radius * np.cos(math.pi * (ys / pitch + cp) + math.pi * j)
        ctrl.append(np.stack([np.full(n_cp2, x), ys, z, np.full(n_cp2, radius)], 1))
        off.append(off[-1] + n_cp2)
    ctrl = np.concatenate(ctrl).astype(np.float32)
    n_yarns = n_warp + n_weft
    phase = (2.0 * math.pi * _rng(seed).random(n_yarns)).astype(np.float32)
    return ctrl, np.array(off, np.int64), np.zeros(n_yarns, np.int32), phase


def camera(eye, look_at, up=(0.0, 0.0, 1.0), vfov_deg: float = 30.0, width: int = 1920,
           height: int = 1080):
    """Pinhole camera record: eye, look-at, up, vertical field of view,
    resolution (the renderer generates the rays from it)."""
    return dict(eye=tuple(float(np.float32(e)) for e in eye),
                look_at=tuple(float(np.float32(e)) for e in look_at),
                up=tuple(float(np.float32(e)) for e in up), vfov=float(np.float32(vfov_deg * DEG)),
                width=int(width), height=int(height))


def weave_camera():
    """Grazing view of the weave: eye 45 units back and 12 up from the
    fabric centre, looking at the centre, 1920 x 1080, 30 degrees."""
    return camera((0.0, -45.0, 12.0), (0.0, 0.0, 0.0))


def pinhole_rays(cam: dict, px, py, jx=None, jy=None):
    """Primary rays through pixels (px, py) (pixel centres, or offsets jx,
    jy in [0, 1)); row 0 is the top of the image.  Returns (o (n, 3), d (n,
    3)) float32 with unit directions.  The renderer's own camera code is
    separate; this generator feeds intersection tests."""
    eye = np.array(cam["eye"], np.float64)
    f = np.array(cam["look_at"], np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.array(cam["up"], np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(0.5 * cam["vfov"])
    W, H = cam["width"], cam["height"]
    jx = 0.5 if jx is None else jx
    jy = 0.5 if jy is None else jy
    sx = (2.0 * (np.asarray(px, np.float64) + jx) / W - 1.0) * th * W / H
    sy = (1.0 - 2.0 * (np.asarray(py, np.float64) + jy) / H) * th
    d = f[None, :] + sx[:, None] * r[None, :] + sy[:, None] * u[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.repeat(eye[None, :], len(d), 0)
    return o.astype(np.float32), d.astype(np.float32)


def random_rays(n: int, seed: int, lo, hi, target_lo=None, target_hi=None):
    """Rays from origins uniform in the box [lo, hi] towards points uniform
    in [target_lo, target_hi] (default: the same box)."""
    rng = _rng(seed)
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    tl = lo if target_lo is None else np.asarray(target_lo, np.float64)
    th = hi if target_hi is None else np.asarray(target_hi, np.float64)
    o = lo + (hi - lo) * rng.random((n, 3))
    t = tl + (th - tl) * rng.random((n, 3))
    d = t - o
    d /= np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-30)
    return o.astype(np.float32), d.astype(np.float32)
