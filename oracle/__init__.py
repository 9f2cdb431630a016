"""FP64 CPU oracle of the BYSDF (arXiv 2401.12724) -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it.

The arithmetic lives in ``bysdf_oracle.c`` (plain C, double precision,
OpenMP over queries); this module only marshals numpy arrays through ctypes.
Queries are the same FP32 arrays the GPU consumes, promoted to double inside.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bysdf_oracle.c")
_SOURCES = [_SRC, os.path.join(_HERE, "yarn_oracle.c"), os.path.join(_HERE, "render_oracle.c")]
_HEADERS = [os.path.join(_HERE, "bysdf_oracle.h"), os.path.join(_HERE, "yarn_oracle.h"),
            os.path.join(_HERE, "render_oracle.h")]
_LIB = os.path.join(_HERE, "liboracle.so")

# flag bits (same numbering as the library's public flags)
PASS_THROUGH = 1 << 0
ILLCOND = 1 << 1
NEARTIE = 1 << 2
NEARTANGENT = 1 << 3
AXIAL = 1 << 4
BACKFACING = 1 << 5
SAMPLE_FAIL = 1 << 6
NEAR_LOBE_BOUNDARY = 1 << 7
NEAR_TIR = 1 << 8
BAD_INPUT = 1 << 9
MARGIN_MASK = ILLCOND | NEARTIE | NEARTANGENT | NEAR_LOBE_BOUNDARY | NEAR_TIR


class OrcParams(C.Structure):
    _fields_ = [
        ("n_plies", C.c_int32), ("fibers_per_ply", C.c_int32), ("K", C.c_int32),
        ("n_iter", C.c_int32), ("tex_size", C.c_int32),
        ("ply_radius", C.c_double), ("ply_center_radius", C.c_double),
        ("fiber_radius", C.c_double), ("ply_twist", C.c_double),
        ("fiber_twist", C.c_double), ("eta", C.c_double), ("albedo", C.c_double * 3),
        ("beta", C.c_double), ("aniso", C.c_double), ("k_spec", C.c_double),
        ("B", C.c_double), ("r", C.c_double), ("sigma_t", C.c_double),
        ("ply_density", C.c_double), ("fiber_density", C.c_double),
        ("shadow_halfwidth", C.c_double),
        ("mig_tables", C.c_int32), ("mig_period", C.c_double), ("mig_blend", C.c_double),
        ("mig_spread", C.c_double), ("mig_seed", C.c_uint32),
    ]


class RenderSettings(C.Structure):
    _fields_ = [
        ("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
        ("vfov", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
        ("crop_x", C.c_int32), ("crop_y", C.c_int32), ("crop_w", C.c_int32), ("crop_h", C.c_int32),
        ("light_corner", C.c_float * 3), ("light_u", C.c_float * 3), ("light_v", C.c_float * 3),
        ("light_radiance", C.c_float * 3), ("env_radiance", C.c_float * 3),
        ("spp", C.c_int32), ("max_depth", C.c_int32), ("lod_px", C.c_float), ("n_h", C.c_int32),
        ("seed", C.c_uint64), ("ray_eps", C.c_float), ("nee", C.c_int32),
        ("multiscale", C.c_int32), ("grad_type", C.c_int32),
    ]


def render_settings_struct(rs: dict) -> RenderSettings:
    s = RenderSettings()
    rs = dict(rs)
    rs.setdefault("nee", 1)
    rs.setdefault("multiscale", 0)
    rs.setdefault("grad_type", -1)
    for k, _ in RenderSettings._fields_:
        v = rs[k]
        if isinstance(v, (tuple, list)):
            getattr(s, k)[:] = [float(x) for x in v]
        else:
            setattr(s, k, v)
    return s


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99, -O2, OpenMP, IEEE math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(f) for f in _SOURCES + _HEADERS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp] + _SOURCES + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = bind(build())
    return _lib


def bind(path: str):
    """Load an oracle library built from these sources (or from a variant of
    them, for the tests that check the pins catch planted mistakes) and
    declare its entry points."""
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    fp = C.POINTER(C.c_float)
    ip = C.POINTER(C.c_int32)
    up = C.POINTER(C.c_uint32)
    pp = C.POINTER(OrcParams)
    tp = C.POINTER(dp)
    L.orc_table.argtypes = [pp, dp]
    L.orc_mig_table.argtypes = [pp, C.c_int64, C.c_int32]
    L.orc_mig_table.restype = C.c_int32
    L.orc_fiber_lookup.argtypes = [pp, dp, C.c_double, C.c_double, C.c_int32, dp]
    L.orc_fiber_lookup.restype = None
    L.orc_eval.argtypes = [pp, tp, C.c_int32, C.c_int64, ip, fp, fp, fp, fp, fp, fp, dp, up,
                           C.c_int]
    L.orc_sample.argtypes = [pp, tp, C.c_int32, C.c_int64, ip, fp, fp, fp, fp, fp, fp, dp,
                             up, C.c_int]
    L.orc_furnace.argtypes = [pp, tp, C.c_int32, C.c_int64, C.c_int32, ip, fp, fp, fp, fp,
                              fp, fp, dp, dp, C.c_int]
    L.orc_eval_far.argtypes = [pp, tp, C.c_int32, C.c_int64, C.c_int32, C.c_double, ip, fp,
                               fp, fp, fp, dp, C.c_int]
    L.orc_eval_multi.argtypes = [pp, tp, C.c_int32, C.c_int64, C.c_int32, ip, fp, fp, fp, fp,
                                 fp, fp, fp, fp, fp, dp, up, C.c_int]
    L.orc_sample_multi.argtypes = [pp, tp, C.c_int32, C.c_int64, C.c_int32, ip, fp, fp, fp,
                                   fp, fp, fp, fp, fp, fp, fp, dp, up, C.c_int]
    L.orc_footprint.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                dp, dp]
    L.orc_footprint.restype = C.c_int32
    L.orc_grad_fd.argtypes = [pp, tp, C.c_int32, C.c_int64, ip, fp, fp, fp, fp, fp, fp,
                              C.c_double, dp, dp, C.c_int]
    L.orc_philox4x32_10.argtypes = [up, up, up]
    L.orc_fresnel.argtypes = [C.c_double, C.c_double]
    L.orc_fresnel.restype = C.c_double
    L.orc_ggx_D.argtypes = [dp, C.c_double, C.c_double]
    L.orc_ggx_D.restype = C.c_double
    L.orc_smith_G1.argtypes = [dp, dp, C.c_double, C.c_double]
    L.orc_smith_G1.restype = C.c_double
    L.orc_vndf.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, dp]
    L.orc_ls_albedo.argtypes = [C.c_double]
    L.orc_ls_albedo.restype = C.c_double
    L.orc_ply_shadow_raw.argtypes = [pp, C.c_double, C.c_double]
    L.orc_ply_shadow_raw.restype = C.c_double
    L.orc_ply_hit.argtypes = [pp, C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_ply_hit.restype = C.c_uint32
    L.orc_set_margins.argtypes = [C.c_double] * 5
    L.orc_nodes.argtypes = [pp, dp, C.c_double, C.c_double, C.c_double, dp, dp, dp]
    L.orc_nodes.restype = C.c_uint32
    L.orc_ply_frame.argtypes = [pp, C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_ply_frame.restype = C.c_uint32
    L.orc_explicit_ply.argtypes = [pp, C.c_double, C.c_double, C.c_double, C.c_double, dp,
                                   C.c_double, dp]
    L.orc_explicit_ply.restype = C.c_int32
    L.orc_frame_x.argtypes = [pp, dp, C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_frame_x.restype = C.c_uint32
    L.orc_camera_footprint.argtypes = [C.c_void_p, C.POINTER(RenderSettings), C.c_double,
                                       C.c_double, dp]
    L.orc_camera_footprint.restype = C.c_int32
    L.orc_scene_create.argtypes = [fp, C.POINTER(C.c_int64), C.c_int32]
    L.orc_scene_create.restype = C.c_void_p
    L.orc_scene_free.argtypes = [C.c_void_p]
    L.orc_scene_frame.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, dp]
    L.orc_intersect.argtypes = [C.c_void_p, C.c_int64, fp, fp, fp, C.c_double, dp, C.c_int]
    L.orc_render.argtypes = [C.c_void_p, pp, tp, C.c_int32, ip, fp, C.POINTER(RenderSettings),
                             dp, dp, dp, C.c_int]
    return L


# ---------------------------------------------------------------- helpers

def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def params_struct(d: dict) -> OrcParams:
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        if name == "albedo":
            for c in range(3):
                p.albedo[c] = float(d["albedo"][c])
        else:
            setattr(p, name, d[name])
    return p


class TypeSet:
    """Parameter records and their fiber tables, built by the oracle."""

    def __init__(self, param_dicts):
        self.dicts = [dict(d) for d in param_dicts]
        n = len(self.dicts)
        self.structs = (OrcParams * n)()
        for i, d in enumerate(self.dicts):
            self.structs[i] = params_struct(d)
        self.tables = []
        cache = {}
        for i, d in enumerate(self.dicts):
            key = (d["fibers_per_ply"], float(d["fiber_radius"]), d["tex_size"],
                   max(1, d["mig_tables"]), float(d["mig_spread"]), d["mig_seed"])
            if key not in cache:
                cache[key] = table(d)
            self.tables.append(cache[key])
        self._tp = (C.POINTER(C.c_double) * n)(*[_ptr(t, C.c_double) for t in self.tables])

    def __len__(self):
        return len(self.dicts)


def table(d: dict) -> np.ndarray:
    """Fiber tables of one parameter record: max(1, mig_tables) tables of
    N_u texels, stacked ((tables x N_u) x 3: dn, rho_hat, G_f)."""
    tab = np.zeros((max(1, d["mig_tables"]) * d["tex_size"], 3), dtype=np.float64)
    p = params_struct(d)
    rc = lib().orc_table(C.byref(p), _ptr(tab, C.c_double))
    if rc != 0:
        raise ValueError("invalid fiber-table parameters")
    return tab


def mig_table(d: dict, q: int, k: int) -> int:
    """Fiber-migration table index of ply k in period q."""
    return int(lib().orc_mig_table(C.byref(params_struct(d)), q, k))


def fiber_lookup(d: dict, tab: np.ndarray, uf: float, vply: float, k: int) -> np.ndarray:
    """Fiber-table values (dn, rho_hat, G_f) at fiber phase uf, ply arc
    length vply, on ply k (tab from table(d))."""
    out = np.zeros(3)
    t = np.ascontiguousarray(tab, np.float64)
    lib().orc_fiber_lookup(C.byref(params_struct(d)), _ptr(t, C.c_double), uf, vply, k,
                           _ptr(out, C.c_double))
    return out


def _types(ts):
    return ts if isinstance(ts, TypeSet) else TypeSet(ts)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def eval(ts, q: dict, nthreads: int = 0):
    """BYSDF value and pdf.  Returns (out[n,13] float64, flags[n] uint32)."""
    ts = _types(ts)
    n = len(q["h"])
    out = np.zeros((n, 13), dtype=np.float64)
    flags = np.zeros(n, dtype=np.uint32)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    h, u, v = _f32(q["h"]), _f32(q["u"]), _f32(q["v"])
    wi, wo = _f32(q["wi"]), _f32(q["wo"])
    sh = _f32(q["shift"]) if q.get("shift") is not None else None
    lib().orc_eval(ts.structs, ts._tp, len(ts), n, _ptr(tpe, C.c_int32), _ptr(h, C.c_float),
                   _ptr(u, C.c_float), _ptr(v, C.c_float), _ptr(wi, C.c_float),
                   _ptr(wo, C.c_float), _ptr(sh, C.c_float), _ptr(out, C.c_double),
                   _ptr(flags, C.c_uint32), nthreads)
    return out, flags


def sample(ts, q: dict, nthreads: int = 0):
    """Importance sampling.  Returns (out[n,12] float64, flags[n] uint32):
    wo(3) weight(3) pdf exit(3) lobe node."""
    ts = _types(ts)
    n = len(q["h"])
    out = np.zeros((n, 12), dtype=np.float64)
    flags = np.zeros(n, dtype=np.uint32)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    h, u, v = _f32(q["h"]), _f32(q["u"]), _f32(q["v"])
    wi, xi = _f32(q["wi"]), _f32(q["xi"])
    sh = _f32(q["shift"]) if q.get("shift") is not None else None
    lib().orc_sample(ts.structs, ts._tp, len(ts), n, _ptr(tpe, C.c_int32), _ptr(h, C.c_float),
                     _ptr(u, C.c_float), _ptr(v, C.c_float), _ptr(wi, C.c_float),
                     _ptr(xi, C.c_float), _ptr(sh, C.c_float), _ptr(out, C.c_double),
                     _ptr(flags, C.c_uint32), nthreads)
    return out, flags


def furnace(ts, q: dict, block: int, nthreads: int = 0):
    ts = _types(ts)
    n = len(q["h"])
    nb = n // block
    mean = np.zeros((nb, 3), dtype=np.float64)
    var = np.zeros((nb, 3), dtype=np.float64)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    h, u, v = _f32(q["h"]), _f32(q["u"]), _f32(q["v"])
    wi, xi = _f32(q["wi"]), _f32(q["xi"])
    sh = _f32(q["shift"]) if q.get("shift") is not None else None
    rc = lib().orc_furnace(ts.structs, ts._tp, len(ts), n, block, _ptr(tpe, C.c_int32),
                           _ptr(h, C.c_float), _ptr(u, C.c_float), _ptr(v, C.c_float),
                           _ptr(wi, C.c_float), _ptr(xi, C.c_float), _ptr(sh, C.c_float),
                           _ptr(mean, C.c_double), _ptr(var, C.c_double), nthreads)
    if rc != 0:
        raise ValueError("block must be >= 2")
    return mean, var


def eval_far(ts, q: dict, n_h: int = 4, zeta: float = 0.5, nthreads: int = 0):
    ts = _types(ts)
    n = len(q["u"])
    out = np.zeros((n, 3), dtype=np.float64)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    u, v = _f32(q["u"]), _f32(q["v"])
    wi, wo = _f32(q["wi"]), _f32(q["wo"])
    lib().orc_eval_far(ts.structs, ts._tp, len(ts), n, n_h, zeta, _ptr(tpe, C.c_int32),
                       _ptr(u, C.c_float), _ptr(v, C.c_float), _ptr(wi, C.c_float),
                       _ptr(wo, C.c_float), _ptr(out, C.c_double), nthreads)
    return out


def eval_multi(ts, q: dict, n_max: int = 4, nthreads: int = 0):
    """Multi-scale BYSDF (Sec. 4.2, Eq. 8-11) at wo over the footprint
    (h1, h, h2) with strata offset zeta.  Returns (out[n,13], flags[n])
    laid out as eval."""
    ts = _types(ts)
    n = len(q["h"])
    out = np.zeros((n, 13), dtype=np.float64)
    flags = np.zeros(n, dtype=np.uint32)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    a = [_f32(q[k]) for k in ("h", "h1", "h2", "zeta", "u", "v", "wi", "wo")]
    sh = _f32(q["shift"]) if q.get("shift") is not None else None
    rc = lib().orc_eval_multi(ts.structs, ts._tp, len(ts), n, n_max, _ptr(tpe, C.c_int32),
                              *[_ptr(x, C.c_float) for x in a], _ptr(sh, C.c_float),
                              _ptr(out, C.c_double), _ptr(flags, C.c_uint32), nthreads)
    if rc != 0:
        raise ValueError("n_max out of range")
    return out, flags


def sample_multi(ts, q: dict, n_max: int = 4, nthreads: int = 0):
    """Multi-scale sampler: xi_s picks a stratum with probability W / sum W.
    Returns (out[n,13], flags[n]): wo(3) weight(3) pdf exit(3) lobe node
    stratum."""
    ts = _types(ts)
    n = len(q["h"])
    out = np.zeros((n, 13), dtype=np.float64)
    flags = np.zeros(n, dtype=np.uint32)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    a = [_f32(q[k]) for k in ("h", "h1", "h2", "zeta", "xi_s", "u", "v", "wi", "xi")]
    sh = _f32(q["shift"]) if q.get("shift") is not None else None
    rc = lib().orc_sample_multi(ts.structs, ts._tp, len(ts), n, n_max, _ptr(tpe, C.c_int32),
                                *[_ptr(x, C.c_float) for x in a], _ptr(sh, C.c_float),
                                _ptr(out, C.c_double), _ptr(flags, C.c_uint32), nthreads)
    if rc != 0:
        raise ValueError("n_max out of range")
    return out, flags


def footprint(h0, h1, h2, zeta, n_max: int = 4):
    """Strata of one footprint: (offsets, weights)."""
    hs = np.zeros(16)
    ws = np.zeros(16)
    k = lib().orc_footprint(float(h0), float(h1), float(h2), float(zeta), n_max,
                            _ptr(hs, C.c_double), _ptr(ws, C.c_double))
    if k < 0:
        raise ValueError("invalid footprint")
    return hs[:k], ws[:k]


def grad_fd(ts, q: dict, gE, rel_step: float = 1e-6, nthreads: int = 0):
    """Central FD of sum gE*E wrt theta.  Returns (grad[n_types,8], per_query[n,8])."""
    ts = _types(ts)
    n = len(q["h"])
    grad = np.zeros((len(ts), 8), dtype=np.float64)
    pq = np.zeros((n, 8), dtype=np.float64)
    tpe = np.ascontiguousarray(q["type"], dtype=np.int32)
    h, u, v = _f32(q["h"]), _f32(q["u"]), _f32(q["v"])
    wi, wo = _f32(q["wi"]), _f32(q["wo"])
    g = _f32(gE)
    lib().orc_grad_fd(ts.structs, ts._tp, len(ts), n, _ptr(tpe, C.c_int32), _ptr(h, C.c_float),
                      _ptr(u, C.c_float), _ptr(v, C.c_float), _ptr(wi, C.c_float),
                      _ptr(wo, C.c_float), _ptr(g, C.c_float), rel_step,
                      _ptr(grad, C.c_double), _ptr(pq, C.c_double), nthreads)
    return grad, pq


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def set_margins(geo=1e-7, shade=2e-6, amplify=1e5, tir=1e-6, xi=1e-6):
    lib().orc_set_margins(geo, shade, amplify, tir, xi)


# thin wrappers of the closed-form internals (used by the pins)
def fresnel(cos_i, eta_rel):
    return lib().orc_fresnel(float(cos_i), float(eta_rel))


def ggx_D(m, ax, ay):
    a = np.ascontiguousarray(m, dtype=np.float64)
    return lib().orc_ggx_D(_ptr(a, C.c_double), ax, ay)


def smith_G1(w, m, ax, ay):
    a = np.ascontiguousarray(w, dtype=np.float64)
    b = np.ascontiguousarray(m, dtype=np.float64)
    return lib().orc_smith_G1(_ptr(a, C.c_double), _ptr(b, C.c_double), ax, ay)


def vndf(wi, ax, ay, u1, u2):
    a = np.ascontiguousarray(wi, dtype=np.float64)
    m = np.zeros(3, dtype=np.float64)
    lib().orc_vndf(_ptr(a, C.c_double), ax, ay, u1, u2, _ptr(m, C.c_double))
    return m


def ls_albedo(mu):
    return lib().orc_ls_albedo(float(mu))


def ply_shadow_raw(d, a, phi):
    p = params_struct(d)
    return lib().orc_ply_shadow_raw(C.byref(p), float(a), float(phi))


def eval_query(d, tab, h, u, v, wi, wo):
    """One evaluation with FP64 inputs (h, u, v as Python floats, wi and wo
    3-vectors): (out[13] as in eval, flags).  Lets a test move an input by a
    few FP64 ulps, below the resolution of the FP32 query arrays."""
    p = params_struct(d)
    t = np.ascontiguousarray(tab, dtype=np.float64)
    a = np.ascontiguousarray(wi, dtype=np.float64)
    b = np.ascontiguousarray(wo, dtype=np.float64)
    out = np.zeros(13, dtype=np.float64)
    fl = lib().orc_eval_query(C.byref(p), _ptr(t, C.c_double), C.c_double(h), C.c_double(u), C.c_double(v),
                              _ptr(a, C.c_double), _ptr(b, C.c_double), _ptr(out, C.c_double))
    return out, fl & 0xffffffff


def eval_multi_query(d, tab, h0, h1, h2, zeta, n_max, u, v, wi, wo):
    """One multi-scale evaluation with FP64 inputs: (out[13] as in
    eval_multi, flags)."""
    p = params_struct(d)
    t = np.ascontiguousarray(tab, dtype=np.float64)
    a = np.ascontiguousarray(wi, dtype=np.float64)
    b = np.ascontiguousarray(wo, dtype=np.float64)
    out = np.zeros(13, dtype=np.float64)
    fl = lib().orc_eval_multi_query(C.byref(p), _ptr(t, C.c_double), C.c_double(h0), C.c_double(h1),
                                    C.c_double(h2), C.c_double(zeta), C.c_int32(n_max), C.c_double(u),
                                    C.c_double(v), _ptr(a, C.c_double), _ptr(b, C.c_double),
                                    _ptr(out, C.c_double))
    return out, fl & 0xffffffff


def ply_hit(d, h, u, v, wi):
    p = params_struct(d)
    w = np.ascontiguousarray(wi, dtype=np.float64)
    out = np.zeros(10 + 8, dtype=np.float64)
    fl = lib().orc_ply_hit(C.byref(p), float(h), float(u), float(v), _ptr(w, C.c_double),
                           _ptr(out, C.c_double))
    return out, fl


def nodes(d, tab, h, u, v, wi, shift=None):
    """Forward-node probe: (array[K,16], flags); columns kind N ell att T
    wt(3) y(3) n_y(3) p2x p2y."""
    p = params_struct(d)
    w = np.ascontiguousarray(wi, dtype=np.float64)
    t = np.ascontiguousarray(tab, dtype=np.float64)
    out = np.zeros((d["K"], 16), dtype=np.float64)
    sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.float64)
    fl = lib().orc_nodes(C.byref(p), _ptr(t, C.c_double), float(h), float(u), float(v),
                         _ptr(w, C.c_double), _ptr(sh, C.c_double), _ptr(out, C.c_double))
    return out, fl


def ply_frame(d, h, u, v, wi):
    """Implicit ply hit with the ply frame: (array[11], flags) = pass, ply,
    hit (x, y, v), tangent (3), normal (3)."""
    p = params_struct(d)
    w = np.ascontiguousarray(wi, dtype=np.float64)
    out = np.zeros(11)
    fl = lib().orc_ply_frame(C.byref(p), float(h), float(u), float(v), _ptr(w, C.c_double),
                             _ptr(out, C.c_double))
    return out, fl


def explicit_ply(d, kappa, h, u, v, wi, step=2e-3):
    """Explicit helical plies around a circular-arc yarn of curvature kappa:
    (first_hit_ok, array[7] = ply, hit (3), tangent (3))."""
    p = params_struct(d)
    w = np.ascontiguousarray(wi, dtype=np.float64)
    out = np.zeros(7)
    ok = lib().orc_explicit_ply(C.byref(p), float(kappa), float(h), float(u), float(v),
                                _ptr(w, C.c_double), float(step), _ptr(out, C.c_double))
    return bool(ok), out


def frame_x(d, tab, h, u, v, wi):
    """Shading-frame probe: (array[16], flags): t b n Gp Gf mu_i w(4)."""
    p = params_struct(d)
    w = np.ascontiguousarray(wi, dtype=np.float64)
    t = np.ascontiguousarray(tab, dtype=np.float64)
    out = np.zeros(16, dtype=np.float64)
    fl = lib().orc_frame_x(C.byref(p), _ptr(t, C.c_double), float(h), float(u), float(v),
                           _ptr(w, C.c_double), _ptr(out, C.c_double))
    return out, fl


# ---------------------------------------------------------------- yarn scenes

HIT_MISS = 1 << 0
HIT_CAP = 1 << 1
HIT_EXCLUDED = 1 << 2
HIT_GRAZING = 1 << 3
HIT_TIE = 1 << 4
HIT_ORIGIN_EDGE = 1 << 5
HIT_MARGIN_MASK = HIT_GRAZING | HIT_TIE | HIT_ORIGIN_EDGE


class Scene:
    """Yarn scene for the intersection oracle: ctrl (n_cp, 4) float32 rows
    (x, y, z, r), yarn_off (n_yarns + 1) int64 CSR offsets."""

    def __init__(self, ctrl, yarn_off):
        self.ctrl = np.ascontiguousarray(ctrl, np.float32)
        self.off = np.ascontiguousarray(yarn_off, np.int64)
        self._h = lib().orc_scene_create(_ptr(self.ctrl, C.c_float),
                                         self.off.ctypes.data_as(C.POINTER(C.c_int64)),
                                         len(self.off) - 1)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_scene_free(self._h)
            self._h = None

    def frame(self, yarn, seg, s):
        """(T(3), N(3), v, position(3)) of the centreline at (yarn, seg, s)."""
        out = np.zeros(10)
        lib().orc_scene_frame(self._h, int(yarn), int(seg), float(s), _ptr(out, C.c_double))
        return out


def intersect(scene: Scene, o, d, t_max, t_min: float = 0.0, nthreads: int = 0):
    """Rays (n, 3) float32 origins and directions, t_max (n,).  Returns
    (n, 16) float64: t, yarn, seg, s, h, v, T(3), N(3), flags, depth, _,
    second-best entry of another yarn."""
    o = np.ascontiguousarray(o, np.float32)
    d = np.ascontiguousarray(d, np.float32)
    tm = np.ascontiguousarray(t_max, np.float32)
    n = len(o)
    out = np.zeros((n, 16))
    lib().orc_intersect(scene._h, n, _ptr(o, C.c_float), _ptr(d, C.c_float), _ptr(tm, C.c_float),
                        float(t_min), _ptr(out, C.c_double), nthreads)
    return out


def camera_footprint(scene: Scene, rs: dict, px: float, py: float):
    """(yarn, h0, h1, h2) of the camera ray through pixel position (px, py)."""
    st = render_settings_struct(rs)
    out = np.zeros(3)
    y = lib().orc_camera_footprint(scene._h, C.byref(st), float(px), float(py),
                                   _ptr(out, C.c_double))
    return int(y), out[0], out[1], out[2]


def render(scene: Scene, ts, yarn_type, yarn_phase, rs: dict, nthreads: int = 0):
    """Crop of the image by the CPU path tracer (render_oracle.c).  ts: a
    TypeSet (or parameter dicts) indexed by yarn_type.  Returns (mean
    (crop_h, crop_w, 3), mean of squares (crop_h, crop_w, 3)); with
    rs["grad_type"] >= 0 also the gradient (crop_h, crop_w, 3, 3) of the
    image with respect to (r, k^B_c, sigma_t) of that type."""
    ts = _types(ts)
    yt = np.ascontiguousarray(yarn_type, np.int32)
    ph = np.ascontiguousarray(yarn_phase, np.float32)
    st = render_settings_struct(rs)
    fb = np.zeros((rs["crop_h"], rs["crop_w"], 3))
    sq = np.zeros_like(fb)
    want = rs.get("grad_type", -1) >= 0
    gr = np.zeros((rs["crop_h"], rs["crop_w"], 3, 3)) if want else None
    lib().orc_render(scene._h, ts.structs, ts._tp, len(ts), _ptr(yt, C.c_int32),
                     _ptr(ph, C.c_float), C.byref(st), _ptr(fb, C.c_double), _ptr(sq, C.c_double),
                     _ptr(gr, C.c_double), nthreads)
    return (fb, sq, gr) if want else (fb, sq)
