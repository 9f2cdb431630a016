"""Python binding of libbysdf.so (include/bysdf.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors (``device='cuda'``), used as plain
device memory; the stream is torch's current stream unless one is given.
The functions carry the names of the C entry points.

Layouts (device tensors):
  queries   type int32[n]; h, u, v float32[n]; wi, wo, xi float32[3, n];
            shift float32[2, n] (optional)
  eval      float32[12, n] rows E_r E_g E_b E_xS E_yS E_xB_rgb E_yB_rgb pdf,
            flags int32[n] (bit pattern of the uint32 flags)
  sample    float32[10, n] rows wo_xyz w_rgb pdf exit_xyz, lobe int32[n],
            node int32[n], flags int32[n]
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# BYSDF_LIB selects another build of the same library (tuning experiments)
LIB_PATH = os.environ.get("BYSDF_LIB", os.path.join(_HERE, "libbysdf.so"))

OK = 0
ERR_INVALID_ARG = -1
ERR_INVALID_PARAM = -2
ERR_OOM = -3
ERR_LAUNCH = -4
ERR_UNSUPPORTED_DEVICE = -5

FLAG_PASS_THROUGH = 1 << 0
FLAG_AXIAL = 1 << 4
FLAG_BACKFACING = 1 << 5
FLAG_SAMPLE_FAIL = 1 << 6
FLAG_BAD_INPUT = 1 << 9

_vp = C.c_void_p


class TypeParams(C.Structure):
    _fields_ = [
        ("n_plies", C.c_int32), ("fibers_per_ply", C.c_int32), ("K", C.c_int32),
        ("n_iter", C.c_int32), ("tex_size", C.c_int32),
        ("ply_radius", C.c_float), ("ply_center_radius", C.c_float),
        ("fiber_radius", C.c_float), ("ply_twist", C.c_float), ("fiber_twist", C.c_float),
        ("eta", C.c_float), ("albedo", C.c_float * 3), ("beta", C.c_float),
        ("aniso", C.c_float), ("k_spec", C.c_float), ("B", C.c_float), ("r", C.c_float),
        ("sigma_t", C.c_float), ("ply_density", C.c_float), ("fiber_density", C.c_float),
        ("shadow_halfwidth", C.c_float),
        ("mig_tables", C.c_int32), ("mig_period", C.c_float), ("mig_blend", C.c_float),
        ("mig_spread", C.c_float), ("mig_seed", C.c_uint32),
    ]


class QuerySoA(C.Structure):
    _fields_ = [(n, _vp) for n in ("type_id", "h", "u", "v", "wi_x", "wi_y", "wi_z",
                                   "wo_x", "wo_y", "wo_z", "shift0", "shift1")]


class EvalOutSoA(C.Structure):
    _fields_ = [(n, _vp) for n in ("E_r", "E_g", "E_b", "E_xS", "E_yS", "E_xB_r", "E_xB_g",
                                   "E_xB_b", "E_yB_r", "E_yB_g", "E_yB_b", "pdf", "flags")]


class SampleSoA(C.Structure):
    _fields_ = [(n, _vp) for n in ("type_id", "h", "u", "v", "wi_x", "wi_y", "wi_z",
                                   "xi0", "xi1", "xi2", "shift0", "shift1")] + [("seed", C.c_uint64)]


class PlyOutSoA(C.Structure):
    _fields_ = [(n, _vp) for n in ("ply", "p_x", "p_y", "p_z", "t_x", "t_y", "t_z", "n_x", "n_y", "n_z",
                                   "flags")]


class FootprintSoA(C.Structure):
    _fields_ = [(n, _vp) for n in ("h1", "h2", "zeta", "xi_s")]


class Schedule(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("grid", C.c_int32), ("use_lds", C.c_int32),
                ("block", C.c_int32), ("min_waves", C.c_int32)]


class SampleOutSoA(C.Structure):
    _fields_ = [(n, _vp) for n in ("wo_x", "wo_y", "wo_z", "w_r", "w_g", "w_b", "pdf",
                                   "exit_x", "exit_y", "exit_z", "lobe", "node", "flags")]


_lib = None


class RaySoA(C.Structure):
    _fields_ = [(k, _vp) for k in ("o_x", "o_y", "o_z", "d_x", "d_y", "d_z", "t_max")]


HIT_FIELDS = ("t", "yarn", "seg", "s", "h", "u", "v", "tan_x", "tan_y", "tan_z", "nrm_x",
              "nrm_y", "nrm_z", "flags")


class HitSoA(C.Structure):
    _fields_ = [(k, _vp) for k in HIT_FIELDS]


class RenderSettings(C.Structure):
    _fields_ = [
        ("eye", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
        ("vfov", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
        ("crop_x", C.c_int32), ("crop_y", C.c_int32), ("crop_w", C.c_int32), ("crop_h", C.c_int32),
        ("light_corner", C.c_float * 3), ("light_u", C.c_float * 3), ("light_v", C.c_float * 3),
        ("light_radiance", C.c_float * 3), ("env_radiance", C.c_float * 3),
        ("spp", C.c_int32), ("max_depth", C.c_int32), ("lod_px", C.c_float), ("n_h", C.c_int32),
        ("seed", C.c_uint64), ("ray_eps", C.c_float), ("spp_batch", C.c_int32),
        ("multiscale", C.c_int32),
    ]


def lib():
    """Load libbysdf.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbysdf.so is not built: run `python -m paper_2401_12724_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.bysdf_version.restype = C.c_char_p
        L.bysdf_last_error.restype = C.c_char_p
        L.bysdf_types_create.argtypes = [C.POINTER(TypeParams), C.c_int32, C.POINTER(_vp), _vp]
        L.bysdf_types_destroy.argtypes = [_vp]
        L.bysdf_types_count.argtypes = [_vp]
        L.bysdf_types_count.restype = C.c_int32
        L.bysdf_types_table.argtypes = [_vp, C.c_int32, C.POINTER(C.c_float), C.c_int64]
        L.bysdf_types_set_theta.argtypes = [_vp, _vp, _vp]
        L.bysdf_eval.argtypes = [_vp, C.POINTER(QuerySoA), C.c_int64, C.POINTER(EvalOutSoA), _vp]
        L.bysdf_sample_pdf.argtypes = [_vp, C.POINTER(SampleSoA), C.c_int64,
                                       C.POINTER(SampleOutSoA), _vp]
        L.bysdf_eval_sample.argtypes = [_vp, C.POINTER(QuerySoA), _vp, _vp, _vp, C.c_int64,
                                        C.POINTER(EvalOutSoA), C.POINTER(SampleOutSoA), _vp]
        L.bysdf_ply_geometry.argtypes = [_vp, C.POINTER(QuerySoA), C.c_int64, C.POINTER(PlyOutSoA), _vp]
        L.bysdf_eval_multi.argtypes = [_vp, C.POINTER(QuerySoA), C.POINTER(FootprintSoA),
                                       C.c_int64, C.c_int32, C.POINTER(EvalOutSoA), _vp]
        L.bysdf_sample_multi.argtypes = [_vp, C.POINTER(SampleSoA), C.POINTER(FootprintSoA),
                                         C.c_int64, C.c_int32, C.POINTER(SampleOutSoA), _vp]
        L.bysdf_furnace_blocks.argtypes = [_vp, C.POINTER(SampleSoA), C.c_int64, C.c_int32, _vp,
                                           _vp, _vp]
        L.bysdf_batched_workspace_size.argtypes = [C.c_int32]
        L.bysdf_batched_workspace_size.restype = C.c_size_t
        L.bysdf_eval_batched.argtypes = [_vp, _vp, C.c_int64, C.POINTER(QuerySoA),
                                         C.POINTER(EvalOutSoA), C.POINTER(Schedule), _vp,
                                         C.c_size_t, _vp]
        L.bysdf_eval_batched_noalloc.argtypes = [_vp, _vp, C.c_int64, C.POINTER(QuerySoA),
                                                 C.POINTER(EvalOutSoA), C.POINTER(Schedule), _vp]
        L.bysdf_backward_workspace_size.argtypes = [C.c_int64, C.c_int32]
        L.bysdf_backward_workspace_size.restype = C.c_size_t
        L.bysdf_eval_backward.argtypes = [_vp, C.POINTER(QuerySoA), C.c_int64, _vp, _vp, _vp, _vp,
                                          _vp, C.c_size_t, _vp]
        L.yarn_scene_create.argtypes = [_vp, _vp, C.c_int32, _vp, _vp, C.POINTER(_vp), _vp]
        L.yarn_scene_destroy.argtypes = [_vp]
        L.yarn_scene_build_threads.argtypes = [C.c_int32]
        L.yarn_scene_info.argtypes = [_vp, C.POINTER(C.c_int64)]
        L.yarn_tube_intersect.argtypes = [_vp, C.POINTER(RaySoA), C.c_int64, C.c_float,
                                          C.POINTER(HitSoA), _vp]
        L.shade_wavefront_workspace_size.argtypes = [C.POINTER(RenderSettings)]
        L.shade_wavefront_workspace_size.restype = C.c_size_t
        L.shade_wavefront.argtypes = [_vp, _vp, C.POINTER(RenderSettings), _vp, _vp, C.c_size_t,
                                      C.POINTER(C.c_int64), _vp]
        L.shade_wavefront_grad_workspace_size.argtypes = [C.POINTER(RenderSettings)]
        L.shade_wavefront_grad_workspace_size.restype = C.c_size_t
        L.shade_wavefront_grad.argtypes = [_vp, _vp, C.POINTER(RenderSettings), C.c_int32, _vp, _vp, _vp,
                                           C.c_size_t, C.POINTER(C.c_int64), _vp]
        L.bysdf_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.bysdf_philox4x32_10.restype = None
        _lib = L
    return _lib


def _check(rc, name):
    if rc != 0:
        msg = lib().bysdf_last_error().decode()
        raise RuntimeError("%s failed (%d): %s" % (name, rc, msg))


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream) if not hasattr(stream, "cuda_stream") else stream.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def params_array(dicts):
    n = len(dicts)
    arr = (TypeParams * n)()
    for i, d in enumerate(dicts):
        p = arr[i]
        for name, _ in TypeParams._fields_:
            if name == "albedo":
                for c in range(3):
                    p.albedo[c] = float(d["albedo"][c])
            else:
                setattr(p, name, d[name])
    return arr


class Types:
    """Owning wrapper of a bysdf_types_t handle."""

    def __init__(self, handle, n_types, dicts):
        self.handle = handle
        self.n_types = n_types
        self.dicts = dicts

    def __del__(self):
        # at interpreter shutdown module globals may already be gone
        if getattr(self, "handle", None) and _lib is not None:
            _lib.bysdf_types_destroy(self.handle)
            self.handle = None


def bysdf_version() -> str:
    return lib().bysdf_version().decode()


def bysdf_types_create(param_dicts, stream=None) -> Types:
    arr = params_array(param_dicts)
    h = _vp()
    _check(lib().bysdf_types_create(arr, len(param_dicts), C.byref(h), _stream(stream)),
           "bysdf_types_create")
    return Types(h, len(param_dicts), [dict(d) for d in param_dicts])


def bysdf_types_destroy(types: Types):
    if types.handle:
        _check(lib().bysdf_types_destroy(types.handle), "bysdf_types_destroy")
        types.handle = None


def bysdf_types_table(types: Types, type_index: int) -> np.ndarray:
    """Fiber tables of a type: ((tables x tex_size) x 3) float32."""
    d = types.dicts[type_index]
    nu = max(1, d.get("mig_tables", 1)) * d["tex_size"]
    out = np.zeros((nu, 3), dtype=np.float32)
    _check(lib().bysdf_types_table(types.handle, type_index,
                                   out.ctypes.data_as(C.POINTER(C.c_float)), out.size),
           "bysdf_types_table")
    return out


def bysdf_types_set_theta(types: Types, theta, stream=None):
    """theta: float32 cuda tensor [n_types, 8] (contiguous)."""
    assert theta.is_cuda and theta.dtype.itemsize == 4 and theta.is_contiguous()
    assert theta.numel() == 8 * types.n_types
    _check(lib().bysdf_types_set_theta(types.handle, theta.data_ptr(), _stream(stream)),
           "bysdf_types_set_theta")


def to_device(q: dict, device="cuda"):
    """numpy query dict -> dict of contiguous torch tensors on the device."""
    import torch
    out = {}
    for k, v in q.items():
        if v is None:
            out[k] = None
            continue
        a = np.ascontiguousarray(v)
        dt = torch.int32 if a.dtype.kind in "iu" else torch.float32
        out[k] = torch.from_numpy(a.astype(np.int32 if dt == torch.int32 else np.float32)).to(device)
    return out


def _qsoa(q):
    s = QuerySoA()
    s.type_id, s.h, s.u, s.v = _ptr(q["type"]), _ptr(q["h"]), _ptr(q["u"]), _ptr(q["v"])
    wi, wo = q["wi"], q["wo"]
    s.wi_x, s.wi_y, s.wi_z = _ptr(wi[0]), _ptr(wi[1]), _ptr(wi[2])
    s.wo_x, s.wo_y, s.wo_z = _ptr(wo[0]), _ptr(wo[1]), _ptr(wo[2])
    sh = q.get("shift")
    s.shift0, s.shift1 = (_ptr(sh[0]), _ptr(sh[1])) if sh is not None else (None, None)
    return s


def _ssoa(q):
    """Sampler queries; without q["xi"] the library draws the uniforms from
    Philox keyed by q["seed"] (default 0)."""
    s = SampleSoA()
    s.type_id, s.h, s.u, s.v = _ptr(q["type"]), _ptr(q["h"]), _ptr(q["u"]), _ptr(q["v"])
    wi, xi = q["wi"], q.get("xi")
    s.wi_x, s.wi_y, s.wi_z = _ptr(wi[0]), _ptr(wi[1]), _ptr(wi[2])
    if xi is not None:
        s.xi0, s.xi1, s.xi2 = _ptr(xi[0]), _ptr(xi[1]), _ptr(xi[2])
    else:
        s.xi0 = s.xi1 = s.xi2 = None
    s.seed = int(q.get("seed") or 0)
    sh = q.get("shift")
    s.shift0, s.shift1 = (_ptr(sh[0]), _ptr(sh[1])) if sh is not None else (None, None)
    return s


def alloc_eval_out(n, device="cuda"):
    import torch
    return (torch.empty((12, n), dtype=torch.float32, device=device),
            torch.empty(n, dtype=torch.int32, device=device))


def bysdf_eval(types: Types, q: dict, out=None, stream=None):
    """Returns (vals float32[12, n], flags int32[n])."""
    n = int(q["h"].numel())
    vals, flags = out if out is not None else alloc_eval_out(n, q["h"].device)
    o = EvalOutSoA()
    names = ("E_r", "E_g", "E_b", "E_xS", "E_yS", "E_xB_r", "E_xB_g", "E_xB_b", "E_yB_r",
             "E_yB_g", "E_yB_b", "pdf")
    for i, nm in enumerate(names):
        setattr(o, nm, _ptr(vals[i]))
    o.flags = _ptr(flags)
    qs = _qsoa(q)
    _check(lib().bysdf_eval(types.handle, C.byref(qs), n, C.byref(o), _stream(stream)),
           "bysdf_eval")
    return vals, flags


def _eval_out_soa(vals, flags):
    o = EvalOutSoA()
    names = ("E_r", "E_g", "E_b", "E_xS", "E_yS", "E_xB_r", "E_xB_g", "E_xB_b", "E_yB_r",
             "E_yB_g", "E_yB_b", "pdf")
    for i, nm in enumerate(names):
        setattr(o, nm, _ptr(vals[i]))
    o.flags = _ptr(flags)
    return o


def bysdf_batched_workspace_size(n_types: int) -> int:
    return int(lib().bysdf_batched_workspace_size(n_types))


def _check_workspace(t, ptr, ws, name):
    """The caller's workspace tensor must hold ws bytes from ptr on."""
    base = t.data_ptr()
    end = base + t.numel() * t.element_size()
    if not (base <= ptr and ptr + ws <= end):
        raise ValueError("%s: workspace holds %d bytes past its pointer, %d needed"
                         % (name, max(0, end - ptr), ws))


def alloc_workspace(nbytes, device="cuda"):
    """Device workspace with a 256-byte aligned pointer: (tensor, ptr)."""
    import torch
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return t, (t.data_ptr() + 255) & ~255


def bysdf_eval_batched(types: Types, offsets, q: dict, out=None, sched=None, workspace=None,
                       stream=None):
    """Heterogeneous batch grouped by type (offsets: int64 cuda CSR).
    sched: dict(chunk, grid, use_lds) or None.  workspace: (tensor, ptr) from
    alloc_workspace or None.  Returns (vals float32[12, n], flags int32[n])."""
    n = int(q["h"].numel())
    vals, flags = out if out is not None else alloc_eval_out(n, q["h"].device)
    o = _eval_out_soa(vals, flags)
    ws = bysdf_batched_workspace_size(types.n_types)
    if workspace is None:
        workspace = alloc_workspace(ws, q["h"].device)
    else:
        _check_workspace(workspace[0], workspace[1], ws, "bysdf_eval_batched")
    sc = None
    if sched is not None:
        sc = Schedule(int(sched["chunk"]), int(sched["grid"]), int(sched["use_lds"]),
                      int(sched.get("block", 0)), int(sched.get("min_waves", 0)))
    qs = _qsoa(q)
    _check(lib().bysdf_eval_batched(types.handle, offsets.data_ptr(), n, C.byref(qs), C.byref(o),
                                    C.byref(sc) if sc is not None else None, workspace[1], ws,
                                    _stream(stream)), "bysdf_eval_batched")
    return vals, flags


def bysdf_eval_batched_noalloc(types: Types, offsets, q: dict, out, sched=None, stream=None):
    """bysdf_eval_batched with its workspace in the library's static device
    memory: the call allocates nothing, so `out` (vals float32[12, n],
    flags int32[n]) must be given.  Returns out."""
    n = int(q["h"].numel())
    vals, flags = out
    o = _eval_out_soa(vals, flags)
    sc = None
    if sched is not None:
        sc = Schedule(int(sched["chunk"]), int(sched["grid"]), int(sched["use_lds"]),
                      int(sched.get("block", 0)), int(sched.get("min_waves", 0)))
    qs = _qsoa(q)
    _check(lib().bysdf_eval_batched_noalloc(types.handle, offsets.data_ptr(), n, C.byref(qs), C.byref(o),
                                            C.byref(sc) if sc is not None else None, _stream(stream)),
           "bysdf_eval_batched_noalloc")
    return vals, flags


def alloc_sample_out(n, device="cuda"):
    import torch
    return (torch.empty((10, n), dtype=torch.float32, device=device),
            torch.empty(n, dtype=torch.int32, device=device),
            torch.empty(n, dtype=torch.int32, device=device),
            torch.empty(n, dtype=torch.int32, device=device))


def bysdf_sample_pdf(types: Types, q: dict, out=None, stream=None):
    """Returns (vals float32[10, n], lobe int32[n], node int32[n], flags int32[n])."""
    n = int(q["h"].numel())
    vals, lobe, node, flags = out if out is not None else alloc_sample_out(n, q["h"].device)
    o = SampleOutSoA()
    names = ("wo_x", "wo_y", "wo_z", "w_r", "w_g", "w_b", "pdf", "exit_x", "exit_y", "exit_z")
    for i, nm in enumerate(names):
        setattr(o, nm, _ptr(vals[i]))
    o.lobe, o.node, o.flags = _ptr(lobe), _ptr(node), _ptr(flags)
    qs = _ssoa(q)
    _check(lib().bysdf_sample_pdf(types.handle, C.byref(qs), n, C.byref(o), _stream(stream)),
           "bysdf_sample_pdf")
    return vals, lobe, node, flags


def bysdf_eval_sample(types: Types, q: dict, out=None, stream=None):
    """Value and pdf at q["wo"] and one direction drawn with q["xi"], per
    query, in one pass.  out: (eval_out, sample_out) as allocated by
    alloc_eval_out / alloc_sample_out.  Returns (eval_vals float32[12, n],
    eval_flags int32[n], sample_vals float32[10, n], lobe, node, sample_flags)."""
    n = int(q["h"].numel())
    eo, so = out if out is not None else (alloc_eval_out(n, q["h"].device),
                                          alloc_sample_out(n, q["h"].device))
    ev, ef = eo
    sv, lobe, node, sf = so
    o = _eval_out_soa(ev, ef)
    s = SampleOutSoA()
    names = ("wo_x", "wo_y", "wo_z", "w_r", "w_g", "w_b", "pdf", "exit_x", "exit_y", "exit_z")
    for i, nm in enumerate(names):
        setattr(s, nm, _ptr(sv[i]))
    s.lobe, s.node, s.flags = _ptr(lobe), _ptr(node), _ptr(sf)
    qs = _qsoa(q)
    xi = q["xi"]
    _check(lib().bysdf_eval_sample(types.handle, C.byref(qs), _ptr(xi[0]), _ptr(xi[1]), _ptr(xi[2]),
                                   n, C.byref(o), C.byref(s), _stream(stream)), "bysdf_eval_sample")
    return ev, ef, sv, lobe, node, sf


def bysdf_ply_geometry(types: Types, q: dict, stream=None):
    """Implicit ply hit per query (Sec. 3.4).  q needs type, h, u, v, wi.
    Returns (ply int32[n], point float32[3, n], tangent float32[3, n],
    normal float32[3, n], flags int32[n])."""
    import torch
    n = int(q["h"].numel())
    dev = q["h"].device
    ply = torch.empty(n, dtype=torch.int32, device=dev)
    vals = torch.empty((9, n), dtype=torch.float32, device=dev)
    flags = torch.empty(n, dtype=torch.int32, device=dev)
    o = PlyOutSoA()
    o.ply, o.flags = _ptr(ply), _ptr(flags)
    for i, nm in enumerate(("p_x", "p_y", "p_z", "t_x", "t_y", "t_z", "n_x", "n_y", "n_z")):
        setattr(o, nm, _ptr(vals[i]))
    s = QuerySoA()
    s.type_id, s.h, s.u, s.v = _ptr(q["type"]), _ptr(q["h"]), _ptr(q["u"]), _ptr(q["v"])
    wi = q["wi"]
    s.wi_x, s.wi_y, s.wi_z = _ptr(wi[0]), _ptr(wi[1]), _ptr(wi[2])
    _check(lib().bysdf_ply_geometry(types.handle, C.byref(s), n, C.byref(o), _stream(stream)),
           "bysdf_ply_geometry")
    return ply, vals[0:3], vals[3:6], vals[6:9], flags


def _fsoa(q, sampler):
    f = FootprintSoA()
    f.h1, f.h2, f.zeta = _ptr(q["h1"]), _ptr(q["h2"]), _ptr(q["zeta"])
    f.xi_s = _ptr(q["xi_s"]) if sampler else None
    return f


def bysdf_eval_multi(types: Types, q: dict, n_max: int = 4, out=None, stream=None):
    """Multi-scale value and pdf at q["wo"] over the footprint (q["h1"],
    q["h"], q["h2"]) with strata offset q["zeta"].  Returns (vals
    float32[12, n], flags int32[n]) as bysdf_eval."""
    n = int(q["h"].numel())
    vals, flags = out if out is not None else alloc_eval_out(n, q["h"].device)
    o = _eval_out_soa(vals, flags)
    qs, fs = _qsoa(q), _fsoa(q, False)
    _check(lib().bysdf_eval_multi(types.handle, C.byref(qs), C.byref(fs), n, n_max, C.byref(o),
                                  _stream(stream)), "bysdf_eval_multi")
    return vals, flags


def bysdf_sample_multi(types: Types, q: dict, n_max: int = 4, out=None, stream=None):
    """Multi-scale sampler (q["xi_s"] draws the stratum).  Returns (vals
    float32[10, n], lobe, node, flags) as bysdf_sample_pdf, with node =
    forward node + 16 x stratum."""
    n = int(q["h"].numel())
    vals, lobe, node, flags = out if out is not None else alloc_sample_out(n, q["h"].device)
    o = SampleOutSoA()
    names = ("wo_x", "wo_y", "wo_z", "w_r", "w_g", "w_b", "pdf", "exit_x", "exit_y", "exit_z")
    for i, nm in enumerate(names):
        setattr(o, nm, _ptr(vals[i]))
    o.lobe, o.node, o.flags = _ptr(lobe), _ptr(node), _ptr(flags)
    qs, fs = _ssoa(q), _fsoa(q, True)
    _check(lib().bysdf_sample_multi(types.handle, C.byref(qs), C.byref(fs), n, n_max, C.byref(o),
                                    _stream(stream)), "bysdf_sample_multi")
    return vals, lobe, node, flags


def bysdf_furnace_blocks(types: Types, q: dict, block: int = 256, mean=None, var=None,
                         stream=None):
    """Returns (mean float32[nb, 3], var float32[nb, 3])."""
    import torch
    n = int(q["h"].numel())
    nb = n // block
    dev = q["h"].device
    mean = mean if mean is not None else torch.empty((nb, 3), dtype=torch.float32, device=dev)
    var = var if var is not None else torch.empty((nb, 3), dtype=torch.float32, device=dev)
    qs = _ssoa(q)
    _check(lib().bysdf_furnace_blocks(types.handle, C.byref(qs), n, block, _ptr(mean), _ptr(var),
                                      _stream(stream)), "bysdf_furnace_blocks")
    return mean, var


def bysdf_backward_workspace_size(n: int, n_types: int) -> int:
    return int(lib().bysdf_backward_workspace_size(n, n_types))


def bysdf_eval_backward(types: Types, q: dict, offsets, grad_E, grad_theta=None,
                        per_query=False, workspace=None, stream=None):
    """Adjoint of bysdf_eval.  offsets: int64 cuda tensor [n_types + 1] (queries
    grouped by type); grad_E: float32 cuda tensor [n, 3].  Returns
    (grad_theta float32[n_types, 8], per_query float32[n, 8] or None)."""
    import torch
    n = int(q["h"].numel())
    dev = q["h"].device
    assert offsets.dtype == torch.int64 and offsets.is_cuda and offsets.numel() == types.n_types + 1
    assert grad_E.is_contiguous() and grad_E.dtype == torch.float32 and grad_E.numel() == 3 * n
    if grad_theta is None:
        grad_theta = torch.empty((types.n_types, 8), dtype=torch.float32, device=dev)
    pq = None
    if per_query is True:
        pq = torch.empty((n, 8), dtype=torch.float32, device=dev)
    elif per_query is not False and per_query is not None:
        pq = per_query
    ws = bysdf_backward_workspace_size(n, types.n_types)
    if workspace is None:
        workspace = torch.empty(ws + 256, dtype=torch.uint8, device=dev)
    aligned = (workspace.data_ptr() + 255) & ~255
    _check_workspace(workspace, aligned, ws, "bysdf_eval_backward")
    qs = _qsoa(q)
    _check(lib().bysdf_eval_backward(types.handle, C.byref(qs), n, offsets.data_ptr(),
                                     grad_E.data_ptr(), grad_theta.data_ptr(), _ptr(pq),
                                     aligned, ws, _stream(stream)), "bysdf_eval_backward")
    return grad_theta, pq


# ---------------------------------------------------------------- yarn scenes

HIT_MISS = 1 << 0
HIT_CAP = 1 << 1
HIT_EXCLUDED = 1 << 2
HIT_BAD_INPUT = 1 << 9


class Scene:
    """Owner of a yarn_scene_t handle."""

    def __init__(self, handle, n_yarns):
        self.handle = handle
        self.n_yarns = n_yarns

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().yarn_scene_destroy(self.handle)
            except TypeError:  # interpreter shutdown: the process releases the memory
                pass
            self.handle = None


def yarn_scene_create(ctrl, yarn_off, yarn_type=None, yarn_phase=None, stream=None) -> Scene:
    """ctrl (n_cp, 4) float32 host rows x y z r; yarn_off (n_yarns + 1)
    int64; yarn_type (n_yarns) int32 and yarn_phase (n_yarns) float32,
    optional.  All host arrays."""
    ctrl = np.ascontiguousarray(ctrl, np.float32)
    off = np.ascontiguousarray(yarn_off, np.int64)
    n_y = len(off) - 1
    ty = None if yarn_type is None else np.ascontiguousarray(yarn_type, np.int32)
    ph = None if yarn_phase is None else np.ascontiguousarray(yarn_phase, np.float32)
    h = _vp()
    rc = lib().yarn_scene_create(ctrl.ctypes.data, off.ctypes.data, n_y,
                                 None if ty is None else ty.ctypes.data,
                                 None if ph is None else ph.ctypes.data, C.byref(h),
                                 _stream(stream))
    _check(rc, "yarn_scene_create")
    return Scene(h.value, n_y)


def yarn_scene_build_threads(n: int) -> None:
    """Host threads later scene builds may use (0: the default)."""
    _check(lib().yarn_scene_build_threads(int(n)), "yarn_scene_build_threads")


def yarn_scene_info(scene: Scene) -> dict:
    info = (C.c_int64 * 6)()
    _check(lib().yarn_scene_info(scene.handle, info), "yarn_scene_info")
    return dict(zip(("n_yarns", "n_cp", "n_spans", "n_nodes", "depth", "bytes"), list(info)))


def alloc_hits(n, device="cuda"):
    import torch
    out = {}
    for k in HIT_FIELDS:
        dt = torch.int32 if k in ("yarn", "seg", "flags") else torch.float32
        out[k] = torch.empty(n, dtype=dt, device=device)
    return out


def yarn_tube_intersect(scene: Scene, o, d, t_max, t_min: float = 0.0, hits=None, stream=None):
    """o, d: float32 device tensors [3, n]; t_max float32 [n].  Returns a
    dict of device tensors keyed by the yarn_hit_soa field names."""
    n = t_max.shape[0]
    assert o.shape == (3, n) and d.shape == (3, n) and o.is_contiguous() and d.is_contiguous()
    if hits is None:
        hits = alloc_hits(n, device=t_max.device)
    r = RaySoA(o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr(), d[0].data_ptr(),
               d[1].data_ptr(), d[2].data_ptr(), t_max.data_ptr())
    hs = HitSoA(*[hits[k].data_ptr() for k in HIT_FIELDS])
    _check(lib().yarn_tube_intersect(scene.handle, C.byref(r), n, float(t_min), C.byref(hs),
                                     _stream(stream)), "yarn_tube_intersect")
    return hits


# ---------------------------------------------------------------- rendering

def render_settings(rs: dict) -> RenderSettings:
    """render_settings from a dict with the field names of the C struct
    (spp_batch defaults to 0: every sample in one pass; multiscale to 0)."""
    st = RenderSettings()
    rs = dict(rs)
    rs.setdefault("spp_batch", 0)
    rs.setdefault("multiscale", 0)
    for k, _ in RenderSettings._fields_:
        v = rs[k]
        if isinstance(v, (tuple, list)):
            getattr(st, k)[:] = [float(x) for x in v]
        else:
            setattr(st, k, v)
    return st


def shade_wavefront_workspace_size(rs: dict) -> int:
    return int(lib().shade_wavefront_workspace_size(C.byref(render_settings(rs))))


def shade_wavefront(scene: Scene, types: Types, rs: dict, fb=None, workspace=None, counts=False,
                    stream=None):
    """Render the crop; returns the device framebuffer float32 [crop_h,
    crop_w, 3] (and the (extension, shadow) ray counts when counts=True,
    which synchronises)."""
    import torch
    st = render_settings(rs)
    nb = int(lib().shade_wavefront_workspace_size(C.byref(st)))
    if nb == 0:
        _check(-2, "shade_wavefront_workspace_size")
    if fb is None:
        fb = torch.empty((rs["crop_h"], rs["crop_w"], 3), dtype=torch.float32, device="cuda")
    if workspace is None:
        workspace = alloc_workspace(nb)
    buf, ptr = workspace
    rc_counts = (C.c_int64 * 2)() if counts else None
    _check(lib().shade_wavefront(scene.handle, types.handle, C.byref(st), fb.data_ptr(), ptr,
                                 buf.numel() - (ptr - buf.data_ptr()), rc_counts, _stream(stream)),
           "shade_wavefront")
    if counts:
        return fb, (int(rc_counts[0]), int(rc_counts[1]))
    return fb


def shade_wavefront_grad_workspace_size(rs: dict) -> int:
    return int(lib().shade_wavefront_grad_workspace_size(C.byref(render_settings(rs))))


def shade_wavefront_grad(scene: Scene, types: Types, rs: dict, grad_type: int = 0, fb=None, grad=None,
                         workspace=None, stream=None):
    """Render the crop and the gradient of the image with respect to (r,
    k^B_c, sigma_t) of type grad_type.  Returns (framebuffer float32
    [crop_h, crop_w, 3], gradient float32 [crop_h, crop_w, 3, 3])."""
    import torch
    st = render_settings(rs)
    nb = shade_wavefront_grad_workspace_size(rs)
    if nb == 0:
        _check(-2, "shade_wavefront_grad_workspace_size")
    if fb is None:
        fb = torch.empty((rs["crop_h"], rs["crop_w"], 3), dtype=torch.float32, device="cuda")
    if grad is None:
        grad = torch.empty((rs["crop_h"], rs["crop_w"], 3, 3), dtype=torch.float32, device="cuda")
    if workspace is None:
        workspace = alloc_workspace(nb)
    buf, ptr = workspace
    _check(lib().shade_wavefront_grad(scene.handle, types.handle, C.byref(st), grad_type, fb.data_ptr(),
                                      grad.data_ptr(), ptr, buf.numel() - (ptr - buf.data_ptr()), None,
                                      _stream(stream)), "shade_wavefront_grad")
    return fb, grad


def bysdf_philox4x32_10(ctr, key):
    """Host call of the renderer's Philox4x32-10 block."""
    c = (C.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (C.c_uint32 * 4)()
    lib().bysdf_philox4x32_10(c, k, o)
    return [int(x) for x in o]
