"""Python binding of the libsbr C-ABI (argument marshalling only).

Every function keeps the name of the C entry point it calls
(``include/sbr.h``).  Arrays may be numpy arrays (host) or torch tensors
(host or on the context's GPU); all arrays of one call must live in the same
memory space, which selects the SBR_IN_DEVICE / SBR_OUT_DEVICE flags.  Every
step of the method runs in the HIP library: when ``libsbr.so`` is missing this
module raises at import time instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbr.so")

SBR_IN_DEVICE = 0x1
SBR_OUT_DEVICE = 0x2
SBR_POL_V = 0
SBR_POL_H = 1
SBR_MAX_BOUNCES = 16
STATUS = {0: "SBR_OK", -1: "SBR_E_INVALID_ARG", -2: "SBR_E_OUT_OF_MEMORY", -3: "SBR_E_DEVICE",
          -4: "SBR_E_CAPACITY", -5: "SBR_E_STATE", -6: "SBR_E_UNSUPPORTED"}


class SbrError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class PathRecord(C.Structure):
    _fields_ = [("tx", C.c_int32), ("rx", C.c_int32), ("order", C.c_int32), ("flags", C.c_int32),
                ("groups", C.c_int32 * SBR_MAX_BOUNCES), ("length_m", C.c_double), ("delay_s", C.c_double),
                ("aod_az", C.c_float), ("aod_el", C.c_float), ("aoa_az", C.c_float), ("aoa_el", C.c_float),
                ("power", C.c_float), ("pad", C.c_int32)]


def _load():
    # One HIP runtime per process: PyTorch-ROCm ships its own libamdhip64 (same
    # soname); loading torch first makes libsbr bind to that runtime, so torch
    # tensors and streams are valid handles for the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2208_10006_amd/build.py (the HIP library is required)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U32, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    sig = {
        "sbr_context_create": [C.c_int, P, P],
        "sbr_synchronize": [P],
        "sbr_scene_build": [P, P, I64, P, P, P, U32, P],
        "sbr_scene_build_batch": [P, I32, P, P, P, P, P, U32, P],
        "sbr_scene_info": [P, P, P, P],
        "sbr_scene_groups": [P, P, P],
        "sbr_trace": [P, P, P, I32, I32, I32, U32, P],
        "sbr_trace_info": [P, P, P],
        "sbr_trace_hits": [P, P, P, U32],
        "sbr_receive": [P, P, P, I32, D, D, U32, P],
        "sbr_paths_info": [P, P, P, P],
        "sbr_paths_count": [P, P],
        "sbr_paths_get": [P, I64, P, P],
        "sbr_paths_events": [P, I64, P, P, P, P],
        "sbr_channel": [P, P, P, I32, P, P, I32, I32, P, P, U32],
        "sbr_path_field": [P, P, P, I32, P, P, I32, I32, P, U32],
        "sbr_stats": [P, P, P, P, U32],
        "sbr_capacity": [P, P, I32, I32, I32, P, I32, I32, P, U32],
        "sbr_port_power": [P, P, I32, I32, I32, P, U32],
        "sbr_capacity_noalloc": [P, P, I32, I32, I32, P, I32, I32, P],
        "sbr_geodesic": [P, I32, I64, I64, P, U32],
        "sbr_geodesic_alpha": [P, I32, P, P, P],
        "sbr_profile_enable": [P, C.c_int],
        "sbr_profile_query": [P, C.c_char_p, P, P],
        "sbr_profile_only": [P, C.c_char_p],
        "sbr_context_count_work": [P, C.c_int],
        "sbr_trace_work": [P, P, P],
        "sbr_context_set_tuning": [P, C.c_char_p, I32],
        "sbr_context_get_tuning": [P, C.c_char_p, P],
        "sbr_trace_batch": [P, I32, P, P, P, P, P, U32, P],
        "sbr_trace_latency": [P, P],
        "sbr_diffract": [P, P, P, I32, P, I32, U32, P],
        "sbr_diff_info": [P, P, P, P, P],
        "sbr_diff_paths": [P, I64, P, P, P],
        "sbr_scene_wedges": [P, P, I64, P, P, P],
        "sbr_diff_channel": [P, P, P, I32, P, P, I32, I32, P, P, U32],
        "sbr_diff_field": [P, P, P, I32, P, P, I32, I32, P, U32],
        "sbr_utd_transition": [P, P, I64, P, U32],
        "sbr_scatter": [P, P, P, I32, P, I32, D, I32, U32, P],
        "sbr_scat_info": [P, P, P, P, P],
        "sbr_scat_paths": [P, I64, P, P, P],
        "sbr_scat_tiles": [P, I64, P, P, P],
        "sbr_scat_channel": [P, P, P, I32, P, P, I32, I32, P, P, U32],
        "sbr_scat_field": [P, P, P, I32, P, P, I32, I32, P, U32],
        "sbr_scatter_lobe_norm": [P, I32, P, I64, P, U32],
        "sbr_stats_all": [P, P, P, P, P, P, U32],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.sbr_release.argtypes = [P]
    L.sbr_release.restype = None
    L.sbr_last_error.restype = C.c_char_p
    L.sbr_version.restype = C.c_char_p
    return L


_lib = _load()


def _call(name, *args):
    st = getattr(_lib, name)(*args)
    if st != 0:
        raise SbrError(name, st, _lib.sbr_last_error().decode(errors="replace"))


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Arr:
    """Pointer to a contiguous array of the given dtype (keeps a reference)."""

    def __init__(self, x, np_dtype, torch_dtype=None):
        self.device = False
        if x is None:
            self.ptr, self.ref = None, None
        elif _is_torch(x):
            import torch
            t = x.contiguous()
            if torch_dtype is not None and t.dtype != torch_dtype:
                t = t.to(torch_dtype)
            self.ref, self.ptr, self.device = t, C.c_void_p(t.data_ptr()), t.is_cuda
        else:
            a = np.ascontiguousarray(x, dtype=np_dtype)
            self.ref, self.ptr = a, a.ctypes.data_as(C.c_void_p)


def _flags(arrs, bit):
    dev = {a.device for a in arrs if a.ref is not None}
    if len(dev) > 1:
        raise ValueError("all arrays of one call must be on the host or all on the GPU")
    return bit if dev == {True} else 0


def _torch_dtypes():
    try:
        import torch
        return torch.float64, torch.float32, torch.int32, torch.complex64
    except ImportError:  # numpy-only use
        return None, None, None, None


F64, F32, I32T, C64 = _torch_dtypes()


class _Handle:
    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and _lib is not None:
            _lib.sbr_release(h)


class Context(_Handle):
    def __init__(self, device: int = 0, stream: Optional[int] = None):
        h = C.c_void_p()
        _call("sbr_context_create", device, C.c_void_p(stream) if stream else None, C.byref(h))
        super().__init__(h)
        self.device = device


def context_for_torch(device: int = 0) -> Context:
    """A context on torch's current stream of `device` (ordering with torch ops)."""
    import torch
    return Context(device, torch.cuda.current_stream(device).cuda_stream)


class Scene(_Handle):
    pass


class Trace(_Handle):
    pass


class Paths(_Handle):
    pass


class Diffraction(_Handle):
    pass


class Scattering(_Handle):
    pass


# ---------------------------------------------------------------- entry points
def sbr_synchronize(ctx: Context):
    _call("sbr_synchronize", ctx.h)


def sbr_scene_build(ctx: Context, tri, eps_r, sigma, rough) -> Scene:
    a = [_Arr(tri, np.float64, F64), _Arr(eps_r, np.float32, F32), _Arr(sigma, np.float32, F32),
         _Arr(rough, np.float32, F32)]
    T = (a[0].ref.numel() if _is_torch(a[0].ref) else a[0].ref.size) // 9
    h = C.c_void_p()
    _call("sbr_scene_build", ctx.h, a[0].ptr, T, a[1].ptr, a[2].ptr, a[3].ptr, _flags(a, SBR_IN_DEVICE), C.byref(h))
    return Scene(h, (ctx,))


def sbr_scene_build_batch(ctx: Context, tris, eps_rs, sigmas, roughs):
    """Scenes built concurrently (worker threads and streams); returns one Scene per input."""
    n = len(tris)
    arrs = [[_Arr(t, np.float64, F64), _Arr(e, np.float32, F32), _Arr(g, np.float32, F32), _Arr(r, np.float32, F32)]
            for t, e, g, r in zip(tris, eps_rs, sigmas, roughs)]
    flags = _flags([a for row in arrs for a in row], SBR_IN_DEVICE)
    T = np.array([(row[0].ref.numel() if _is_torch(row[0].ref) else row[0].ref.size) // 9 for row in arrs], np.int64)
    ptrs = [(C.c_void_p * n)(*[row[k].ptr for row in arrs]) for k in range(4)]
    out = (C.c_void_p * n)()
    _call("sbr_scene_build_batch", ctx.h, n, ptrs[0], T.ctypes.data_as(C.c_void_p), ptrs[1], ptrs[2], ptrs[3], flags,
          out)
    return [Scene(C.c_void_p(out[i]), (ctx,)) for i in range(n)]


def sbr_scene_info(scene: Scene):
    g, p, d = C.c_int32(), C.c_int32(), C.c_int32()
    _call("sbr_scene_info", scene.h, C.byref(g), C.byref(p), C.byref(d))
    return {"groups": g.value, "planes": p.value, "bvh_depth": d.value}


def sbr_scene_groups(scene: Scene, T: int):
    g = np.zeros(T, np.int32)
    p = np.zeros(T, np.int32)
    _call("sbr_scene_groups", scene.h, g.ctypes.data_as(C.c_void_p), p.ctypes.data_as(C.c_void_p))
    return g, p


def sbr_trace(ctx: Context, scene: Scene, tx, geodesic_N: int, max_bounces: int) -> Trace:
    a = _Arr(tx, np.float64, F64)
    n = (a.ref.numel() if _is_torch(a.ref) else a.ref.size) // 3
    h = C.c_void_p()
    _call("sbr_trace", ctx.h, scene.h, a.ptr, n, geodesic_N, max_bounces, _flags([a], SBR_IN_DEVICE), C.byref(h))
    tr = Trace(h, (ctx, scene, a))
    tr.Nt, tr.N, tr.K = n, geodesic_N, max_bounces
    tr.R = 10 * geodesic_N * geodesic_N + 2
    return tr


def sbr_trace_batch(ctx: Context, scenes, txs, geodesic_N, max_bounces):
    """One breadth-first persistent launch per bounce over all problems; returns traces."""
    n = len(scenes)
    arrs = [_Arr(t, np.float64, F64) for t in txs]
    flags = _flags(arrs, SBR_IN_DEVICE)
    sc = (C.c_void_p * n)(*[x.h for x in scenes])
    tx = (C.c_void_p * n)(*[a.ptr for a in arrs])
    nt = np.array([(a.ref.numel() if _is_torch(a.ref) else a.ref.size) // 3 for a in arrs], np.int32)
    nv = np.ascontiguousarray(geodesic_N, np.int32)
    kv = np.ascontiguousarray(max_bounces, np.int32)
    out = (C.c_void_p * n)()
    _call("sbr_trace_batch", ctx.h, n, sc, tx, nt.ctypes.data_as(C.c_void_p), nv.ctypes.data_as(C.c_void_p),
          kv.ctypes.data_as(C.c_void_p), flags, out)
    res = []
    for i in range(n):
        tr = Trace(C.c_void_p(out[i]), (ctx, scenes[i], arrs[i]))
        tr.Nt, tr.N, tr.K = int(nt[i]), int(nv[i]), int(kv[i])
        tr.R = 10 * tr.N * tr.N + 2
        res.append(tr)
    return res


def sbr_trace_latency(tr: Trace) -> float:
    v = C.c_double()
    _call("sbr_trace_latency", tr.h, C.byref(v))
    return v.value


def sbr_trace_info(tr: Trace):
    r, s = C.c_int64(), C.c_int64()
    _call("sbr_trace_info", tr.h, C.byref(r), C.byref(s))
    return {"rays": r.value, "segments": s.value}


def sbr_trace_hits(tr: Trace, out=None, uv=None):
    """Hit triangles [rays, K+1] (global ray ids); with uv (True or an array
    [rays, K+1, 2] float32) also the barycentric (u, v) of every hit, NaN
    where the chain has ended: returns (seq, uv) then."""
    if out is None:
        out = np.zeros((tr.Nt * tr.R, tr.K + 1), np.int32)
    o = _Arr(out, np.int32)
    arrs = [o]
    u = None
    if uv is not None and uv is not False:
        if uv is True:
            uv = np.zeros((tr.Nt * tr.R, tr.K + 1, 2), np.float32)
        u = _Arr(uv, np.float32)
        arrs.append(u)
    _call("sbr_trace_hits", tr.h, o.ptr, u.ptr if u is not None else None, _flags(arrs, SBR_OUT_DEVICE))
    return out if u is None else (out, uv)


def sbr_receive(ctx: Context, tr: Trace, rx, alpha_rad: float = 0.0, radius_coeff: float = 1.0) -> Paths:
    a = _Arr(rx, np.float64, F64)
    n = (a.ref.numel() if _is_torch(a.ref) else a.ref.size) // 3
    h = C.c_void_p()
    _call("sbr_receive", ctx.h, tr.h, a.ptr, n, float(alpha_rad), float(radius_coeff), _flags([a], SBR_IN_DEVICE),
          C.byref(h))
    ps = Paths(h, (ctx, tr))
    ps.Nr, ps.Nt, ps.K = n, tr.Nt, tr.K
    return ps


def sbr_paths_info(ps: Paths):
    e, k, n = C.c_int64(), C.c_int64(), C.c_int64()
    _call("sbr_paths_info", ps.h, C.byref(e), C.byref(k), C.byref(n))
    return {"events": e.value, "keys": k.value, "paths": n.value}


def sbr_paths_count(ps: Paths) -> int:
    n = C.c_int64()
    _call("sbr_paths_count", ps.h, C.byref(n))
    return n.value


def sbr_paths_events(ps: Paths):
    """(ray, rx, k) of every capture event (unordered)."""
    n = sbr_paths_info(ps)["events"]
    ray = np.zeros(n, np.uint32)
    rx = np.zeros(n, np.int32)
    k = np.zeros(n, np.int32)
    w = C.c_int64()
    _call("sbr_paths_events", ps.h, n, ray.ctypes.data_as(C.c_void_p), rx.ctypes.data_as(C.c_void_p),
          k.ctypes.data_as(C.c_void_p), C.byref(w))
    return ray.astype(np.int64), rx, k


def sbr_paths_get(ps: Paths):
    """Structured numpy array of path records (ordered by rx, tx, delay)."""
    n = sbr_paths_count(ps)
    buf = (PathRecord * max(n, 1))()
    w = C.c_int64()
    _call("sbr_paths_get", ps.h, n, buf, C.byref(w))
    dt = np.dtype([("tx", np.int32), ("rx", np.int32), ("order", np.int32), ("flags", np.int32),
                   ("groups", np.int32, (SBR_MAX_BOUNCES,)), ("length_m", np.float64), ("delay_s", np.float64),
                   ("aod_az", np.float32), ("aod_el", np.float32), ("aoa_az", np.float32), ("aoa_el", np.float32),
                   ("power", np.float32), ("pad", np.int32)])
    assert dt.itemsize == C.sizeof(PathRecord)
    return np.frombuffer(bytes(buf), dtype=dt, count=n).copy()


def _field_args(freq, atm_db, atm_deg):
    return [_Arr(freq, np.float64, F64), _Arr(atm_db, np.float32, F32), _Arr(atm_deg, np.float32, F32)]


def sbr_channel(ctx: Context, ps: Paths, freq, atm_db_per_m=None, atm_deg_per_m=None, pol_tx=SBR_POL_V,
                pol_rx=SBR_POL_V, H_c64=None, H_c128=None):
    """Fills H_c64 ([Nf, Nr, Nt] complex64 or float32 [..., 2]) and/or H_c128."""
    fa = _field_args(freq, atm_db_per_m, atm_deg_per_m)
    nf = (fa[0].ref.numel() if _is_torch(fa[0].ref) else fa[0].ref.size)
    outs = [_Arr(H_c64, np.complex64), _Arr(H_c128, np.complex128)]
    inf = _flags(fa, SBR_IN_DEVICE)
    outf = _flags(outs, SBR_OUT_DEVICE)
    _call("sbr_channel", ctx.h, ps.h, fa[0].ptr, nf, fa[1].ptr, fa[2].ptr, pol_tx, pol_rx, outs[0].ptr, outs[1].ptr,
          inf | outf)
    for x, a in zip((H_c64, H_c128), outs):
        if x is not None and not _is_torch(x) and a.ref is not x:
            np.copyto(x, a.ref)


def sbr_path_field(ctx: Context, ps: Paths, freq, atm_db_per_m=None, atm_deg_per_m=None, pol_tx=SBR_POL_V,
                   pol_rx=SBR_POL_V):
    fa = _field_args(freq, atm_db_per_m, atm_deg_per_m)
    nf = (fa[0].ref.numel() if _is_torch(fa[0].ref) else fa[0].ref.size)
    n = sbr_paths_count(ps)
    out = np.zeros((n, nf), np.complex128)
    o = _Arr(out, np.complex128)
    _call("sbr_path_field", ctx.h, ps.h, fa[0].ptr, nf, fa[1].ptr, fa[2].ptr, pol_tx, pol_rx, o.ptr,
          _flags(fa, SBR_IN_DEVICE))
    return out


# ---------------------------------------------------------------- diffraction
def sbr_diffract(ctx: Context, sc: Scene, tx, rx) -> Diffraction:
    """First-order edge-diffraction paths of every (Tx, Rx) pair over the scene's wedges."""
    a = [_Arr(tx, np.float64, F64), _Arr(rx, np.float64, F64)]
    nt = (a[0].ref.numel() if _is_torch(a[0].ref) else a[0].ref.size) // 3
    nr = (a[1].ref.numel() if _is_torch(a[1].ref) else a[1].ref.size) // 3
    h = C.c_void_p()
    _call("sbr_diffract", ctx.h, sc.h, a[0].ptr, nt, a[1].ptr, nr, _flags(a, SBR_IN_DEVICE), C.byref(h))
    d = Diffraction(h, (ctx, sc))
    d.Nt, d.Nr = nt, nr
    return d


def sbr_diff_info(d: Diffraction):
    w, c, g, n = (C.c_int64() for _ in range(4))
    _call("sbr_diff_info", d.h, C.byref(w), C.byref(c), C.byref(g), C.byref(n))
    return {"wedges": w.value, "candidates": c.value, "geometric": g.value, "paths": n.value}


def sbr_diff_paths(d: Diffraction):
    """(ids [n, 3] int32: tx, rx, wedge; rec [n, 8]: Q xyz, s', s, beta0, phi', phi)."""
    n = sbr_diff_info(d)["paths"]
    ids = np.zeros((n, 3), np.int32)
    rec = np.zeros((n, 8), np.float64)
    w = C.c_int64()
    _call("sbr_diff_paths", d.h, n, ids.ctypes.data_as(C.c_void_p), rec.ctypes.data_as(C.c_void_p), C.byref(w))
    return ids, rec


def sbr_scene_wedges(ctx: Context, sc: Scene):
    """(geo [W, 8]: start xyz, end xyz, exterior angle / pi, length; groups [W, 2])."""
    cnt = C.c_int64()
    _call("sbr_scene_wedges", ctx.h, sc.h, 0, None, None, C.byref(cnt))
    geo = np.zeros((cnt.value, 8), np.float64)
    grp = np.zeros((cnt.value, 2), np.int32)
    _call("sbr_scene_wedges", ctx.h, sc.h, cnt.value, geo.ctypes.data_as(C.c_void_p),
          grp.ctypes.data_as(C.c_void_p), C.byref(cnt))
    return geo, grp


def sbr_diff_channel(ctx: Context, d: Diffraction, freq, atm_db_per_m=None, atm_deg_per_m=None, pol_tx=SBR_POL_V,
                     pol_rx=SBR_POL_V, H_c64=None, H_c128=None):
    """Adds the diffracted fields to H_c64 and/or H_c128 ([Nf, Nr, Nt])."""
    fa = _field_args(freq, atm_db_per_m, atm_deg_per_m)
    nf = (fa[0].ref.numel() if _is_torch(fa[0].ref) else fa[0].ref.size)
    outs = [_Arr(H_c64, np.complex64), _Arr(H_c128, np.complex128)]
    _call("sbr_diff_channel", ctx.h, d.h, fa[0].ptr, nf, fa[1].ptr, fa[2].ptr, pol_tx, pol_rx, outs[0].ptr,
          outs[1].ptr, _flags(fa, SBR_IN_DEVICE) | _flags(outs, SBR_OUT_DEVICE))
    for x, a in zip((H_c64, H_c128), outs):
        if x is not None and not _is_torch(x) and a.ref is not x:
            np.copyto(x, a.ref)


def sbr_diff_field(ctx: Context, d: Diffraction, freq, atm_db_per_m=None, atm_deg_per_m=None, pol_tx=SBR_POL_V,
                   pol_rx=SBR_POL_V):
    fa = _field_args(freq, atm_db_per_m, atm_deg_per_m)
    nf = (fa[0].ref.numel() if _is_torch(fa[0].ref) else fa[0].ref.size)
    n = sbr_diff_info(d)["paths"]
    out = np.zeros((n, nf), np.complex128)
    _call("sbr_diff_field", ctx.h, d.h, fa[0].ptr, nf, fa[1].ptr, fa[2].ptr, pol_tx, pol_rx,
          out.ctypes.data_as(C.c_void_p), _flags(fa, SBR_IN_DEVICE))
    return out


def sbr_utd_transition(ctx: Context, X):
    x = np.ascontiguousarray(X, np.float64)
    out = np.zeros(x.size, np.complex128)
    _call("sbr_utd_transition", ctx.h, x.ctypes.data_as(C.c_void_p), x.size, out.ctypes.data_as(C.c_void_p), 0)
    return out.reshape(x.shape)


# ---------------------------------------------------------------- directive scattering
def sbr_scatter(ctx: Context, sc: Scene, tx, rx, tile_area, alpha) -> Scattering:
    """First-order directive scattering paths of every (Tx, Rx) pair over the scene's surface tiles."""
    a = [_Arr(tx, np.float64, F64), _Arr(rx, np.float64, F64)]
    nt = (a[0].ref.numel() if _is_torch(a[0].ref) else a[0].ref.size) // 3
    nr = (a[1].ref.numel() if _is_torch(a[1].ref) else a[1].ref.size) // 3
    h = C.c_void_p()
    _call("sbr_scatter", ctx.h, sc.h, a[0].ptr, nt, a[1].ptr, nr, float(tile_area), int(alpha),
          _flags(a, SBR_IN_DEVICE), C.byref(h))
    d = Scattering(h, (ctx, sc))
    d.Nt, d.Nr = nt, nr
    return d


def sbr_scat_info(d: Scattering):
    t, c, g, n = (C.c_int64() for _ in range(4))
    _call("sbr_scat_info", d.h, C.byref(t), C.byref(c), C.byref(g), C.byref(n))
    return {"tiles": t.value, "candidates": c.value, "clear_legs": g.value, "paths": n.value}


def sbr_scat_paths(d: Scattering):
    """(ids [n, 3] int32: tx, rx, tile; rec [n, 2]: r_i, r_s)."""
    n = sbr_scat_info(d)["paths"]
    ids = np.zeros((n, 3), np.int32)
    rec = np.zeros((n, 2), np.float64)
    w = C.c_int64()
    _call("sbr_scat_paths", d.h, n, ids.ctypes.data_as(C.c_void_p), rec.ctypes.data_as(C.c_void_p), C.byref(w))
    return ids, rec


def sbr_scat_tiles(d: Scattering):
    """(geo [n, 4]: centroid xyz, area; tri [n] int32)."""
    n = sbr_scat_info(d)["tiles"]
    geo = np.zeros((n, 4), np.float64)
    tri = np.zeros(n, np.int32)
    cnt = C.c_int64()
    _call("sbr_scat_tiles", d.h, n, geo.ctypes.data_as(C.c_void_p), tri.ctypes.data_as(C.c_void_p), C.byref(cnt))
    return geo, tri


def sbr_scat_channel(ctx: Context, d: Scattering, freq, atm_db_per_m=None, atm_deg_per_m=None, pol_tx=SBR_POL_V,
                     pol_rx=SBR_POL_V, H_c64=None, H_c128=None):
    """Adds the scattered fields to H_c64 and/or H_c128 ([Nf, Nr, Nt])."""
    fa = _field_args(freq, atm_db_per_m, atm_deg_per_m)
    nf = (fa[0].ref.numel() if _is_torch(fa[0].ref) else fa[0].ref.size)
    outs = [_Arr(H_c64, np.complex64), _Arr(H_c128, np.complex128)]
    _call("sbr_scat_channel", ctx.h, d.h, fa[0].ptr, nf, fa[1].ptr, fa[2].ptr, pol_tx, pol_rx, outs[0].ptr,
          outs[1].ptr, _flags(fa, SBR_IN_DEVICE) | _flags(outs, SBR_OUT_DEVICE))
    for x, a in zip((H_c64, H_c128), outs):
        if x is not None and not _is_torch(x) and a.ref is not x:
            np.copyto(x, a.ref)


def sbr_scat_field(ctx: Context, d: Scattering, freq, atm_db_per_m=None, atm_deg_per_m=None, pol_tx=SBR_POL_V,
                   pol_rx=SBR_POL_V):
    fa = _field_args(freq, atm_db_per_m, atm_deg_per_m)
    nf = (fa[0].ref.numel() if _is_torch(fa[0].ref) else fa[0].ref.size)
    n = sbr_scat_info(d)["paths"]
    out = np.zeros((n, nf), np.complex128)
    _call("sbr_scat_field", ctx.h, d.h, fa[0].ptr, nf, fa[1].ptr, fa[2].ptr, pol_tx, pol_rx,
          out.ctypes.data_as(C.c_void_p), _flags(fa, SBR_IN_DEVICE))
    return out


def sbr_scatter_lobe_norm(ctx: Context, alpha, cos_i):
    x = np.ascontiguousarray(cos_i, np.float64)
    out = np.zeros(x.size, np.float64)
    _call("sbr_scatter_lobe_norm", ctx.h, int(alpha), x.ctypes.data_as(C.c_void_p), x.size,
          out.ctypes.data_as(C.c_void_p), 0)
    return out.reshape(x.shape)


def sbr_stats(ps: Paths):
    nseg = ps.Nr * ps.Nt
    pg = np.zeros((ps.Nr, ps.Nt), np.float32)
    tau = np.zeros((ps.Nr, ps.Nt), np.float32)
    ang = np.zeros((ps.Nr, ps.Nt, 4), np.float32)
    _call("sbr_stats", ps.h, pg.ctypes.data_as(C.c_void_p), tau.ctypes.data_as(C.c_void_p),
          ang.ctypes.data_as(C.c_void_p), 0)
    return pg, tau, ang



def sbr_stats_all(ps: Paths, d: "Diffraction" = None, sc: "Scattering" = None):
    """Per-link path gain, RMS delay spread and mean angles over the
    reflection paths of ps and, when given, the diffraction paths of d and
    the scattering paths of sc."""
    pg = np.zeros((ps.Nr, ps.Nt), np.float32)
    tau = np.zeros((ps.Nr, ps.Nt), np.float32)
    ang = np.zeros((ps.Nr, ps.Nt, 4), np.float32)
    _call("sbr_stats_all", ps.h, d.h if d is not None else None, sc.h if sc is not None else None,
          pg.ctypes.data_as(C.c_void_p), tau.ctypes.data_as(C.c_void_p), ang.ctypes.data_as(C.c_void_p), 0)
    return pg, tau, ang

def sbr_stats_device(ps: Paths, pg, tau, ang):
    """Device outputs (torch tensors on the context device)."""
    arrs = [_Arr(pg, np.float32), _Arr(tau, np.float32), _Arr(ang, np.float32)]
    _call("sbr_stats", ps.h, arrs[0].ptr, arrs[1].ptr, arrs[2].ptr, SBR_OUT_DEVICE)


def sbr_capacity(ctx: Context, H_c64, snr_db, normalize: int = 1):
    h = _Arr(H_c64, np.complex64)
    shape = tuple(h.ref.shape)
    Nf, Nr, Nt = shape[:3]
    s = _Arr(snr_db, np.float64, F64)
    ns = (s.ref.numel() if _is_torch(s.ref) else s.ref.size)
    out = np.zeros(ns, np.float64)
    _call("sbr_capacity", ctx.h, h.ptr, Nf, Nr, Nt, s.ptr, ns, int(normalize), out.ctypes.data_as(C.c_void_p),
          _flags([h, s], SBR_IN_DEVICE))
    return out


def sbr_port_power(ctx: Context, H_c64, out=None):
    """P[q][p] = band mean of |H_f[q][p]|^2 (FP64).  H_c64: complex64 [Nf, Nr, Nt]
    (numpy or a contiguous device tensor).  out: None (returns numpy [Nr, Nt]) or a
    float64 device tensor of Nr*Nt values (queued on the context stream)."""
    h = _Arr(H_c64, np.complex64)
    Nf, Nr, Nt = tuple(h.ref.shape)[:3]
    if out is None:
        res = np.zeros((Nr, Nt), np.float64)
        _call("sbr_port_power", ctx.h, h.ptr, Nf, Nr, Nt, res.ctypes.data_as(C.c_void_p), _flags([h], SBR_IN_DEVICE))
        return res
    if not (_is_torch(out) and out.is_cuda and out.dtype == F64 and out.is_contiguous() and out.numel() >= Nr * Nt):
        raise ValueError("out must be a contiguous float64 device tensor of Nr*Nt values")
    _call("sbr_port_power", ctx.h, h.ptr, Nf, Nr, Nt, C.c_void_p(out.data_ptr()),
          _flags([h], SBR_IN_DEVICE) | SBR_OUT_DEVICE)
    return out


def sbr_capacity_noalloc(ctx: Context, H_c64, snr_db, out, normalize: int = 1):
    """Allocation-free capacity: H_c64 (complex64 [Nf, Nr, Nt]) and out (float64
    [Nsnr]) are tensors on the context's device, snr_db a host sequence.
    Queued on the context stream; synchronise before reading out."""
    if not (_is_torch(H_c64) and H_c64.is_cuda and _is_torch(out) and out.is_cuda):
        raise ValueError("sbr_capacity_noalloc takes device tensors for H and the output")
    if H_c64.dtype != C64 or not H_c64.is_contiguous() or out.dtype != F64 or not out.is_contiguous():
        raise ValueError("H must be contiguous complex64 and out contiguous float64")
    Nf, Nr, Nt = tuple(H_c64.shape)[:3]
    snr = np.ascontiguousarray(snr_db, np.float64)
    if out.numel() < snr.size:
        raise ValueError("out holds fewer values than snr_db")
    _call("sbr_capacity_noalloc", ctx.h, C.c_void_p(H_c64.data_ptr()), Nf, Nr, Nt,
          snr.ctypes.data_as(C.c_void_p), snr.size, int(normalize), C.c_void_p(out.data_ptr()))


def sbr_geodesic(ctx: Context, N: int, first: int = 0, count: Optional[int] = None):
    R = 10 * N * N + 2
    count = R - first if count is None else count
    out = np.zeros((count, 3), np.float64)
    _call("sbr_geodesic", ctx.h, N, first, count, out.ctypes.data_as(C.c_void_p), 0)
    return out


def sbr_geodesic_alpha(ctx: Context, N: int):
    m, lo, hi = C.c_double(), C.c_double(), C.c_double()
    _call("sbr_geodesic_alpha", ctx.h, N, C.byref(m), C.byref(lo), C.byref(hi))
    return m.value, lo.value, hi.value


def sbr_profile_enable(ctx: Context, enable: bool = True):
    _call("sbr_profile_enable", ctx.h, int(enable))


def sbr_profile_only(ctx: Context, kernel: Optional[str]):
    _call("sbr_profile_only", ctx.h, kernel.encode() if kernel else None)


def sbr_profile_query(ctx: Context, kernel: str):
    """(total_ms, launches) of one kernel class since profiling was enabled."""
    ms, n = C.c_double(), C.c_int64()
    _call("sbr_profile_query", ctx.h, kernel.encode(), C.byref(ms), C.byref(n))
    return ms.value, n.value


def sbr_context_count_work(ctx: Context, enable: bool = True):
    _call("sbr_context_count_work", ctx.h, int(enable))


def sbr_trace_work(tr: Trace):
    nv, nt = C.c_int64(), C.c_int64()
    _call("sbr_trace_work", tr.h, C.byref(nv), C.byref(nt))
    return {"node_visits": nv.value, "tri_tests": nt.value}


def sbr_context_set_tuning(ctx: Context, key: str, value: int):
    _call("sbr_context_set_tuning", ctx.h, key.encode(), int(value))


def sbr_context_get_tuning(ctx: Context, key: str) -> int:
    v = C.c_int32()
    _call("sbr_context_get_tuning", ctx.h, key.encode(), C.byref(v))
    return v.value


def sbr_version() -> str:
    return _lib.sbr_version().decode()


# ---------------------------------------------------------------- convenience
@dataclass
class Result:
    scene: Scene
    trace: Trace
    paths: Paths
    H: np.ndarray          # [Nf, Nr, Nt] complex128
    records: np.ndarray


def run_workload(ctx: Context, w, alpha: float = 0.0, coeff: Optional[float] = None, pol_tx=SBR_POL_V,
                 pol_rx=SBR_POL_V) -> Result:
    """Scene build -> trace -> receive -> channel on host arrays (tests / examples)."""
    sc = sbr_scene_build(ctx, w.tri, w.eps_r, w.sigma, w.rough)
    tr = sbr_trace(ctx, sc, w.tx, w.geodesic_N, w.max_bounces)
    ps = sbr_receive(ctx, tr, w.rx, alpha if alpha else w.alpha, w.radius_coeff if coeff is None else coeff)
    H = np.zeros((len(w.freq), len(w.rx), len(w.tx)), np.complex128)
    sbr_channel(ctx, ps, w.freq, w.atm_db_per_m, w.atm_deg_per_m, pol_tx, pol_rx, H_c128=H)
    return Result(sc, tr, ps, H, sbr_paths_get(ps))
