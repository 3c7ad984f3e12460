"""MI355X (gfx950) MFA evaluator and ray caster: Python binding.

Thin wrappers over the C ABI of include/mfa.h.  Device buffers are torch
tensors on the GPU; work goes on torch's current stream.  Every step of the
computation runs in the library's HIP kernels; this module only marshals
arguments.  There is no CPU fallback: without the built library every call
raises.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import MFAError  # noqa: F401

__all__ = ["Model", "Server", "decode_points", "decode_grid", "render_frame", "MFAError",
           "quantize", "default_knots", "version"]

_DTYPES = {"f32": L.MFA_F32, "bf16": L.MFA_BF16, "f16": L.MFA_F16}


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> C.c_void_p:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


class Model:
    """A resident model (mfa_model_create).

    spec: an object with attributes grid (3 ints), lo, hi (3 floats), edges
    (3 arrays of grid[a]+1 floats), voxel, and blocks, each with degree (3
    ints), knots (3 float64 arrays) and ctrl (float64 or float32 array of
    shape n0 x n1 x n2).
    """

    def __init__(self, spec, storage: str = "f32"):
        if storage not in _DTYPES:
            raise ValueError(f"storage must be one of {sorted(_DTYPES)}")
        lib = L.lib()
        self.storage = storage
        self._keep = []
        dom = L.DomainDesc()
        for a in range(3):
            dom.grid[a] = int(spec.grid[a])
            dom.lo[a] = float(spec.lo[a])
            dom.hi[a] = float(spec.hi[a])
            e = np.ascontiguousarray(spec.edges[a], dtype=np.float64)
            self._keep.append(e)
            dom.edges[a] = e.ctypes.data_as(C.POINTER(C.c_double))
        dom.voxel = float(spec.voxel)
        nb = len(spec.blocks)
        descs = (L.BlockDesc * nb)()
        for b, blk in enumerate(spec.blocks):
            ctrl = np.asarray(blk.ctrl)
            if ctrl.dtype == np.float32:
                ctrl = np.ascontiguousarray(ctrl)
                cdt = L.MFA_F32
            else:
                ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
                cdt = L.MFA_F64
            self._keep.append(ctrl)
            d = descs[b]
            for a in range(3):
                d.degree[a] = int(blk.degree[a])
                d.n_ctrl[a] = int(ctrl.shape[a])
                if blk.knots is not None and blk.knots[a] is not None:
                    k = np.ascontiguousarray(blk.knots[a], dtype=np.float64)
                    self._keep.append(k)
                    d.knots[a] = k.ctypes.data_as(C.POINTER(C.c_double))
            d.ctrl = ctrl.ctypes.data
            d.ctrl_dtype = cdt
        h = C.c_void_p()
        L.check(lib.mfa_model_create(C.byref(dom), descs, nb, _DTYPES[storage], C.byref(h)))
        self._h = h
        self._keep = []
        self.grid = [int(g) for g in spec.grid]
        self.shapes = [tuple(int(s) for s in np.asarray(blk.ctrl).shape) for blk in spec.blocks]

    @property
    def handle(self) -> C.c_void_p:
        if self._h is None:
            raise RuntimeError("model destroyed")
        return self._h

    def info(self) -> dict:
        inf = L.ModelInfo()
        L.check(L.lib().mfa_model_info(self.handle, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in L.ModelInfo._fields_}

    def export_ctrl(self, block: int = 0) -> np.ndarray:
        """Stored bits of one block: uint32 (FP32) or uint16 (BF16/FP16)."""
        shape = self.shapes[block]
        dt = np.uint32 if self.storage == "f32" else np.uint16
        out = np.zeros(shape, dtype=dt)
        L.check(L.lib().mfa_model_export_ctrl(self.handle, block, out.ctypes.data, out.nbytes))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().mfa_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def decode_points(model: Model, xyz, out=None, dbg: bool = False, sorted_order: bool = False,
                  value_only: bool = False, stream=None, noalloc: bool = False):
    """Value and world gradient at points xyz (CUDA float32, shape (3, n)).

    Returns out (n, 4) float32 = (f, df/dx, df/dy, df/dz), or with
    value_only (n,) float32 = f, and, if dbg, an int32 (n, 4) tensor of
    (span0, span1, span2, block).  noalloc: the sorted decode through
    mfa_decode_points_noalloc (library-held static scratch, no allocation).
    """
    torch = _torch()
    if xyz.dim() != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must have shape (3, n)")
    n = int(xyz.shape[1])
    px = _dev_ptr(xyz, torch.float32, name="xyz")
    shape = (n,) if value_only else (n, 4)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=xyz.device)
    po = _dev_ptr(out, torch.float32, shape, "out")
    d = None
    pd = C.c_void_p()
    if dbg:
        d = torch.empty((n, 4), dtype=torch.int32, device=xyz.device)
        pd = C.c_void_p(d.data_ptr())
    flags = (L.MFA_DECODE_SORTED if sorted_order else 0) | (L.MFA_DECODE_VALUE if value_only else 0)
    fn = L.lib().mfa_decode_points_noalloc if noalloc else L.lib().mfa_decode_points
    L.check(fn(model.handle, px, n, flags, po, pd, _stream_ptr(stream)))
    return (out, d) if dbg else out


def decode_grid(model: Model, axis_u: Sequence, out=None, spans: bool = False,
                value_only: bool = False, stream=None):
    """Value and world gradient on the tensor grid of three CUDA float64
    parameter tables.  Returns out (r0, r1, r2, 4), or with value_only
    (r0, r1, r2) = f, and, if spans, an int32 tensor of the r0 + r1 + r2
    per-entry spans."""
    torch = _torch()
    if len(axis_u) != 3:
        raise ValueError("need three axis tables")
    res = (C.c_int32 * 3)(*[int(t.numel()) for t in axis_u])
    ptrs = (C.c_void_p * 3)(*[_dev_ptr(t, torch.float64, name=f"axis_u[{a}]").value
                              for a, t in enumerate(axis_u)])
    shape = (res[0], res[1], res[2]) if value_only else (res[0], res[1], res[2], 4)
    dev = axis_u[0].device
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    po = _dev_ptr(out, torch.float32, shape, "out")
    sp = None
    ps = C.c_void_p()
    if spans:
        sp = torch.empty((res[0] + res[1] + res[2],), dtype=torch.int32, device=dev)
        ps = C.c_void_p(sp.data_ptr())
    flags = L.MFA_DECODE_VALUE if value_only else 0
    L.check(L.lib().mfa_decode_grid(model.handle, ptrs, res, flags, po, ps, _stream_ptr(stream)))
    return (out, sp) if spans else out


def render_partial(model: Model, cam: dict, params: dict, w: int, h: int, block_lo, block_hi,
                   tf_dev=None, out=None, key=None, nsamp: bool = False, stream=None, device=None):
    """Partial image of the samples owned by blocks in [block_lo, block_hi)
    per axis (object-space split).  Returns rgba (h, w, 4) float32 and the
    depth keys (h, w) float64, plus int32 (h, w, 2) sample counts if nsamp."""
    torch = _torch()
    dev = device or torch.device("cuda", torch.cuda.current_device())
    if tf_dev is None:
        tf_dev = torch.as_tensor(np.ascontiguousarray(params["tf"], dtype=np.float32), device=dev)
    cobj = make_camera(cam)
    pobj = make_params(params, tf_dev)
    if out is None:
        out = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
    if key is None:
        key = torch.empty((h, w), dtype=torch.float64, device=dev)
    po = _dev_ptr(out, torch.float32, (h, w, 4), "out")
    pk = _dev_ptr(key, torch.float64, (h, w), "key")
    dbg = None
    ns = None
    if nsamp:
        dbg = L.RenderDebug()
        ns = torch.zeros((h, w, 2), dtype=torch.int32, device=dev)
        dbg.nsamp = ns.data_ptr()
    L.check(L.lib().mfa_render_partial(model.handle, C.byref(cobj), C.byref(pobj),
                                       (C.c_int32 * 3)(*[int(v) for v in block_lo]),
                                       (C.c_int32 * 3)(*[int(v) for v in block_hi]), int(w), int(h),
                                       po, pk, C.byref(dbg) if dbg is not None else None,
                                       _stream_ptr(stream)))
    return (out, key, ns) if nsamp else (out, key)


def render_iso(model: Model, cam: dict, params: dict, w: int, h: int, iso: float, rgb,
               out=None, depth=None, debug: bool = False, stream=None, device=None):
    """First-hit isosurface of level iso (surface colour rgb).  Returns rgba
    (h, w, 4) float32 and the hit depths (h, w) float64 (+inf: no hit), plus
    int32 (h, w, 2) (K, hit sample or -1) and int32 (h, w) evaluated-value
    counts if debug."""
    torch = _torch()
    dev = device or torch.device("cuda", torch.cuda.current_device())
    cobj = make_camera(cam)
    pobj = make_params(params, None)
    if out is None:
        out = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
    if depth is None:
        depth = torch.empty((h, w), dtype=torch.float64, device=dev)
    po = _dev_ptr(out, torch.float32, (h, w, 4), "out")
    pd = _dev_ptr(depth, torch.float64, (h, w), "depth")
    dbg = None
    if debug:
        dbg = L.RenderDebug()
        ns = torch.zeros((h, w, 2), dtype=torch.int32, device=dev)
        ne = torch.zeros((h, w), dtype=torch.int32, device=dev)
        dbg.nsamp = ns.data_ptr()
        dbg.neval = ne.data_ptr()
    L.check(L.lib().mfa_render_iso(model.handle, C.byref(cobj), C.byref(pobj), float(iso),
                                   (C.c_float * 3)(*[float(v) for v in rgb]), int(w), int(h), po, pd,
                                   C.byref(dbg) if dbg is not None else None, _stream_ptr(stream)))
    return (out, depth, ns, ne) if debug else (out, depth)


def composite_over(images: Sequence, keys: Sequence, out=None, stream=None):
    """Depth-ordered "over" of partial images (CUDA float32 (h, w, 4) each)
    by their keys (CUDA float64 (h, w) each)."""
    torch = _torch()
    g = len(images)
    if g != len(keys) or g == 0:
        raise ValueError("need as many keys as images")
    h, w = int(images[0].shape[0]), int(images[0].shape[1])
    pi = (C.c_void_p * g)(*[_dev_ptr(t, torch.float32, (h, w, 4), f"images[{i}]").value
                            for i, t in enumerate(images)])
    pk = (C.c_void_p * g)(*[_dev_ptr(t, torch.float64, (h, w), f"keys[{i}]").value
                            for i, t in enumerate(keys)])
    if out is None:
        out = torch.empty((h, w, 4), dtype=torch.float32, device=images[0].device)
    po = _dev_ptr(out, torch.float32, (h, w, 4), "out")
    L.check(L.lib().mfa_composite_over(g, pi, pk, w, h, po, _stream_ptr(stream)))
    return out


def encode_workspace_bytes(res: Sequence[int], n_ctrl: Sequence[int]) -> int:
    """Device scratch bytes that encode_grid needs for these sizes."""
    out = C.c_int64()
    L.check(L.lib().mfa_encode_workspace((C.c_int32 * 3)(*[int(v) for v in res]),
                                         (C.c_int32 * 3)(*[int(v) for v in n_ctrl]), C.byref(out)))
    return int(out.value)


def encode_grid(values, axis_u: Sequence, degree: Sequence[int], n_ctrl: Sequence[int],
                knots: Optional[Sequence] = None, out=None, work=None, stream=None):
    """Fixed-knot least-squares control points (FP64 CUDA tensor (n0, n1,
    n2)) of the CUDA float32 samples values (r0, r1, r2) at the tensor grid
    of host float64 parameter tables axis_u; knots[a] None = clamped
    uniform.  work: optional CUDA uint8 scratch of encode_workspace_bytes."""
    torch = _torch()
    if len(axis_u) != 3 or len(degree) != 3 or len(n_ctrl) != 3:
        raise ValueError("need three axes")
    res = [int(v) for v in values.shape] if values.dim() == 3 else None
    if res is None:
        raise ValueError("values must be (r0, r1, r2)")
    tabs = [np.ascontiguousarray(np.asarray(u, dtype=np.float64)) for u in axis_u]
    for a in range(3):
        if tabs[a].shape != (res[a],):
            raise ValueError(f"axis_u[{a}] must hold {res[a]} parameters")
    pv = _dev_ptr(values, torch.float32, tuple(res), "values")
    nb = encode_workspace_bytes(res, n_ctrl)
    if work is None:
        work = torch.empty((nb,), dtype=torch.uint8, device=values.device)
    pw = _dev_ptr(work, torch.uint8, name="work")
    shape = tuple(int(v) for v in n_ctrl)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=values.device)
    po = _dev_ptr(out, torch.float64, shape, "out")
    kn = None
    if knots is not None:
        kts = [None if k is None else np.ascontiguousarray(np.asarray(k, dtype=np.float64))
               for k in knots]
        kn = (C.c_void_p * 3)(*[None if k is None else k.ctypes.data for k in kts])
    L.check(L.lib().mfa_encode_grid((C.c_int32 * 3)(*res),
                                    (C.c_void_p * 3)(*[t.ctypes.data for t in tabs]), pv,
                                    (C.c_int32 * 3)(*[int(v) for v in degree]),
                                    (C.c_int32 * 3)(*[int(v) for v in n_ctrl]), kn, po, pw,
                                    int(work.numel()), _stream_ptr(stream)))
    return out


def encode_adaptive_workspace_bytes(res: Sequence[int], max_ctrl: Sequence[int]) -> int:
    """Device scratch bytes that encode_adaptive needs for these sizes."""
    out = C.c_int64()
    L.check(L.lib().mfa_encode_adaptive_workspace((C.c_int32 * 3)(*[int(v) for v in res]),
                                                  (C.c_int32 * 3)(*[int(v) for v in max_ctrl]),
                                                  C.byref(out)))
    return int(out.value)


def encode_adaptive(values, axis_u: Sequence, degree: Sequence[int], n_init: Sequence[int],
                    e_max: float, max_ctrl: Optional[Sequence[int]] = None, max_fits: int = 10,
                    work=None, stream=None):
    """Encoding with knot insertion (mfa_encode_adaptive) of the CUDA float32
    samples values (r0, r1, r2) at the host float64 parameter tables axis_u.
    Returns (knots: three float64 arrays, ctrl: FP64 CUDA tensor (n0, n1,
    n2), history: list of ((n0, n1, n2), largest relative error) per fit).
    max_ctrl defaults to res."""
    torch = _torch()
    if values.dim() != 3 or len(axis_u) != 3 or len(degree) != 3 or len(n_init) != 3:
        raise ValueError("values must be (r0, r1, r2), with three axes of parameters")
    res = [int(v) for v in values.shape]
    mc = [int(v) for v in (max_ctrl if max_ctrl is not None else res)]
    tabs = [np.ascontiguousarray(np.asarray(u, dtype=np.float64)) for u in axis_u]
    for a in range(3):
        if tabs[a].shape != (res[a],):
            raise ValueError(f"axis_u[{a}] must hold {res[a]} parameters")
    pv = _dev_ptr(values, torch.float32, tuple(res), "values")
    nb = encode_adaptive_workspace_bytes(res, mc)
    if work is None:
        work = torch.empty((nb,), dtype=torch.uint8, device=values.device)
    pw = _dev_ptr(work, torch.uint8, name="work")
    cap = mc[0] * mc[1] * mc[2]
    ctrl = torch.empty((cap,), dtype=torch.float64, device=values.device)
    kout = [np.zeros(mc[a] + int(degree[a]) + 1) for a in range(3)]
    hist = np.zeros((max(int(max_fits), 1), 4))
    n_out = (C.c_int32 * 3)()
    n_fits = C.c_int32()
    L.check(L.lib().mfa_encode_adaptive(
        (C.c_int32 * 3)(*res), (C.c_void_p * 3)(*[t.ctypes.data for t in tabs]), pv,
        (C.c_int32 * 3)(*[int(v) for v in degree]), (C.c_int32 * 3)(*[int(v) for v in n_init]),
        (C.c_int32 * 3)(*mc), float(e_max), int(max_fits),
        (C.c_void_p * 3)(*[k.ctypes.data for k in kout]), n_out,
        C.c_void_p(ctrl.data_ptr()), cap, hist.ctypes.data, C.byref(n_fits), pw,
        int(work.numel()), _stream_ptr(stream)))
    n = [int(n_out[a]) for a in range(3)]
    knots = [kout[a][:n[a] + int(degree[a]) + 1].copy() for a in range(3)]
    history = [((int(h[0]), int(h[1]), int(h[2])), float(h[3])) for h in hist[:n_fits.value]]
    return knots, ctrl[:n[0] * n[1] * n[2]].view(*n), history


class EncodePlan:
    """mfa_encode_plan for one grid shape (res samples -> n_ctrl control
    points, degrees, knots, parameter tables), holding its CUDA workspace;
    apply() encodes one block's CUDA float32 samples (res) into FP64 control
    points (n_ctrl) on the stream, asynchronously."""

    def __init__(self, res, axis_u, degree, n_ctrl, knots=None, device=None, stream=None):
        torch = _torch()
        self.res = tuple(int(v) for v in res)
        self.n_ctrl = tuple(int(v) for v in n_ctrl)
        tabs = [np.ascontiguousarray(np.asarray(u, dtype=np.float64)) for u in axis_u]
        for a in range(3):
            if tabs[a].shape != (self.res[a],):
                raise ValueError(f"axis_u[{a}] must hold {self.res[a]} parameters")
        nb = encode_workspace_bytes(self.res, self.n_ctrl)
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.work = torch.empty((nb,), dtype=torch.uint8, device=dev)
        kn = None
        if knots is not None:
            kts = [None if k is None else np.ascontiguousarray(np.asarray(k, dtype=np.float64))
                   for k in knots]
            kn = (C.c_void_p * 3)(*[None if k is None else k.ctypes.data for k in kts])
        L.check(L.lib().mfa_encode_plan((C.c_int32 * 3)(*self.res),
                                        (C.c_void_p * 3)(*[t.ctypes.data for t in tabs]),
                                        (C.c_int32 * 3)(*[int(v) for v in degree]),
                                        (C.c_int32 * 3)(*self.n_ctrl), kn,
                                        C.c_void_p(self.work.data_ptr()), int(self.work.numel()),
                                        _stream_ptr(stream)))

    def apply(self, values, out=None, stream=None):
        torch = _torch()
        pv = _dev_ptr(values, torch.float32, self.res, "values")
        if out is None:
            out = torch.empty(self.n_ctrl, dtype=torch.float64, device=values.device)
        po = _dev_ptr(out, torch.float64, self.n_ctrl, "out")
        L.check(L.lib().mfa_encode_apply((C.c_int32 * 3)(*self.res), (C.c_int32 * 3)(*self.n_ctrl),
                                         pv, po, C.c_void_p(self.work.data_ptr()),
                                         int(self.work.numel()), _stream_ptr(stream)))
        return out


def make_camera(cam: dict) -> L.Camera:
    c = L.Camera()
    c.kind = int(cam["kind"])
    for a in range(3):
        c.eye[a] = float(cam["eye"][a])
        c.forward[a] = float(cam["forward"][a])
        c.right[a] = float(cam["right"][a])
        c.up[a] = float(cam["up"][a])
    c.sx = float(cam["sx"])
    c.sy = float(cam["sy"])
    return c


def make_params(params: dict, tf_dev) -> L.RenderParams:
    """tf_dev None: no transfer function (isosurface renders)."""
    torch = _torch()
    p = L.RenderParams()
    p.tf_rgba = None if tf_dev is None else _dev_ptr(tf_dev, torch.float32, (256, 4), "tf").value
    p.vmin = float(params.get("vmin", 0.0))
    p.vmax = float(params.get("vmax", 1.0))
    p.step = float(params["step"])
    p.max_samples = int(params["max_samples"])
    p.ert_alpha = float(params.get("ert_alpha", 2.0))
    p.ka, p.kd, p.ks = float(params["ka"]), float(params["kd"]), float(params["ks"])
    p.g0 = float(params["g0"])
    p.shininess = int(params["shininess"])
    return p


def render_frame(model: Model, cam: dict, params: dict, w: int, h: int, tf_dev=None, out=None,
                 nsamp: bool = False, alpha: bool = False, neval: bool = False, stream=None,
                 device=None):
    """Ray-casts a w x h image.  params as produced by synth.render_params
    (tf may be given as a CUDA (256,4) float32 tensor in tf_dev).  Returns
    rgba (h, w, 4) float32 and optional int32 (h, w, 2) sample counts and
    float32 (h, w, max_samples) per-sample opacities and int32 (h, w)
    evaluated-sample counts, in that order, for the ones asked for."""
    torch = _torch()
    dev = device or torch.device("cuda", torch.cuda.current_device())
    if tf_dev is None:
        tf_dev = torch.as_tensor(np.ascontiguousarray(params["tf"], dtype=np.float32), device=dev)
    cobj = make_camera(cam)
    pobj = make_params(params, tf_dev)
    if out is None:
        out = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
    po = _dev_ptr(out, torch.float32, (h, w, 4), "out")
    dbg = None
    extra = []
    if nsamp or alpha or neval:
        dbg = L.RenderDebug()
        if nsamp:
            ns = torch.zeros((h, w, 2), dtype=torch.int32, device=dev)
            dbg.nsamp = ns.data_ptr()
            extra.append(ns)
        if alpha:
            ms = int(params["max_samples"])
            al = torch.zeros((h, w, ms), dtype=torch.float32, device=dev)
            dbg.alpha = al.data_ptr()
            dbg.alpha_stride = ms
            extra.append(al)
        if neval:
            ne = torch.zeros((h, w), dtype=torch.int32, device=dev)
            dbg.neval = ne.data_ptr()
            extra.append(ne)
    L.check(L.lib().mfa_render_frame(model.handle, C.byref(cobj), C.byref(pobj), int(w), int(h), po,
                                     C.byref(dbg) if dbg is not None else None,
                                     _stream_ptr(stream)))
    return (out, *extra) if extra else out


FILTERS = {"trilinear": L.FILTER_TRILINEAR, "catmull_rom": L.FILTER_CATMULL_ROM,
           "cubic_bspline": L.FILTER_CUBIC_BSPLINE, "marschner_lobb": L.FIELD_MARSCHNER_LOBB}


def render_volume(samples, kind: str, lo, hi, cam: dict, params: dict, w: int, h: int, dims=None,
                  tf_dev=None, out=None, nsamp: bool = False, alpha: bool = False, stream=None,
                  device=None):
    """Ray-casts a volume of samples (CUDA float32 (N0, N1, N2) on the grid
    lo + i (hi - lo) / (N - 1)) through the local filter kind ("trilinear",
    "catmull_rom", "cubic_bspline"), or the analytic Marschner-Lobb field
    ("marschner_lobb", samples None, dims giving the default step).  Returns
    rgba (h, w, 4) and optional int32 (h, w, 2) sample counts and float32
    (h, w, max_samples) opacities, as render_frame."""
    torch = _torch()
    dev = device or torch.device("cuda", torch.cuda.current_device())
    d = L.VolumeDesc()
    d.kind = FILTERS[kind]
    if samples is not None:
        dims = tuple(int(v) for v in samples.shape)
        d.samples = _dev_ptr(samples, torch.float32, dims, "samples").value
    else:
        d.samples = None
    for a in range(3):
        d.dims[a] = int(dims[a])
        d.lo[a] = float(lo[a])
        d.hi[a] = float(hi[a])
    if tf_dev is None:
        tf_dev = torch.as_tensor(np.ascontiguousarray(params["tf"], dtype=np.float32), device=dev)
    cobj = make_camera(cam)
    pobj = make_params(params, tf_dev)
    if out is None:
        out = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
    po = _dev_ptr(out, torch.float32, (h, w, 4), "out")
    dbg = None
    extra = []
    if nsamp or alpha:
        dbg = L.RenderDebug()
        if nsamp:
            ns = torch.zeros((h, w, 2), dtype=torch.int32, device=dev)
            dbg.nsamp = ns.data_ptr()
            extra.append(ns)
        if alpha:
            ms = int(params["max_samples"])
            al = torch.zeros((h, w, ms), dtype=torch.float32, device=dev)
            dbg.alpha = al.data_ptr()
            dbg.alpha_stride = ms
            extra.append(al)
    L.check(L.lib().mfa_render_volume(C.byref(d), C.byref(cobj), C.byref(pobj), int(w), int(h), po,
                                      C.byref(dbg) if dbg is not None else None,
                                      _stream_ptr(stream)))
    return (out, *extra) if extra else out


class Server:
    """Request loop over resident models (mfa_server_*).

    fake_item_us switches to the host-only fake executor (no device work;
    each batch takes fake_item_us per work item); with it, fake_fail_batch
    = k makes the k-th batch fail as a device error would."""

    def __init__(self, hbm_budget_bytes: int, queue_cap: int = 1024, max_batch_items: int = 0,
                 fake_item_us: Optional[float] = None, fake_fail_batch: int = 0):
        cfg = L.ServerConfig()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.queue_cap = int(queue_cap)
        cfg.max_batch_items = int(max_batch_items)
        cfg.flags = L.MFA_SERVER_FAKE_EXECUTOR if fake_item_us is not None else 0
        cfg.fake_item_us = float(fake_item_us or 0.0)
        cfg.fake_fail_batch = int(fake_fail_batch)
        h = C.c_void_p()
        L.check(L.lib().mfa_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}          # ticket -> objects kept alive until done

    def add_model(self, model: Optional[Model]) -> int:
        mid = C.c_int32()
        L.check(L.lib().mfa_server_add_model(self._h, model.handle if model is not None else None,
                                             C.byref(mid)))
        return mid.value

    def _submit(self, req, keep) -> int:
        t = C.c_uint64()
        L.check(L.lib().mfa_server_submit(self._h, C.byref(req), C.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def submit_render(self, model_id: int, cam: dict, params: dict, w: int, h: int, rgba,
                      tf_dev=None) -> int:
        torch = _torch()
        req = L.Request()
        req.kind = L.MFA_REQ_RENDER
        req.model_id = model_id
        keep = [rgba]
        if tf_dev is not None or isinstance(rgba, torch.Tensor):
            if tf_dev is None:
                tf_dev = torch.as_tensor(np.ascontiguousarray(params["tf"], dtype=np.float32),
                                         device=rgba.device)
            req.params = make_params(params, tf_dev)
            req.rgba = _dev_ptr(rgba, torch.float32, (h, w, 4), "rgba").value
            keep.append(tf_dev)
        else:                    # fake executor: any non-null address
            req.params = L.RenderParams()
            req.rgba = int(rgba)
        if cam is not None:
            req.camera = make_camera(cam)
        req.w, req.h = int(w), int(h)
        return self._submit(req, keep)

    def submit_points(self, model_id: int, xyz, out, n: Optional[int] = None) -> int:
        torch = _torch()
        req = L.Request()
        req.kind = L.MFA_REQ_POINTS
        req.model_id = model_id
        if isinstance(xyz, torch.Tensor):
            # xyz is read as [3][n] from its start; a larger buffer may carry
            # a smaller n (its first 3n floats are the coordinates)
            n = int(xyz.shape[1]) if n is None else int(n)
            req.xyz = _dev_ptr(xyz, torch.float32, None, "xyz").value
            req.out = _dev_ptr(out, torch.float32, None, "out").value
            if xyz.numel() < 3 * n or out.numel() < 4 * n:
                raise ValueError("xyz / out smaller than 3n / 4n floats")
        else:                    # fake executor: any non-null addresses
            req.xyz, req.out = int(xyz), int(out)
        req.n = int(n)
        return self._submit(req, [xyz, out])

    def poll(self, ticket: int) -> dict:
        st = L.RequestStats()
        L.check(L.lib().mfa_server_poll(self._h, ticket, C.byref(st)))
        return {f: getattr(st, f) for f, _ in L.RequestStats._fields_}

    def wait(self, ticket: int) -> dict:
        st = L.RequestStats()
        L.check(L.lib().mfa_server_wait(self._h, ticket, C.byref(st)))
        self._keep.pop(ticket, None)
        return {f: getattr(st, f) for f, _ in L.RequestStats._fields_}

    def release(self, ticket: int) -> None:
        L.check(L.lib().mfa_server_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def close(self):
        if getattr(self, "_h", None) is not None:
            L.lib().mfa_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def quantize(x: np.ndarray, dtype: str) -> np.ndarray:
    """Host-side storage rounding of the library (no device work)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.uint32 if dtype == "f32" else np.uint16)
    L.check(L.lib().mfa_quantize(x.ctypes.data, x.size, _DTYPES[dtype], out.ctypes.data))
    return out


def default_knots(n: int, p: int) -> np.ndarray:
    out = np.zeros(n + p + 1)
    L.check(L.lib().mfa_default_knots(n, p, out.ctypes.data))
    return out


def version() -> str:
    return L.lib().mfa_version().decode()
