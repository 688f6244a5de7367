"""ctypes binding of the C oracle (oracle/soup_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark call it; the product path never does.

All functions take a ``workloads.Scene`` and a ``workloads.View`` (plain
numpy containers) and return numpy arrays. Gradients come back as float64.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoup_oracle.so")

BG_KEY = np.uint64(0xFFFFFFFFFFFFFFFF)


class _Scene(C.Structure):
    _fields_ = [("T", C.c_int32), ("G", C.c_int32), ("C", C.c_int32), ("n_layers", C.c_int32),
                ("dims", C.POINTER(C.c_int32)), ("verts", C.c_void_p), ("feats", C.c_void_p),
                ("mlp", C.c_void_p)]


class _View(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("view_id", C.c_uint32), ("M", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint32), ("mode", C.c_int32),
                ("background", C.c_float * 3), ("edge_pairs", C.c_int32), ("near_w", C.c_float),
                ("analysis", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("covered_pixels", C.c_int64), ("covering_fragments", C.c_int64),
                ("decodes", C.c_int64), ("winners", C.c_int64), ("front_fragments", C.c_int64)]


class _PScene(C.Structure):
    _fields_ = [("T", C.c_int32), ("R", C.c_int32), ("verts", C.c_void_p), ("tex", C.c_void_p),
                ("mlp", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_forward.argtypes = [P, P, P, P, P, P, P]
        L.orc_backward.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.orc_forward_pixels.argtypes = [P, P, P, C.c_int64, P, P, P, P]
        L.orc_backward_pixels.argtypes = [P, P, P, C.c_int64, P, P, P, P, P, P]
        L.orc_pixel_fragments.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P]
        L.orc_color_f64.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P]
        L.orc_exp.argtypes = [C.c_float]
        L.orc_exp.restype = C.c_float
        L.orc_sigmoid.argtypes = [C.c_float]
        L.orc_sigmoid.restype = C.c_float
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_uniform.restype = C.c_float
        L.orc_count_valid.argtypes = [P, P, P]
        L.orc_count_valid.restype = C.c_int64
        L.orc_threads.restype = C.c_int
        L.orc_mc_count.argtypes = [C.c_int]
        L.orc_mc_lookup.argtypes = [C.c_int, C.c_float, C.c_float, P, P]
        L.orc_mc_assemble.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P]
        L.orc_mc_assemble_bwd.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P, P]
        L.orc_sh2.argtypes = [P, P]
        L.orc_sh2.restype = None
        L.orc_view_dir.argtypes = [P, P, C.c_int32, C.c_int32, P]
        L.orc_pforward.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_pbackward.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
        L.orc_pforward_pixels.argtypes = [P, P, P, P, C.c_int64, P, P, P, P]
        L.orc_pbackward_pixels.argtypes = [P, P, P, P, C.c_int64, P, P, P, P, P, P]
        L.orc_pcolor_f64.argtypes = [P, P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the numpy buffers the C structs point to."""

    def __init__(self, scene, view, opts):
        self.verts = np.ascontiguousarray(scene.verts, dtype=np.float32)
        self.feats = np.ascontiguousarray(scene.feats, dtype=np.float32)
        self.mlp = np.ascontiguousarray(scene.mlp, dtype=np.float32)
        self.dims = np.ascontiguousarray(np.asarray(scene.dims, dtype=np.int32))
        self.M = np.ascontiguousarray(view.M, dtype=np.float32)
        self.s = _Scene(self.verts.shape[0], self.feats.shape[1], self.feats.shape[3],
                        len(scene.dims) - 1, self.dims.ctypes.data_as(C.POINTER(C.c_int32)),
                        self.verts.ctypes.data, self.feats.ctypes.data, self.mlp.ctypes.data)
        self.v = _View(view.width, view.height, view.view_id, self.M.ctypes.data)
        self.o = _Opts(opts.seed, opts.step, opts.mode, (C.c_float * 3)(*opts.background),
                       opts.edge_pairs, opts.near_w, opts.analysis)

    def args(self):
        return C.byref(self.s), C.byref(self.v), C.byref(self.o)


class Opts:
    def __init__(self, seed: int = 0, step: int = 0, mode: int = 0, background=(0.0, 0.0, 0.0),
                 edge_pairs: int = 0, near_w: float = 0.1, analysis: int = 0):
        self.seed, self.step, self.mode = int(seed), int(step), int(mode)
        self.background = tuple(float(b) for b in background)
        self.edge_pairs, self.near_w, self.analysis = int(edge_pairs), float(near_w), int(analysis)


def n_params(dims: Sequence[int]) -> int:
    return int(sum(o * i + o for i, o in zip(dims[:-1], dims[1:])))


def forward(scene, view, opts: Opts, want_logp: bool = True):
    k = _Keep(scene, view, opts)
    H, W = view.height, view.width
    vis = np.empty(H * W, np.uint64)
    color = np.empty(H * W * 3, np.float32)
    logp = np.empty(H * W, np.float64) if want_logp else None
    st = _Stats()
    rc = lib().orc_forward(*k.args(), _ptr(vis), _ptr(color), _ptr(logp) if want_logp else None,
                           C.byref(st))
    if rc != 0:
        raise ValueError("oracle forward rejected its arguments")
    stats = {f: int(getattr(st, f)) for f, _ in _Stats._fields_}
    return (vis.reshape(H, W), color.reshape(H, W, 3),
            logp.reshape(H, W) if want_logp else None, stats)


def backward(scene, view, opts: Opts, vis, color, grad_color, grad_logp=None, out=None):
    """Gradients of one view; with out = (gv, gf, gm) (contiguous float64
    arrays of the gradient shapes) they are added into those arrays."""
    k = _Keep(scene, view, opts)
    T, G, Cc = scene.verts.shape[0], scene.feats.shape[1], scene.feats.shape[3]
    if out is not None:
        gv, gf, gm = (o.reshape(-1) for o in out)
        assert gv.size == T * 9 and gf.size == T * G * G * Cc and gm.size == n_params(scene.dims)
        assert all(o.dtype == np.float64 and o.flags.c_contiguous for o in out)
    else:
        gv = np.zeros(T * 9, np.float64)
        gf = np.zeros(T * G * G * Cc, np.float64)
        gm = np.zeros(n_params(scene.dims), np.float64)
    vis = np.ascontiguousarray(vis, dtype=np.uint64).ravel()
    color = np.ascontiguousarray(color, dtype=np.float32).ravel()
    gc = np.ascontiguousarray(grad_color, dtype=np.float32).ravel()
    gl = None if grad_logp is None else np.ascontiguousarray(grad_logp, dtype=np.float32).ravel()
    rc = lib().orc_backward(*k.args(), _ptr(vis), _ptr(color), _ptr(gc),
                            _ptr(gl) if gl is not None else None, _ptr(gv), _ptr(gf), _ptr(gm))
    if rc != 0:
        raise ValueError("oracle backward rejected its arguments")
    return gv.reshape(T, 3, 3), gf.reshape(T, G, G, Cc), gm


def forward_pixels(scene, view, opts: Opts, xy: np.ndarray):
    k = _Keep(scene, view, opts)
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    vis = np.empty(n, np.uint64)
    color = np.empty(n * 3, np.float32)
    logp = np.empty(n, np.float64)
    rc = lib().orc_forward_pixels(*k.args(), n, _ptr(xy), _ptr(vis), _ptr(color), _ptr(logp))
    if rc != 0:
        raise ValueError("oracle forward_pixels rejected its arguments")
    return vis, color.reshape(n, 3), logp


def backward_pixels(scene, view, opts: Opts, xy, grad_color, grad_logp=None):
    k = _Keep(scene, view, opts)
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    T, G, Cc = scene.verts.shape[0], scene.feats.shape[1], scene.feats.shape[3]
    gv = np.zeros(T * 9, np.float64)
    gf = np.zeros(T * G * G * Cc, np.float64)
    gm = np.zeros(n_params(scene.dims), np.float64)
    gc = np.ascontiguousarray(grad_color, dtype=np.float32).reshape(-1)
    gl = None if grad_logp is None else np.ascontiguousarray(grad_logp, dtype=np.float32).reshape(-1)
    rc = lib().orc_backward_pixels(*k.args(), n, _ptr(xy), _ptr(gc),
                                   _ptr(gl) if gl is not None else None, _ptr(gv), _ptr(gf), _ptr(gm))
    if rc != 0:
        raise ValueError("oracle backward_pixels rejected its arguments")
    return gv.reshape(T, 3, 3), gf.reshape(T, G, G, Cc), gm


def pixel_fragments(scene, view, opts: Opts, x: int, y: int, cap: int = 4096):
    k = _Keep(scene, view, opts)
    tri = np.zeros(cap, np.uint32)
    key = np.zeros(cap, np.uint64)
    alpha = np.zeros(cap, np.float32)
    o3 = np.zeros(cap, np.float32)
    u = np.zeros(cap, np.float32)
    dl = np.zeros(cap, np.float64)
    win = C.c_int32(0)
    n = lib().orc_pixel_fragments(*k.args(), x, y, cap, _ptr(tri), _ptr(key), _ptr(alpha), _ptr(o3),
                                  _ptr(u), _ptr(dl), C.byref(win))
    if n < 0:
        raise ValueError("oracle pixel_fragments rejected its arguments")
    m = min(n, cap)
    return dict(n=n, tri=tri[:m], key=key[:m], alpha=alpha[:m], o3=o3[:m], u=u[:m],
                dlogit=dl[:m], winner=int(win.value))


def color_f64(scene, view, opts: Opts, tri: int, x: int, y: int):
    k = _Keep(scene, view, opts)
    rgb = np.zeros(3, np.float64)
    a = C.c_double(0)
    rc = lib().orc_color_f64(*k.args(), tri, x, y, _ptr(rgb), C.byref(a))
    if rc < 0:
        raise ValueError("bad arguments")
    return (rgb, a.value) if rc == 1 else (None, None)


def exp(x: float) -> float:
    return float(lib().orc_exp(x))


def sigmoid(x: float) -> float:
    return float(lib().orc_sigmoid(x))


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, pixel: int, tri: int, view_id: int, step: int) -> float:
    return float(lib().orc_uniform(seed, pixel, tri, view_id, step))


def count_valid(scene, view, opts: Opts) -> int:
    k = _Keep(scene, view, opts)
    return int(lib().orc_count_valid(*k.args()))


def threads() -> int:
    return int(lib().orc_threads())


# ---------------------------------------------------------------------------
# Paper form (Section 3.3; Supplement B.3, B.6): mesh-colour texture, opacity
# outside the MLP, deferred shading with spherical harmonics. A paper-form
# scene has verts [T,3,3], tex [T,V(R),8] (activated), mlp (the 16-16-16-3
# MLP's flat parameters) and R.
# ---------------------------------------------------------------------------

N_PCH = 8


def mc_count(R: int) -> int:
    return int(lib().orc_mc_count(R))


def pmlp_params() -> int:
    return int(lib().orc_pmlp_params())


def mc_lookup(R: int, b1: float, b2: float):
    idx = np.zeros(3, np.int32)
    w = np.zeros(3, np.float32)
    lib().orc_mc_lookup(R, b1, b2, _ptr(idx), _ptr(w))
    return idx, w


def mc_assemble(raw: Sequence[np.ndarray], Rmin: int, Rmax: Optional[int] = None):
    """tex [T, V(Rmax), 8] = sigmoid(sum of the learnable levels sampled at the
    level-Rmax grid's vertices); raw[l] is [T, V(Rmin + l), 8]; Rmax defaults
    to the top learnable level."""
    raw = [np.ascontiguousarray(r, dtype=np.float32) for r in raw]
    Rtop = Rmin + len(raw) - 1
    Rmax = Rtop if Rmax is None else Rmax
    T = raw[0].shape[0]
    for l, r in enumerate(raw):
        assert r.shape == (T, mc_count(Rmin + l), N_PCH)
    tex = np.empty((T, mc_count(Rmax), N_PCH), np.float32)
    ptrs = (C.c_void_p * len(raw))(*[r.ctypes.data for r in raw])
    if lib().orc_mc_assemble(T, Rmin, Rtop, Rmax, ptrs, _ptr(tex)) != 0:
        raise ValueError("oracle mc_assemble rejected its arguments")
    return tex


def mc_assemble_bwd(tex, grad_tex, Rmin: int, n_levels: int, Rmax: Optional[int] = None):
    tex = np.ascontiguousarray(tex, dtype=np.float32)
    gt = np.ascontiguousarray(grad_tex, dtype=np.float32)
    T = tex.shape[0]
    Rtop = Rmin + n_levels - 1
    Rmax = Rtop if Rmax is None else Rmax
    outs = [np.zeros((T, mc_count(Rmin + l), N_PCH), np.float64) for l in range(n_levels)]
    ptrs = (C.c_void_p * n_levels)(*[o.ctypes.data for o in outs])
    if lib().orc_mc_assemble_bwd(T, Rmin, Rtop, Rmax, _ptr(tex), _ptr(gt), ptrs) != 0:
        raise ValueError("oracle mc_assemble_bwd rejected its arguments")
    return outs


def sh2(d) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float32)
    out = np.zeros(9, np.float32)
    lib().orc_sh2(_ptr(d), _ptr(out))
    return out


def view_dir(view, minv, x: int, y: int) -> np.ndarray:
    M = np.ascontiguousarray(view.M, dtype=np.float32)
    Mi = np.ascontiguousarray(minv, dtype=np.float32).reshape(16)
    v = _View(view.width, view.height, view.view_id, M.ctypes.data)
    d = np.zeros(3, np.float32)
    if lib().orc_view_dir(C.byref(v), _ptr(Mi), x, y, _ptr(d)) != 0:
        raise ValueError("bad pixel")
    return d


class _PKeep:
    def __init__(self, ps, view, minv, opts):
        self.verts = np.ascontiguousarray(ps.verts, dtype=np.float32)
        self.tex = np.ascontiguousarray(ps.tex, dtype=np.float32)
        self.mlp = np.ascontiguousarray(ps.mlp, dtype=np.float32)
        T = self.verts.shape[0]
        assert self.tex.shape == (T, mc_count(ps.R), N_PCH) and self.mlp.size == pmlp_params()
        self.M = np.ascontiguousarray(view.M, dtype=np.float32)
        self.Minv = np.ascontiguousarray(minv, dtype=np.float32).reshape(16)
        self.s = _PScene(T, ps.R, self.verts.ctypes.data, self.tex.ctypes.data, self.mlp.ctypes.data)
        self.v = _View(view.width, view.height, view.view_id, self.M.ctypes.data)
        self.o = _Opts(opts.seed, opts.step, opts.mode, (C.c_float * 3)(*opts.background),
                       opts.edge_pairs, opts.near_w, opts.analysis)

    def args(self):
        return C.byref(self.s), C.byref(self.v), _ptr(self.Minv), C.byref(self.o)


def pforward(ps, view, minv, opts: Opts, want_logp: bool = True):
    k = _PKeep(ps, view, minv, opts)
    H, W = view.height, view.width
    vis = np.empty(H * W, np.uint64)
    color = np.empty(H * W * 3, np.float32)
    logp = np.empty(H * W, np.float64) if want_logp else None
    st = _Stats()
    rc = lib().orc_pforward(*k.args(), _ptr(vis), _ptr(color), _ptr(logp) if want_logp else None, C.byref(st))
    if rc != 0:
        raise ValueError("oracle pforward rejected its arguments")
    stats = {f: int(getattr(st, f)) for f, _ in _Stats._fields_}
    return vis.reshape(H, W), color.reshape(H, W, 3), (logp.reshape(H, W) if want_logp else None), stats


def pbackward(ps, view, minv, opts: Opts, vis, color, grad_color, grad_logp=None, out=None):
    """Gradients of one paper-form view (float64): d verts [T,3,3], d tex
    [T,V,8], d mlp; with out = (gv, gt, gm) they are added into those arrays."""
    k = _PKeep(ps, view, minv, opts)
    T, V = k.tex.shape[0], k.tex.shape[1]
    if out is not None:
        gv, gt, gm = (o.reshape(-1) for o in out)
        assert gv.size == T * 9 and gt.size == T * V * N_PCH and gm.size == pmlp_params()
        assert all(o.dtype == np.float64 and o.flags.c_contiguous for o in out)
    else:
        gv = np.zeros(T * 9, np.float64)
        gt = np.zeros(T * V * N_PCH, np.float64)
        gm = np.zeros(pmlp_params(), np.float64)
    vis = np.ascontiguousarray(vis, dtype=np.uint64).ravel()
    color = np.ascontiguousarray(color, dtype=np.float32).ravel()
    gc = np.ascontiguousarray(grad_color, dtype=np.float32).ravel()
    gl = None if grad_logp is None else np.ascontiguousarray(grad_logp, dtype=np.float32).ravel()
    rc = lib().orc_pbackward(*k.args(), _ptr(vis), _ptr(color), _ptr(gc), _ptr(gl) if gl is not None else None,
                             _ptr(gv), _ptr(gt), _ptr(gm))
    if rc != 0:
        raise ValueError("oracle pbackward rejected its arguments")
    return gv.reshape(T, 3, 3), gt.reshape(T, V, N_PCH), gm


def pforward_pixels(ps, view, minv, opts: Opts, xy):
    k = _PKeep(ps, view, minv, opts)
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    vis = np.empty(n, np.uint64)
    color = np.empty(n * 3, np.float32)
    logp = np.empty(n, np.float64)
    if lib().orc_pforward_pixels(*k.args(), n, _ptr(xy), _ptr(vis), _ptr(color), _ptr(logp)) != 0:
        raise ValueError("oracle pforward_pixels rejected its arguments")
    return vis, color.reshape(n, 3), logp


def pbackward_pixels(ps, view, minv, opts: Opts, xy, grad_color, grad_logp=None):
    k = _PKeep(ps, view, minv, opts)
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    T, V = k.tex.shape[0], k.tex.shape[1]
    gv = np.zeros(T * 9, np.float64)
    gt = np.zeros(T * V * N_PCH, np.float64)
    gm = np.zeros(pmlp_params(), np.float64)
    gc = np.ascontiguousarray(grad_color, dtype=np.float32).reshape(-1)
    gl = None if grad_logp is None else np.ascontiguousarray(grad_logp, dtype=np.float32).reshape(-1)
    if lib().orc_pbackward_pixels(*k.args(), n, _ptr(xy), _ptr(gc), _ptr(gl) if gl is not None else None,
                                  _ptr(gv), _ptr(gt), _ptr(gm)) != 0:
        raise ValueError("oracle pbackward_pixels rejected its arguments")
    return gv.reshape(T, 3, 3), gt.reshape(T, V, N_PCH), gm


def pcolor_f64(ps, view, minv, opts: Opts, tri: int, x: int, y: int):
    k = _PKeep(ps, view, minv, opts)
    rgb = np.zeros(3, np.float64)
    a = C.c_double(0)
    rc = lib().orc_pcolor_f64(*k.args(), tri, x, y, _ptr(rgb), C.byref(a))
    if rc < 0:
        raise ValueError("bad arguments")
    return (rgb, a.value) if rc == 1 else (None, None)
