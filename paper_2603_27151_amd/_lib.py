"""ctypes binding of libdiffsoup.so (include/diffsoup.h), argument
marshalling only: every step of the rasterization runs in the library's HIP
kernels. Functions carry the C names; tensors are torch tensors on the GPU
(device memory and streams come from PyTorch).

The library is loaded from this package directory. If it is missing the
import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffsoup.so")

SOUP_OK = 0
STATUS = {0: "SOUP_OK", 1: "SOUP_ERR_INVALID", 2: "SOUP_ERR_OOM", 3: "SOUP_ERR_CAPACITY",
          4: "SOUP_ERR_HIP", 5: "SOUP_ERR_UNSUPPORTED"}
BG_KEY = 0xFFFFFFFFFFFFFFFF


class soup_scene(C.Structure):
    _fields_ = [("T", C.c_int32), ("G", C.c_int32), ("C", C.c_int32), ("n_layers", C.c_int32),
                ("dims", C.POINTER(C.c_int32)), ("verts", C.c_void_p), ("feats", C.c_void_p),
                ("mlp", C.c_void_p)]


class soup_views(C.Structure):
    _fields_ = [("V", C.c_int32), ("width", C.POINTER(C.c_int32)), ("height", C.POINTER(C.c_int32)),
                ("view_id", C.POINTER(C.c_uint32)), ("view_proj", C.POINTER(C.c_float))]


class soup_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint32), ("mode", C.c_int32),
                ("background", C.c_float * 3), ("edge_pairs", C.c_int32), ("near_w", C.c_float),
                ("accumulate", C.c_int32), ("reuse_bins", C.c_int32)]


class soup_pscene(C.Structure):
    _fields_ = [("T", C.c_int32), ("R", C.c_int32), ("verts", C.c_void_p), ("tex", C.c_void_p),
                ("mlp", C.c_void_p)]


class soup_stats(C.Structure):
    _fields_ = [("pixels", C.c_int64), ("tiles", C.c_int64), ("bin_entries", C.c_int64),
                ("visible_tris", C.c_int64), ("decodes", C.c_int64), ("covered_pixels", C.c_int64)]


EXPORTS = ["soup_ctx_create", "soup_ctx_destroy", "soup_last_error", "soup_ctx_set_tile",
           "soup_ctx_get_tile", "soup_ctx_set_counting", "soup_last_stats", "soup_rasterize_fwd",
           "soup_rasterize_bwd", "soup_render", "soup_loss_l2", "soup_selftest_sigmoid",
           "soup_selftest_uniform", "soup_ctx_set_timing", "soup_read_timings", "soup_ctx_set_static",
           "soup_ctx_check", "soup_coverage_count", "soup_edge_lengths", "soup_adaptive_plan",
           "soup_adaptive_apply", "soup_loss_l1_ssim", "soup_adam_step", "soup_loss_l1_ssim_noalloc",
           "soup_pforward", "soup_pbackward", "soup_pbackward_levels", "soup_mc_assemble",
           "soup_mc_assemble_bwd", "soup_ctx_workspace_bytes", "soup_probe_copy", "soup_probe_read",
           "soup_probe_atomic", "soup_probe_fma", "soup_probe_mfma"]
TIMING_KINDS = ["setup", "scan", "scatter", "sort", "raster_fwd", "decode_bwd", "edge", "vertex_chain",
                "mlp_reduce", "logp", "loss", "fill", "replay", "grad_reduce", "coverage", "edge_lengths",
                "adaptive_apply", "train_loss", "adam", "shade", "assemble", "assemble_bwd"]
PMLP_PARAMS = 595
ACT_REMOVE, ACT_KEEP, ACT_SPLIT0 = 0, 1, 2
PLAN_PRUNE_ZERO, PLAN_FILL = 1, 2

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc, gfx950); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.soup_ctx_create.argtypes = [C.POINTER(P), C.c_int]
    L.soup_ctx_destroy.argtypes = [P]
    L.soup_ctx_destroy.restype = None
    L.soup_last_error.argtypes = [P]
    L.soup_last_error.restype = C.c_char_p
    L.soup_ctx_set_tile.argtypes = [P, C.c_int32]
    L.soup_ctx_get_tile.argtypes = [P]
    L.soup_ctx_set_counting.argtypes = [P, C.c_int32]
    L.soup_last_stats.argtypes = [P, C.POINTER(soup_stats)]
    L.soup_rasterize_fwd.argtypes = [P, C.POINTER(soup_scene), C.POINTER(soup_views), C.POINTER(soup_opts),
                                     P, P, P, P]
    L.soup_rasterize_bwd.argtypes = [P, C.POINTER(soup_scene), C.POINTER(soup_views), C.POINTER(soup_opts),
                                     P, P, P, P, P, P, P, P]
    L.soup_render.argtypes = [P, C.POINTER(soup_scene), C.c_int32, C.POINTER(soup_views),
                              C.POINTER(soup_opts), C.POINTER(P), P]
    L.soup_loss_l2.argtypes = [P, P, P, C.c_int64, P, P, P, P]
    L.soup_selftest_sigmoid.argtypes = [P, P, P, C.c_int64, P]
    L.soup_selftest_uniform.argtypes = [P, C.c_uint64, P, P, C.c_uint32, C.c_uint32, P, C.c_int64, P]
    L.soup_ctx_set_static.argtypes = [P, C.c_int32]
    L.soup_ctx_check.argtypes = [P]
    L.soup_ctx_set_timing.argtypes = [P, C.c_int32]
    L.soup_read_timings.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.soup_coverage_count.argtypes = [P, P, C.c_int64, C.c_int32, P, P]
    L.soup_edge_lengths.argtypes = [P, P, C.c_int32, C.POINTER(soup_views), C.c_float, P, P]
    L.soup_adaptive_plan.argtypes = [P, P, P, C.c_int32, C.c_float, C.c_int32, C.c_int32, P, P,
                                     C.POINTER(C.c_int32)]
    L.soup_adaptive_apply.argtypes = [P, C.POINTER(soup_scene), P, P, C.c_int32, P, P, P]
    L.soup_loss_l1_ssim.argtypes = [P, P, P, C.POINTER(soup_views), C.c_float, P, P, P, P]
    L.soup_loss_l1_ssim_noalloc.argtypes = [P, P, P, C.POINTER(soup_views), C.c_float, P, P, P, P]
    L.soup_adam_step.argtypes = [P, P, P, P, P, C.c_int64, C.c_int32, C.c_float, C.c_double, C.c_double, C.c_float,
                                 C.c_int32, P]
    L.soup_pforward.argtypes = [P, C.POINTER(soup_pscene), C.POINTER(soup_views), P, C.POINTER(soup_opts),
                                P, P, P, P]
    L.soup_pbackward.argtypes = [P, C.POINTER(soup_pscene), C.POINTER(soup_views), P, C.POINTER(soup_opts),
                                 P, P, P, P, P, P, P, P]
    L.soup_pbackward_levels.argtypes = [P, C.POINTER(soup_pscene), C.POINTER(soup_views), P, C.POINTER(soup_opts),
                                        P, P, P, P, C.c_int32, C.c_int32, P, P, P, P]
    L.soup_mc_assemble.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P]
    L.soup_mc_assemble_bwd.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P, C.c_int32, P]
    L.soup_ctx_workspace_bytes.argtypes = [P, C.POINTER(C.c_int64)]
    L.soup_probe_copy.argtypes = [P, P, P, C.c_int64, P]
    L.soup_probe_read.argtypes = [P, P, C.c_int64, P, C.c_int64, P]
    L.soup_probe_atomic.argtypes = [P, P, C.c_int64, C.c_int64, P]
    L.soup_probe_fma.argtypes = [P, P, C.c_int64, C.c_int32, P]
    L.soup_probe_mfma.argtypes = [P, P, C.c_int64, C.c_int32, P]
    for name in ["soup_pforward", "soup_pbackward", "soup_pbackward_levels", "soup_mc_assemble",
                 "soup_mc_assemble_bwd", "soup_ctx_workspace_bytes", "soup_probe_copy", "soup_probe_read",
                 "soup_probe_atomic", "soup_probe_fma", "soup_probe_mfma"]:
        getattr(L, name).restype = C.c_int
    for name in ["soup_ctx_create", "soup_ctx_set_tile", "soup_ctx_set_counting", "soup_last_stats",
                 "soup_rasterize_fwd", "soup_rasterize_bwd", "soup_render", "soup_loss_l2",
                 "soup_selftest_sigmoid", "soup_selftest_uniform", "soup_ctx_set_timing",
                 "soup_read_timings", "soup_ctx_set_static", "soup_ctx_check", "soup_coverage_count",
                 "soup_edge_lengths", "soup_adaptive_plan", "soup_adaptive_apply", "soup_loss_l1_ssim",
                 "soup_adam_step", "soup_loss_l1_ssim_noalloc"]:
        getattr(L, name).restype = C.c_int
    L.soup_ctx_get_tile.restype = C.c_int32
    _lib = L
    return L


class SoupError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class _Holder:
    """Keeps host arrays alive while a C struct points at them."""

    def __init__(self):
        self.keep = []

    def arr(self, a, ctype):
        a = np.ascontiguousarray(a)
        self.keep.append(a)
        return a.ctypes.data_as(C.POINTER(ctype))


def make_scene(h: _Holder, verts, feats, mlp, dims: Sequence[int]) -> soup_scene:
    T = int(verts.shape[0])
    G = int(feats.shape[1])
    Cc = int(feats.shape[3])
    for name, t in (("verts", verts), ("feats", feats), ("mlp", mlp)):
        if not t.is_cuda or t.dtype.itemsize != 4 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(verts.shape[1:]) != (3, 3) or tuple(feats.shape) != (T, G, G, Cc):
        raise ValueError("verts must be [T,3,3] and feats [T,G,G,C]")
    d = np.asarray(dims, np.int32)
    return soup_scene(T, G, Cc, len(dims) - 1, h.arr(d, C.c_int32), _ptr(verts), _ptr(feats), _ptr(mlp))


def make_pscene(verts, tex, mlp, R: int) -> soup_pscene:
    T = int(verts.shape[0])
    V = ((1 << R) + 1) * ((1 << R) + 2) // 2
    for name, t in (("verts", verts), ("tex", tex), ("mlp", mlp)):
        if not t.is_cuda or t.dtype.itemsize != 4 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(verts.shape[1:]) != (3, 3) or tuple(tex.shape) != (T, V, 8) or mlp.numel() != PMLP_PARAMS:
        raise ValueError(f"verts must be [T,3,3], tex [T,{V},8] and mlp [{PMLP_PARAMS}]")
    return soup_pscene(T, int(R), _ptr(verts), _ptr(tex), _ptr(mlp))


def make_views(h: _Holder, widths, heights, view_ids, view_proj) -> soup_views:
    w = np.asarray(widths, np.int32)
    hh = np.asarray(heights, np.int32)
    vid = np.asarray(view_ids, np.uint32)
    M = np.ascontiguousarray(np.asarray(view_proj, np.float32).reshape(-1, 16))
    if not (len(w) == len(hh) == len(vid) == M.shape[0]):
        raise ValueError("views: widths, heights, view_ids and view_proj disagree in length")
    return soup_views(len(w), h.arr(w, C.c_int32), h.arr(hh, C.c_int32), h.arr(vid, C.c_uint32),
                      h.arr(M, C.c_float))


def make_opts(seed=0, step=0, mode=0, background=(0.0, 0.0, 0.0), edge_pairs=0, near_w=0.1,
              accumulate=0, reuse_bins=0) -> soup_opts:
    return soup_opts(int(seed) & 0xFFFFFFFFFFFFFFFF, int(step), int(mode), (C.c_float * 3)(*background),
                     int(edge_pairs), float(near_w), int(accumulate), int(reuse_bins))


class Ctx:
    """Owns one soup_ctx (workspaces on one device)."""

    def __init__(self, device: int = 0):
        L = lib()
        p = C.c_void_p()
        st = L.soup_ctx_create(C.byref(p), int(device))
        if st != SOUP_OK:
            raise SoupError(st, f"soup_ctx_create(device={device}) failed")
        self.p = p
        self.device = device

    def close(self):
        if self.p:
            lib().soup_ctx_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != SOUP_OK:
            raise SoupError(st, lib().soup_last_error(self.p).decode())

    def set_tile(self, tile: int):
        self.check(lib().soup_ctx_set_tile(self.p, int(tile)))

    @property
    def tile(self) -> int:
        return int(lib().soup_ctx_get_tile(self.p))

    def set_static(self, on: bool):
        """Static-capacity mode (no synchronisation or allocation; HIP-graph capturable)."""
        self.check(lib().soup_ctx_set_static(self.p, 1 if on else 0))

    def check_overflow(self):
        """Raises SoupError(SOUP_ERR_CAPACITY) if a static-mode call overflowed since the last check."""
        self.check(lib().soup_ctx_check(self.p))

    def set_counting(self, on: bool):
        self.check(lib().soup_ctx_set_counting(self.p, 1 if on else 0))

    def set_timing(self, on: bool):
        self.check(lib().soup_ctx_set_timing(self.p, 1 if on else 0))

    def read_timings(self) -> dict:
        """{kind: (total ms, launches)} of the events recorded since the last read."""
        n = len(TIMING_KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self.check(lib().soup_read_timings(self.p, ms, cnt))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(TIMING_KINDS)}

    def workspace_bytes(self) -> int:
        n = C.c_int64(0)
        self.check(lib().soup_ctx_workspace_bytes(self.p, C.byref(n)))
        return int(n.value)

    def stats(self) -> dict:
        s = soup_stats()
        self.check(lib().soup_last_stats(self.p, C.byref(s)))
        return {f: int(getattr(s, f)) for f, _ in soup_stats._fields_}


# ---------------------------------------------------------------------------
# entry points (C names; torch tensors in, torch tensors out)
# ---------------------------------------------------------------------------

def soup_rasterize_fwd(ctx: Ctx, scene: soup_scene, views: soup_views, opts: soup_opts, vis, color,
                       logp=None, stream=None):
    ctx.check(lib().soup_rasterize_fwd(ctx.p, C.byref(scene), C.byref(views), C.byref(opts), _ptr(vis),
                                       _ptr(color), _ptr(logp), _stream(stream)))


def soup_rasterize_bwd(ctx: Ctx, scene: soup_scene, views: soup_views, opts: soup_opts, vis, color,
                       grad_color, grad_logp, grad_verts, grad_feats, grad_mlp, stream=None):
    ctx.check(lib().soup_rasterize_bwd(ctx.p, C.byref(scene), C.byref(views), C.byref(opts), _ptr(vis),
                                       _ptr(color), _ptr(grad_color), _ptr(grad_logp), _ptr(grad_verts),
                                       _ptr(grad_feats), _ptr(grad_mlp), _stream(stream)))


def soup_render(ctx: Ctx, scenes: Sequence[soup_scene], views: soup_views, opts: soup_opts, colors,
                stream=None):
    R = len(scenes)
    arr = (soup_scene * R)(*scenes)
    outs = (C.c_void_p * R)(*[_ptr(c) for c in colors])
    ctx.check(lib().soup_render(ctx.p, arr, R, C.byref(views), C.byref(opts), outs, _stream(stream)))


def soup_loss_l2(ctx: Ctx, color, target, grad_color, grad_logp, loss=None, stream=None):
    P = color.numel() // 3
    ctx.check(lib().soup_loss_l2(ctx.p, _ptr(color), _ptr(target), P, _ptr(grad_color), _ptr(grad_logp),
                                 _ptr(loss), _stream(stream)))


def soup_selftest_sigmoid(ctx: Ctx, x, y, stream=None):
    ctx.check(lib().soup_selftest_sigmoid(ctx.p, _ptr(x), _ptr(y), x.numel(), _stream(stream)))


def soup_selftest_uniform(ctx: Ctx, seed, pixel, tri, view_id, step, u, stream=None):
    ctx.check(lib().soup_selftest_uniform(ctx.p, int(seed), _ptr(pixel), _ptr(tri), int(view_id), int(step),
                                          _ptr(u), u.numel(), _stream(stream)))


def soup_coverage_count(ctx: Ctx, vis, T: int, counts, stream=None):
    ctx.check(lib().soup_coverage_count(ctx.p, _ptr(vis), vis.numel(), int(T), _ptr(counts), _stream(stream)))


def soup_edge_lengths(ctx: Ctx, verts, views: soup_views, near_w: float, rel_len, stream=None):
    ctx.check(lib().soup_edge_lengths(ctx.p, _ptr(verts), int(verts.shape[0]), C.byref(views), float(near_w),
                                      _ptr(rel_len), _stream(stream)))


def soup_adaptive_plan(counts: np.ndarray, rel_len: np.ndarray, split_frac: float, target: int, flags: int = 0):
    """Host arrays in, (actions int32 [T], offsets int32 [T], n_new) out; needs no GPU."""
    cnt = np.ascontiguousarray(counts, dtype=np.uint32)
    rel = np.ascontiguousarray(rel_len, dtype=np.float32).reshape(-1)
    T = cnt.shape[0]
    if rel.shape[0] != 3 * T:
        raise ValueError("rel_len must hold 3 lengths per triangle")
    act = np.zeros(T, np.int32)
    off = np.zeros(T, np.int32)
    n = C.c_int32(0)
    st = lib().soup_adaptive_plan(None, cnt.ctypes.data_as(C.c_void_p), rel.ctypes.data_as(C.c_void_p), T,
                                  float(split_frac), int(target), int(flags), act.ctypes.data_as(C.c_void_p),
                                  off.ctypes.data_as(C.c_void_p), C.byref(n))
    if st != 0:
        raise SoupError(st, "soup_adaptive_plan: bad arguments")
    return act, off, int(n.value)


def soup_adaptive_apply(ctx: Ctx, scene: soup_scene, actions, offsets, n_new: int, verts_out, feats_out,
                        stream=None):
    ctx.check(lib().soup_adaptive_apply(ctx.p, C.byref(scene), _ptr(actions), _ptr(offsets), int(n_new),
                                        _ptr(verts_out), _ptr(feats_out), _stream(stream)))


def soup_loss_l1_ssim(ctx: Ctx, color, target, views: soup_views, lam: float, grad_color, grad_logp, loss=None,
                      stream=None):
    ctx.check(lib().soup_loss_l1_ssim(ctx.p, _ptr(color), _ptr(target), C.byref(views), float(lam),
                                      _ptr(grad_color), _ptr(grad_logp), _ptr(loss), _stream(stream)))


def soup_loss_l1_ssim_noalloc(ctx: Ctx, color, target, views: soup_views, lam: float, grad_color, grad_logp,
                              loss=None, stream=None):
    ctx.check(lib().soup_loss_l1_ssim_noalloc(ctx.p, _ptr(color), _ptr(target), C.byref(views), float(lam),
                                              _ptr(grad_color), _ptr(grad_logp), _ptr(loss), _stream(stream)))


def soup_adam_step(ctx: Ctx, p, g, m, v, vec: int, lr: float, beta1: float, beta2: float, eps: float, t: int,
                   stream=None):
    ctx.check(lib().soup_adam_step(ctx.p, _ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), int(vec), float(lr),
                                   float(beta1), float(beta2), float(eps), int(t), _stream(stream)))


def soup_pforward(ctx: Ctx, scene: soup_pscene, views: soup_views, inv_view_proj, opts: soup_opts, vis, color,
                  logp=None, stream=None):
    mi = np.ascontiguousarray(np.asarray(inv_view_proj, np.float32).reshape(-1, 16))
    if mi.shape[0] != views.V:
        raise ValueError("inv_view_proj needs one 4x4 matrix per view")
    ctx.check(lib().soup_pforward(ctx.p, C.byref(scene), C.byref(views), mi.ctypes.data_as(C.c_void_p),
                                  C.byref(opts), _ptr(vis), _ptr(color), _ptr(logp), _stream(stream)))


def soup_pbackward(ctx: Ctx, scene: soup_pscene, views: soup_views, inv_view_proj, opts: soup_opts, vis, color,
                   grad_color, grad_logp, grad_verts, grad_tex, grad_mlp, stream=None):
    mi = np.ascontiguousarray(np.asarray(inv_view_proj, np.float32).reshape(-1, 16))
    if mi.shape[0] != views.V:
        raise ValueError("inv_view_proj needs one 4x4 matrix per view")
    ctx.check(lib().soup_pbackward(ctx.p, C.byref(scene), C.byref(views), mi.ctypes.data_as(C.c_void_p),
                                   C.byref(opts), _ptr(vis), _ptr(color), _ptr(grad_color), _ptr(grad_logp),
                                   _ptr(grad_verts), _ptr(grad_tex), _ptr(grad_mlp), _stream(stream)))


def soup_pbackward_levels(ctx: Ctx, scene: soup_pscene, views: soup_views, inv_view_proj, opts: soup_opts, vis,
                          color, grad_color, grad_logp, Rmin: int, grad_verts, grad_raw: Sequence, grad_mlp,
                          stream=None):
    """grad_raw: device tensors of the learnable levels Rmin, Rmin + 1, ..."""
    mi = np.ascontiguousarray(np.asarray(inv_view_proj, np.float32).reshape(-1, 16))
    if mi.shape[0] != views.V:
        raise ValueError("inv_view_proj needs one 4x4 matrix per view")
    ptrs = (C.c_void_p * len(grad_raw))(*[_ptr(r) for r in grad_raw])
    Rtop = Rmin + len(grad_raw) - 1
    ctx.check(lib().soup_pbackward_levels(ctx.p, C.byref(scene), C.byref(views), mi.ctypes.data_as(C.c_void_p),
                                          C.byref(opts), _ptr(vis), _ptr(color), _ptr(grad_color),
                                          _ptr(grad_logp), int(Rmin), Rtop, _ptr(grad_verts), ptrs,
                                          _ptr(grad_mlp), _stream(stream)))


def soup_mc_assemble(ctx: Ctx, raw: Sequence, Rmin: int, Rmax: int, tex, stream=None):
    """raw: device tensors of the learnable levels Rmin, Rmin + 1, ...; tex [T, V(Rmax), 8]."""
    ptrs = (C.c_void_p * len(raw))(*[_ptr(r) for r in raw])
    Rtop = Rmin + len(raw) - 1
    ctx.check(lib().soup_mc_assemble(ctx.p, int(tex.shape[0]), int(Rmin), Rtop, int(Rmax), ptrs, _ptr(tex),
                                     _stream(stream)))


def soup_mc_assemble_bwd(ctx: Ctx, tex, grad_tex, Rmin: int, Rmax: int, grad_raw: Sequence, accumulate: int = 0,
                         stream=None):
    ptrs = (C.c_void_p * len(grad_raw))(*[_ptr(r) for r in grad_raw])
    Rtop = Rmin + len(grad_raw) - 1
    ctx.check(lib().soup_mc_assemble_bwd(ctx.p, int(tex.shape[0]), int(Rmin), Rtop, int(Rmax), _ptr(tex),
                                         _ptr(grad_tex), ptrs, int(accumulate), _stream(stream)))


# measured ceilings (kernels of known work; the caller times them on `stream`)
def soup_probe_copy(ctx: Ctx, src, dst, stream=None):
    ctx.check(lib().soup_probe_copy(ctx.p, _ptr(src), _ptr(dst), int(src.numel() * src.element_size()),
                                    _stream(stream)))


def soup_probe_read(ctx: Ctx, src, partial, stream=None):
    ctx.check(lib().soup_probe_read(ctx.p, _ptr(src), int(src.numel() * src.element_size()), _ptr(partial),
                                    int(partial.numel()), _stream(stream)))


def soup_probe_atomic(ctx: Ctx, slots, n_ops: int, stream=None):
    ctx.check(lib().soup_probe_atomic(ctx.p, _ptr(slots), int(slots.numel()), int(n_ops), _stream(stream)))


def soup_probe_fma(ctx: Ctx, out, iters: int, stream=None):
    ctx.check(lib().soup_probe_fma(ctx.p, _ptr(out), int(out.numel()), int(iters), _stream(stream)))


def soup_probe_mfma(ctx: Ctx, out, iters: int, stream=None):
    ctx.check(lib().soup_probe_mfma(ctx.p, _ptr(out), int(out.numel()), int(iters), _stream(stream)))
