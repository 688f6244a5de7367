"""Torch-facing API of the rasterizer: device-resident scenes and views, the
forward / backward calls and a torch.autograd.Function whose backward is the
library's adjoint kernel (fragments are recomputed from the saved
visibility buffer, never stored).

All arithmetic runs in libdiffsoup.so; this module only allocates outputs
with torch and marshals pointers.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib


@dataclasses.dataclass
class DeviceScene:
    verts: torch.Tensor        # [T,3,3] float32, cuda
    feats: torch.Tensor        # [T,G,G,C]
    mlp: torch.Tensor          # [n_params]
    dims: List[int]

    @staticmethod
    def from_host(scene, device="cuda") -> "DeviceScene":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return DeviceScene(t(scene.verts), t(scene.feats), t(scene.mlp), list(scene.dims))

    @property
    def T(self) -> int:
        return int(self.verts.shape[0])

    def n_params(self) -> int:
        d = self.dims
        return int(sum(o * i + o for i, o in zip(d[:-1], d[1:])))

    def c_struct(self, h: _lib._Holder, verts=None, feats=None, mlp=None) -> _lib.soup_scene:
        return _lib.make_scene(h, self.verts if verts is None else verts, self.feats if feats is None else feats,
                               self.mlp if mlp is None else mlp, self.dims)


@dataclasses.dataclass
class Views:
    widths: np.ndarray
    heights: np.ndarray
    view_ids: np.ndarray
    view_proj: np.ndarray      # [V,4,4] float32 (host)

    @staticmethod
    def from_list(views) -> "Views":
        return Views(np.array([v.width for v in views], np.int32), np.array([v.height for v in views], np.int32),
                     np.array([v.view_id for v in views], np.uint32),
                     np.stack([np.asarray(v.M, np.float32) for v in views]))

    @property
    def V(self) -> int:
        return int(len(self.widths))

    @property
    def pixels(self) -> int:
        return int((self.widths.astype(np.int64) * self.heights).sum())

    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.widths.astype(np.int64) * self.heights)])

    def c_struct(self, h: _lib._Holder) -> _lib.soup_views:
        return _lib.make_views(h, self.widths, self.heights, self.view_ids, self.view_proj)


@dataclasses.dataclass
class Opts:
    seed: int = 0
    step: int = 0
    mode: int = 0              # 0 stochastic masking, 1 threshold
    background: tuple = (0.0, 0.0, 0.0)
    edge_pairs: int = 0        # 0 all pairs, 1 id change, 2 none
    near_w: float = 0.1
    accumulate: int = 0        # backward: 1 = add into the gradient outputs
    reuse_bins: int = 0        # backward: 1 = reuse the last forward's setup and tile lists (same data)

    def c_struct(self) -> _lib.soup_opts:
        return _lib.make_opts(self.seed, self.step, self.mode, self.background, self.edge_pairs, self.near_w,
                              self.accumulate, self.reuse_bins)


_ctx_cache = {}


def context(device: Optional[int] = None) -> _lib.Ctx:
    if device is None:
        device = torch.cuda.current_device()
    c = _ctx_cache.get(device)
    if c is None:
        c = _ctx_cache[device] = _lib.Ctx(device)
    return c


def rasterize_fwd(scene: DeviceScene, views: Views, opts: Opts, want_logp: bool = False,
                  ctx: Optional[_lib.Ctx] = None, stream=None, out=None):
    """vis [P] int64 (uint64 bits), color [P,3], logp [P] or None.
    out: optional preallocated (vis, color, logp-or-None)."""
    ctx = ctx or context()
    dev = scene.verts.device
    P = views.pixels
    if out is not None:
        vis, color, logp = out
    else:
        vis = torch.empty(P, dtype=torch.int64, device=dev)
        color = torch.empty(P, 3, dtype=torch.float32, device=dev)
        logp = torch.empty(P, dtype=torch.float32, device=dev) if want_logp else None
    h = _lib._Holder()
    _lib.soup_rasterize_fwd(ctx, scene.c_struct(h), views.c_struct(h), opts.c_struct(), vis, color, logp, stream)
    return vis, color, logp


def rasterize_bwd(scene: DeviceScene, views: Views, opts: Opts, vis, color, grad_color, grad_logp=None,
                  ctx: Optional[_lib.Ctx] = None, stream=None, out=None):
    ctx = ctx or context()
    if out is None:
        gv = torch.empty_like(scene.verts)
        gf = torch.empty_like(scene.feats)
        gm = torch.empty_like(scene.mlp)
    else:
        gv, gf, gm = out
    h = _lib._Holder()
    _lib.soup_rasterize_bwd(ctx, scene.c_struct(h), views.c_struct(h), opts.c_struct(), vis, color,
                            grad_color.contiguous(), None if grad_logp is None else grad_logp.contiguous(),
                            gv, gf, gm, stream)
    return gv, gf, gm


def render(scenes: Sequence[DeviceScene], views: Views, opts: Opts, colors=None, ctx=None, stream=None):
    """Forward-only batched render: request r = scenes[r] seen from view r."""
    ctx = ctx or context()
    if colors is None:
        colors = [torch.empty(int(views.heights[r]), int(views.widths[r]), 3, dtype=torch.float32,
                              device=scenes[r].verts.device) for r in range(len(scenes))]
    h = _lib._Holder()
    _lib.soup_render(ctx, [s.c_struct(h) for s in scenes], views.c_struct(h), opts.c_struct(), colors, stream)
    return colors


def loss_l2(color, target, ctx=None, stream=None, out=None):
    """L = mean over P*3 of (color - target)^2: (loss [1], dL/dcolor [P,3],
    per-pixel score weights [P]). out: optional preallocated (loss, gc, gl)."""
    ctx = ctx or context()
    if out is not None:
        loss, gc, gl = out
    else:
        gc = torch.empty_like(color)
        gl = torch.empty(color.shape[0], dtype=torch.float32, device=color.device)
        loss = torch.empty(1, dtype=torch.float32, device=color.device)
    _lib.soup_loss_l2(ctx, color, target, gc, gl, loss, stream)
    return loss, gc, gl


class SoupRasterize(torch.autograd.Function):
    """(verts, feats, mlp) -> (color [P,3], logp [P]).

    The gradient of logp is the per-pixel weight of the score term: a loss
    written as L(color) + (L_pixel(color).detach() * logp).sum() reproduces
    the estimator of Eq. (8) (Algorithm A1's L * s). The visibility buffer
    is saved; the backward recomputes fragments from it."""

    @staticmethod
    def forward(fctx, verts, feats, mlp, dims, views: Views, opts: Opts):
        scene = DeviceScene(verts.contiguous(), feats.contiguous(), mlp.contiguous(), list(dims))
        # keep the tile lists and the log of decoded fragments for the backward
        vis, color, logp = rasterize_fwd(scene, views, dataclasses.replace(opts, reuse_bins=1),
                                         want_logp=opts.mode == 0)
        if logp is None:
            logp = torch.zeros(color.shape[0], dtype=torch.float32, device=color.device)
        fctx.save_for_backward(scene.verts, scene.feats, scene.mlp, vis, color)
        fctx.dims, fctx.views, fctx.opts = list(dims), views, opts
        fctx.mark_non_differentiable(vis)
        return color, logp, vis

    @staticmethod
    def backward(fctx, grad_color, grad_logp, _grad_vis):
        verts, feats, mlp, vis, color = fctx.saved_tensors
        scene = DeviceScene(verts, feats, mlp, fctx.dims)
        if grad_color is None:
            grad_color = torch.zeros_like(color)
        # autograd refuses a backward whose saved tensors were modified in
        # place, so the forward's setup and tile lists still describe these
        # vertices (the library rebuilds them if another call intervened)
        opts = dataclasses.replace(fctx.opts, reuse_bins=1)
        gv, gf, gm = rasterize_bwd(scene, fctx.views, opts, vis, color, grad_color, grad_logp)
        return gv, gf, gm, None, None, None


def rasterize(verts, feats, mlp, dims, views: Views, opts: Opts):
    """Differentiable rasterization: returns (color [P,3], logp [P], vis [P])."""
    return SoupRasterize.apply(verts, feats, mlp, dims, views, opts)


# ---------------------------------------------------------------------------
# Adaptive control of primitives (Section 3.4; Supplement B)

def coverage_count(vis, T: int, counts=None, ctx=None, stream=None):
    """Pixels won per triangle from visibility keys (any views of one scene),
    added into `counts` (uint32 [T] on the device; a fresh zeroed one by
    default)."""
    ctx = ctx or context()
    if counts is None:
        counts = torch.zeros(int(T), dtype=torch.int32, device=vis.device)
    _lib.soup_coverage_count(ctx, vis, T, counts, stream)
    return counts


def edge_lengths(verts, views: Views, near_w: float = 0.1, ctx=None, stream=None):
    """[T,3] float32: each edge's longest screen-space length over the views,
    in units of the view's height (0 where no view sees the triangle)."""
    ctx = ctx or context()
    rel = torch.empty(int(verts.shape[0]), 3, dtype=torch.float32, device=verts.device)
    h = _lib._Holder()
    _lib.soup_edge_lengths(ctx, verts, views.c_struct(h), near_w, rel, stream)
    return rel


def adaptive_plan(counts, rel_len, split_frac: float = 0.2, target: int = 0, prune_zero: bool = False,
                  fill: bool = False):
    """Host plan: (actions [T], offsets [T], n_new) as numpy int32 arrays."""
    flags = (_lib.PLAN_PRUNE_ZERO if prune_zero else 0) | (_lib.PLAN_FILL if fill else 0)
    if isinstance(counts, torch.Tensor):
        counts = counts.cpu().numpy().view(np.uint32)
    if isinstance(rel_len, torch.Tensor):
        rel_len = rel_len.cpu().numpy()
    return _lib.soup_adaptive_plan(counts, rel_len, split_frac, target, flags)


def adaptive_apply(scene: DeviceScene, actions, offsets, n_new: int, ctx=None, stream=None) -> DeviceScene:
    """The soup after a plan: kept triangles, halves of split ones (vertices
    and resampled textures); the MLP is shared with `scene`."""
    ctx = ctx or context()
    dev = scene.verts.device
    act = torch.as_tensor(np.ascontiguousarray(actions, np.int32)).to(dev)
    off = torch.as_tensor(np.ascontiguousarray(offsets, np.int32)).to(dev)
    G, Cc = int(scene.feats.shape[1]), int(scene.feats.shape[3])
    v = torch.empty(int(n_new), 3, 3, dtype=torch.float32, device=dev)
    f = torch.empty(int(n_new), G, G, Cc, dtype=torch.float32, device=dev)
    h = _lib._Holder()
    _lib.soup_adaptive_apply(ctx, scene.c_struct(h), act, off, n_new, v, f, stream)
    return DeviceScene(v, f, scene.mlp, list(scene.dims))


# ---------------------------------------------------------------------------
# Training step (Section 3.4 "Loss function"; Supplement, hyperparameters)

def loss_l1_ssim(color, target, views: Views, lam: float = 0.8, ctx=None, stream=None, out=None):
    """lam L1 + (1 - lam) D-SSIM over the views' images: (loss [1], dL/dcolor
    [P,3], per-pixel score weights [P] summing to the loss)."""
    ctx = ctx or context()
    if out is not None:
        loss, gc, gl = out
    else:
        gc = torch.empty_like(color)
        gl = torch.empty(color.shape[0], dtype=torch.float32, device=color.device)
        loss = torch.empty(1, dtype=torch.float32, device=color.device)
    h = _lib._Holder()
    _lib.soup_loss_l1_ssim(ctx, color, target, views.c_struct(h), lam, gc, gl, loss, stream)
    return loss, gc, gl


def adam_step(p, g, m, v, lr: float, t: int, vec: int = 1, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, ctx=None, stream=None):
    """In-place Adam (vec = 1) or VectorAdam (vec = 3) step t >= 1 on p, m, v
    (v holds one entry per vec-vector)."""
    ctx = ctx or context()
    _lib.soup_adam_step(ctx, p, g, m, v, vec, lr, beta1, beta2, eps, t, stream)


# ---------------------------------------------------------------------------
# Paper form (Section 3.3; Supplement B.3, B.6): mesh-colour texture, opacity
# outside the MLP, deferred shading

@dataclasses.dataclass
class PDeviceScene:
    verts: torch.Tensor        # [T,3,3] float32, cuda
    tex: torch.Tensor          # [T,V(R),8], activated
    mlp: torch.Tensor          # [595]
    R: int

    @staticmethod
    def from_host(ps, device="cuda") -> "PDeviceScene":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return PDeviceScene(t(ps.verts), t(ps.tex), t(ps.mlp), int(ps.R))

    @property
    def T(self) -> int:
        return int(self.verts.shape[0])

    def c_struct(self) -> _lib.soup_pscene:
        return _lib.make_pscene(self.verts, self.tex, self.mlp, self.R)


def inv_view_proj(views: Views) -> np.ndarray:
    """Per view the inverse of its view-projection, in float64 rounded once
    to float32 (the deferred shading's view directions)."""
    return np.linalg.inv(views.view_proj.astype(np.float64)).astype(np.float32)


def pforward(scene: PDeviceScene, views: Views, opts: Opts, minv=None, want_logp: bool = False, ctx=None,
             stream=None, out=None):
    """vis [P] int64, color [P,3], logp [P] or None (the paper form)."""
    ctx = ctx or context()
    dev = scene.verts.device
    P = views.pixels
    if out is not None:
        vis, color, logp = out
    else:
        vis = torch.empty(P, dtype=torch.int64, device=dev)
        color = torch.empty(P, 3, dtype=torch.float32, device=dev)
        logp = torch.empty(P, dtype=torch.float32, device=dev) if want_logp else None
    minv = inv_view_proj(views) if minv is None else minv
    h = _lib._Holder()
    _lib.soup_pforward(ctx, scene.c_struct(), views.c_struct(h), minv, opts.c_struct(), vis, color, logp, stream)
    return vis, color, logp


def pbackward(scene: PDeviceScene, views: Views, opts: Opts, vis, color, grad_color, grad_logp=None, minv=None,
              ctx=None, stream=None, out=None):
    """(d verts [T,3,3], d tex [T,V,8], d mlp [595]) of the paper form."""
    ctx = ctx or context()
    if out is None:
        gv = torch.empty_like(scene.verts)
        gt = torch.empty_like(scene.tex)
        gm = torch.empty_like(scene.mlp)
    else:
        gv, gt, gm = out
    minv = inv_view_proj(views) if minv is None else minv
    h = _lib._Holder()
    _lib.soup_pbackward(ctx, scene.c_struct(), views.c_struct(h), minv, opts.c_struct(), vis, color,
                        grad_color.contiguous(), None if grad_logp is None else grad_logp.contiguous(), gv, gt, gm,
                        stream)
    return gv, gt, gm


def pbackward_levels(scene: PDeviceScene, views: Views, opts: Opts, vis, color, grad_color, Rmin: int,
                     n_levels: int, grad_logp=None, minv=None, ctx=None, stream=None, out=None):
    """(d verts [T,3,3], [d level Rmin + l, [T,V,8], for l < n_levels], d mlp [595]) of the paper
    form, scene.tex being the assembly of those levels onto level scene.R."""
    ctx = ctx or context()
    T = scene.T
    if out is None:
        gv = torch.empty_like(scene.verts)
        gr = [torch.empty(T, mc_vertices(Rmin + l), 8, dtype=torch.float32, device=scene.tex.device)
              for l in range(n_levels)]
        gm = torch.empty_like(scene.mlp)
    else:
        gv, gr, gm = out
    minv = inv_view_proj(views) if minv is None else minv
    h = _lib._Holder()
    _lib.soup_pbackward_levels(ctx, scene.c_struct(), views.c_struct(h), minv, opts.c_struct(), vis, color,
                               grad_color.contiguous(), None if grad_logp is None else grad_logp.contiguous(), Rmin,
                               gv, gr, gm, stream)
    return gv, gr, gm


def mc_vertices(R: int) -> int:
    n = 1 << R
    return (n + 1) * (n + 2) // 2


def mc_assemble(raw: Sequence[torch.Tensor], Rmin: int, Rmax: int, out=None, ctx=None, stream=None):
    """tex [T,V(Rmax),8] = sigmoid(sum of the learnable levels Rmin.. sampled at the finest vertices)."""
    ctx = ctx or context()
    T = int(raw[0].shape[0])
    tex = out if out is not None else torch.empty(T, mc_vertices(Rmax), 8, dtype=torch.float32,
                                                  device=raw[0].device)
    _lib.soup_mc_assemble(ctx, [r.contiguous() for r in raw], Rmin, Rmax, tex, stream)
    return tex


def mc_assemble_bwd(tex, grad_tex, Rmin: int, n_levels: int, Rmax: int, out=None, accumulate: int = 0, ctx=None,
                    stream=None):
    ctx = ctx or context()
    T = int(tex.shape[0])
    if out is None:
        out = [torch.empty(T, mc_vertices(Rmin + l), 8, dtype=torch.float32, device=tex.device)
               for l in range(n_levels)]
    _lib.soup_mc_assemble_bwd(ctx, tex, grad_tex.contiguous(), Rmin, Rmax, out, accumulate, stream)
    return out
