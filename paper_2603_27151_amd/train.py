"""Training loop around the rasterizer (Section 3.4; Supplement B, Algorithm
A1 and hyperparameters): each iteration renders a batch of views with
stochastic opacity masking, evaluates lambda L1 + (1 - lambda) D-SSIM on the
stochastic rendering, runs the backward (colour, score and edge terms) and
takes one optimiser step: VectorAdam for vertex positions, Adam for the
texture features and the MLP, with learning rates decaying exponentially to
1/100 over training. Every `adapt_every` iterations the adaptive control of
primitives runs (coverage over a batch of views, edge lengths over a sample
of views, plan, rebuild), and the optimiser state is reset for the rebuilt
soup (its moments belong to triangles that may no longer exist).

Every step runs in the library's kernels; this module only sequences calls.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import raster as R


@dataclasses.dataclass
class TrainConfig:
    iters: int = 10_000
    batch: int = 4                 # views per iteration
    lam: float = 0.8               # L1 weight
    lr_verts: float = 1e-3         # synthetic scenes; 1e-2 for real ones
    lr_feats: float = 5e-2
    lr_mlp: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    adapt_every: int = 0           # 0: no adaptive control
    split_frac: float = 0.2
    edge_views: int = 20
    target_tris: Optional[int] = None
    seed: int = 0x5EED


class Trainer:
    def __init__(self, scene: R.DeviceScene, views: Sequence, targets: Sequence[np.ndarray],
                 cfg: Optional[TrainConfig] = None, ctx=None):
        cfg = cfg or TrainConfig()
        self.cfg = cfg
        self.ctx = ctx or R.context()
        self.scene = scene
        self.views = list(views)
        dev = scene.verts.device
        self.targets = [torch.from_numpy(np.ascontiguousarray(t, np.float32).reshape(-1, 3)).to(dev)
                        for t in targets]
        self.target_tris = cfg.target_tris if cfg.target_tris is not None else scene.T
        self.t = 0
        self.rng = np.random.default_rng(cfg.seed)
        self._reset_state()

    def _reset_state(self):
        s = self.scene
        z = torch.zeros_like
        self.m = [z(s.verts), z(s.feats), z(s.mlp)]
        self.v = [torch.zeros(s.T * 3, dtype=torch.float32, device=s.verts.device), z(s.feats), z(s.mlp)]
        self.k = 0   # optimiser step count since the last reset

    def lr(self, lr0: float) -> float:
        n = self.cfg.iters
        return lr0 if n <= 1 else lr0 * math.pow(0.01, min(self.t, n - 1) / (n - 1))

    def step(self) -> float:
        cfg = self.cfg
        pick = self.rng.choice(len(self.views), size=min(cfg.batch, len(self.views)), replace=False)
        vs = R.Views.from_list([self.views[i] for i in pick])
        target = torch.cat([self.targets[i] for i in pick])
        opts = R.Opts(seed=cfg.seed, step=self.t)
        opts_b = R.Opts(seed=cfg.seed, step=self.t, reuse_bins=1)
        vis, color, _ = R.rasterize_fwd(self.scene, vs, opts, ctx=self.ctx)
        loss, gc, gl = R.loss_l1_ssim(color, target, vs, cfg.lam, ctx=self.ctx)
        gv, gf, gm = R.rasterize_bwd(self.scene, vs, opts_b, vis, color, gc, gl, ctx=self.ctx)
        self.k += 1
        s = self.scene
        R.adam_step(s.verts.view(-1), gv.view(-1), self.m[0].view(-1), self.v[0], self.lr(cfg.lr_verts), self.k,
                    vec=3, beta1=cfg.beta1, beta2=cfg.beta2, eps=cfg.eps, ctx=self.ctx)
        R.adam_step(s.feats.view(-1), gf.view(-1), self.m[1].view(-1), self.v[1].view(-1), self.lr(cfg.lr_feats),
                    self.k, beta1=cfg.beta1, beta2=cfg.beta2, eps=cfg.eps, ctx=self.ctx)
        R.adam_step(s.mlp, gm, self.m[2], self.v[2], self.lr(cfg.lr_mlp), self.k, beta1=cfg.beta1,
                    beta2=cfg.beta2, eps=cfg.eps, ctx=self.ctx)
        self.t += 1
        if cfg.adapt_every and self.t % cfg.adapt_every == 0:
            self.adapt()
        return float(loss.item())

    def adapt(self):
        """Coverage over one pass of all views, edge lengths over a sample of
        views, then prune and split to the triangle budget."""
        cfg = self.cfg
        s = self.scene
        counts = torch.zeros(s.T, dtype=torch.int32, device=s.verts.device)
        for i0 in range(0, len(self.views), max(1, cfg.batch)):
            vs = R.Views.from_list(self.views[i0:i0 + cfg.batch])
            vis, _, _ = R.rasterize_fwd(s, vs, R.Opts(seed=cfg.seed, step=self.t), ctx=self.ctx)
            R.coverage_count(vis, s.T, counts=counts, ctx=self.ctx)
        k = min(cfg.edge_views, len(self.views))
        sample = R.Views.from_list([self.views[i] for i in self.rng.choice(len(self.views), size=k, replace=False)])
        rel = R.edge_lengths(s.verts, sample, ctx=self.ctx)
        act, off, n = R.adaptive_plan(counts, rel, cfg.split_frac, target=self.target_tris)
        self.scene = R.adaptive_apply(s, act, off, n, ctx=self.ctx)
        self._reset_state()
        return act, n
