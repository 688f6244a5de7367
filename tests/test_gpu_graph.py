"""Static-capacity mode: a whole fwd -> loss -> bwd step captured into one
HIP graph (torch.cuda.graph) and replayed, against the same step run
eagerly; and the overflow report of a static-mode call whose lists outgrow
the workspaces sized before (the lists are bounded on the device, so the
call completes and only flags the overflow)."""
import sys

import numpy as np
import pytest

from paper_2603_27151_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-graph]", *a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    d = float(torch.linalg.norm(b))
    return float(torch.linalg.norm(a - b)) / (d if d > 0 else 1.0)


class _Step:
    """fwd -> L2 loss -> bwd into preallocated buffers on one stream."""

    def __init__(self, R, ctx, ds, vs, opts, target):
        self.R, self.ctx, self.ds, self.vs, self.opts, self.target = R, ctx, ds, vs, opts, target
        P = vs.pixels
        dev = ds.verts.device
        self.vis = torch.empty(P, dtype=torch.int64, device=dev)
        self.col = torch.empty(P, 3, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.gc = torch.empty(P, 3, dtype=torch.float32, device=dev)
        self.gl = torch.empty(P, dtype=torch.float32, device=dev)
        self.gv = torch.empty_like(ds.verts)
        self.gf = torch.empty_like(ds.feats)
        self.gm = torch.empty_like(ds.mlp)

    def __call__(self):
        R = self.R
        R.rasterize_fwd(self.ds, self.vs, self.opts, ctx=self.ctx, out=(self.vis, self.col, None))
        R.loss_l2(self.col, self.target, ctx=self.ctx, out=(self.loss, self.gc, self.gl))
        R.rasterize_bwd(self.ds, self.vs, self.opts, self.vis, self.col, self.gc, self.gl, ctx=self.ctx,
                        out=(self.gv, self.gf, self.gm))

    def snapshot(self):
        return [t.clone() for t in (self.vis, self.col, self.loss, self.gv, self.gf, self.gm)]


@pytest.mark.parametrize("tile,reuse", [(8, 0), (16, 0), (16, 1)])
def test_graph_replay_matches_eager(tile, reuse):
    from paper_2603_27151_amd import _lib
    from paper_2603_27151_amd import raster as R
    wl = W.batched(with_targets=True, n_views=6, T=20000)
    _say(f"case: batched 6 views, 20000 triangles, tile {tile}, reuse_bins {reuse}")
    ds = R.DeviceScene.from_host(wl.scene)
    vs = R.Views.from_list(wl.views)
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    ctx = _lib.Ctx(0)
    ctx.set_tile(tile)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # reuse = 1: the forward keeps its tile lists and fragment log for the backward
        step = _Step(R, ctx, ds, vs, R.Opts(seed=wl.seed, step=wl.step, reuse_bins=reuse), target)
        step()   # eager: sizes every workspace
        step()
        torch.cuda.synchronize()
        ref = step.snapshot()
        ctx.set_static(True)
        step()   # static mode, not captured
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ctx.check_overflow()
    got = step.snapshot()
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        for t in (step.vis, step.col, step.gv, step.gf, step.gm):
            t.fill_(float("nan") if t.is_floating_point() else -7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ctx.check_overflow()
        got = step.snapshot()
        _say(f"replay {rep}: grads rel {_rel(got[3], ref[3]):.2e} {_rel(got[4], ref[4]):.2e} {_rel(got[5], ref[5]):.2e}")
        assert torch.equal(got[0], ref[0]), "visibility differs from the eager step"
        assert torch.equal(got[1], ref[1]), "colours differ from the eager step"
        assert _rel(got[2], ref[2]) < 1e-5   # the loss is a float-atomic sum over all pixels
        for k in (3, 4, 5):   # gradient sums: float atomics, order may differ
            assert _rel(got[k], ref[k]) < 1e-5
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        float((x * x).sum())
    ctx.set_static(False)
    ctx.close()


def test_static_overflow_is_flagged_not_fatal():
    from paper_2603_27151_amd import _lib
    from paper_2603_27151_amd import raster as R
    wl = W.batched(with_targets=True, n_views=4, T=20000)
    _say("case: batched 4 views, 20000 triangles; static call with larger triangles")
    ds = R.DeviceScene.from_host(wl.scene)
    vs = R.Views.from_list(wl.views)
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    ctx = _lib.Ctx(0)
    step = _Step(R, ctx, ds, vs, R.Opts(seed=wl.seed, step=wl.step), target)
    step()
    torch.cuda.synchronize()
    ctx.set_static(True)
    # same buffers (same descriptors), triangles scaled 4x about their centres:
    # about 16x the tile-list entries the workspaces were sized for
    c = ds.verts.mean(dim=1, keepdim=True)
    ds.verts.copy_(c + 4.0 * (ds.verts - c))
    step()
    torch.cuda.synchronize()
    with pytest.raises(_lib.SoupError, match="overflowed"):
        ctx.check_overflow()
    ctx.check_overflow()   # the flag was cleared
    ctx.set_static(False)
    step()                 # eager again: grows the workspaces, no error
    torch.cuda.synchronize()
    ctx.close()
