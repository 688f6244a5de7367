"""The timed step itself against the oracle, and the step's work counts.

* The benchmark's own step object (bench.Step: forward keeping its tile
  lists and fragment log, L2 loss, backward from that log) on the full
  batched workload (50,000 triangles, 64 views, 27.75 Mpixel), run the way
  the benchmark times it: static-capacity mode, captured once into a HIP
  graph and replayed. Every pixel's visibility and colour and every element
  of every gradient tensor is compared with the oracle's full-image forward
  and backward of the same views, fed the step's own upstream gradients.
* The counts the benchmark reports (covered pixels, winners, the backward's
  decodes E) equal the oracle's exactly.
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_27151_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BG = np.uint64(0xFFFFFFFFFFFFFFFF)


def _say(*a):
    PT.say("gpu-step", *a)


def _bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    return bench


@pytest.mark.parametrize("name", ["tiny", "single"])
def test_counts_match_oracle(name):
    """Covered pixels (forward), winners (visibility buffer) and the
    backward's decodes E (winner + every fragment in front of it; every
    fragment of a background pixel) against the oracle's statistics."""
    from paper_2603_27151_amd import _lib
    from paper_2603_27151_amd import raster as R
    wl = W.by_name(name)
    _say(f"case: counts {name}")
    ds = R.DeviceScene.from_host(wl.scene)
    vs = R.Views.from_list(wl.views)
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    ctx = _lib.Ctx(0)
    ctx.set_counting(True)
    for reuse in (0, 1):
        o = R.Opts(seed=wl.seed, step=wl.step, reuse_bins=reuse)
        vis, col, _ = R.rasterize_fwd(ds, vs, o, ctx=ctx)
        st_f = ctx.stats()
        _, gc, gl = R.loss_l2(col, target, ctx=ctx)
        R.rasterize_bwd(ds, vs, o, vis, col, gc, gl, ctx=ctx)
        st_b = ctx.stats()
        torch.cuda.synchronize()
        ref = [O.forward(wl.scene, v, O.Opts(seed=wl.seed, step=wl.step), want_logp=False)[3] for v in wl.views]
        cov = sum(r["covered_pixels"] for r in ref)
        win = sum(r["winners"] for r in ref)
        dec = sum(r["decodes"] for r in ref)
        assert int(gl.ne(0).sum()) == vs.pixels        # every pixel carries a score weight
        _say(f"reuse {reuse}: covered {st_f['covered_pixels']}/{cov} winners {int((vis != -1).sum())}/{win} "
             f"E {st_b['decodes']}/{dec}")
        assert st_f["covered_pixels"] == cov
        assert int((vis != -1).sum()) == win
        assert st_b["decodes"] == dec
        assert st_b["covered_pixels"] == -1
    ctx.close()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_bench_step_full_size_matches_oracle():
    from paper_2603_27151_amd import _lib
    from paper_2603_27151_amd import raster as R
    bench = _bench()
    wl = W.batched()
    _say(f"case: bench step, batched T={wl.scene.T} V={len(wl.views)} P={wl.pixels}, tile 16, static + graph")
    ds = R.DeviceScene.from_host(wl.scene)
    vs = R.Views.from_list(wl.views)
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    ctx = _lib.Ctx(0)
    ctx.set_tile(16)
    step = bench.Step(R, ctx, ds, vs, target, wl.seed, wl.step)
    step()
    step()
    torch.cuda.synchronize()
    g = step.capture(_say)
    for rep in range(2):
        for t in (step.vis, step.color, step.gc, step.gl, step.gv, step.gf, step.gm):
            t.fill_(float("nan") if t.is_floating_point() else -7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ctx.check_overflow()
    ctx.set_static(False)
    vis = step.vis.cpu().numpy().view(np.uint64)
    col = step.color.cpu().numpy()
    gc = step.gc.cpu().numpy()
    gl = step.gl.cpu().numpy()
    gpu = [step.gv.cpu().numpy(), step.gf.cpu().numpy(), step.gm.cpu().numpy()]
    del g
    ctx.close()
    _say("gpu step done; oracle over every view")
    oo = O.Opts(seed=wl.seed, step=wl.step)
    sc = wl.scene
    rv = np.zeros(sc.verts.shape, np.float64)
    rf = np.zeros(sc.feats.shape, np.float64)
    rm = np.zeros(sc.mlp.shape, np.float64)
    off = vs.offsets()
    t0 = time.perf_counter()
    n_win = 0
    for i, v in enumerate(wl.views):
        a, b = int(off[i]), int(off[i + 1])
        r_vis, r_col, _, st = O.forward(sc, v, oo, want_logp=False)
        mism = np.flatnonzero(vis[a:b] != r_vis.ravel())
        assert mism.size == 0, f"view {i}: {mism.size} visibility mismatches, first pixel {mism[0]}"
        PT.assert_colours(col[a:b], r_col.reshape(-1, 3))
        n_win += st["winners"]
        O.backward(sc, v, oo, r_vis, r_col, gc[a:b], gl[a:b], out=(rv, rf, rm))
        if i % 8 == 7:
            _say(f"oracle views {i + 1}/{len(wl.views)} in {time.perf_counter() - t0:.1f} s")
    assert int((vis != BG).sum()) == n_win
    PT.assert_grads(gpu, (rv, rf, rm), tag="gpu-step")
