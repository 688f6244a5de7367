"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bar (tests/parity.py): visibility buffer bit-exact (triangle id and mask
draws); colours within 1e-5 relative; every gradient tensor within 1e-4
normwise (||gpu - oracle|| / ||oracle||) and element by element within
1e-4 |oracle_i| + 1e-6 max|oracle|.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_27151_amd import workloads as W
from tests import parity as PT
from tests import scenes as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


def _raster():
    from paper_2603_27151_amd import raster as R
    return R


def _dev_scene(scene):
    return _raster().DeviceScene.from_host(scene)


def _views(views):
    return _raster().Views.from_list(views)


def _opts(seed=0, step=0, mode=0, bg=(0.0, 0.0, 0.0), edge_pairs=0):
    return _raster().Opts(seed=seed, step=step, mode=mode, background=bg, edge_pairs=edge_pairs)


def _oopts(seed=0, step=0, mode=0, bg=(0.0, 0.0, 0.0), edge_pairs=0):
    return O.Opts(seed=seed, step=step, mode=mode, background=bg, edge_pairs=edge_pairs)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


normwise = PT.normwise


def assert_grads(gpu, ref, tol=1e-4, names=("verts", "feats", "mlp")):
    PT.assert_grads(gpu, ref, tol, names, tag="gpu-parity")


assert_colours = PT.assert_colours


def oracle_full(wl, opts_o, targets=True):
    """Oracle forward + L2-loss backward over all views (small configs)."""
    out = []
    P = wl.pixels
    gv = gf = gm = None
    for i, v in enumerate(wl.views):
        vis, col, logp, st = O.forward(wl.scene, v, opts_o)
        out.append((vis, col, logp, st))
    return out


def l2_grads(colors, targets, P):
    """dL/dcolor and the score weights of L = mean over P*3 of (c - t)^2."""
    gcs, gls = [], []
    for c, t in zip(colors, targets):
        d = c.astype(np.float32) - t
        gcs.append((2.0 * d / np.float32(3 * P)).astype(np.float32))
        gls.append(((d * d).sum(-1) / np.float32(3 * P)).astype(np.float32))
    return gcs, gls


# --------------------------------------------------------------------------
# contract pieces, bit for bit
# --------------------------------------------------------------------------

def test_sigmoid_bit_exact():
    R = _raster()
    ctx = R.context()
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 4, 200000), rng.uniform(-100, 100, 50000),
                        np.array([0.0, -0.0, 87.0, -87.0, 88.0, -88.0, 30.0, -30.0, 1e-30, -1e-30,
                                  np.inf, -np.inf, 17.328679, -17.328679])]).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    from paper_2603_27151_amd import _lib
    _lib.soup_selftest_sigmoid(ctx, xd, yd)
    y = yd.cpu().numpy()
    ref = np.array([O.sigmoid(float(v)) for v in x], np.float32)
    bad = np.flatnonzero(y.view(np.uint32) != ref.view(np.uint32))
    assert bad.size == 0, f"{bad.size} mismatches, first x={x[bad[0]]!r} gpu={y[bad[0]]!r} cpu={ref[bad[0]]!r}"


def test_uniform_bit_exact():
    R = _raster()
    ctx = R.context()
    rng = np.random.default_rng(1)
    n = 100000
    pix = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    tri = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    from paper_2603_27151_amd import _lib
    u = torch.empty(n, dtype=torch.float32, device="cuda")
    seed = 0x123456789ABCDEF0
    _lib.soup_selftest_uniform(ctx, seed, torch.from_numpy(pix.view(np.int32)).cuda(),
                               torch.from_numpy(tri.view(np.int32)).cuda(), 7, 3, u)
    got = u.cpu().numpy()
    ref = np.array([O.uniform(seed, int(p), int(t), 7, 3) for p, t in zip(pix[:20000], tri[:20000])], np.float32)
    assert np.array_equal(got[:20000], ref)


# --------------------------------------------------------------------------
# full-image parity on the small workloads
# --------------------------------------------------------------------------

def _fwd_bwd_case(wl, tile=16, mode=0, edge_pairs=0, bg=(0.0, 0.0, 0.0), check_bwd=True, logp=True):
    R = _raster()
    ctx = R.context()
    ctx.set_tile(tile)
    _say(f"case {wl.name} T={wl.scene.T} V={len(wl.views)} tile={tile} mode={mode} edge={edge_pairs}")
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    opts = _opts(wl.seed, wl.step, mode, bg, edge_pairs)
    oo = _oopts(wl.seed, wl.step, mode, bg, edge_pairs)
    vis, col, lp = R.rasterize_fwd(ds, vs, opts, want_logp=logp)
    torch.cuda.synchronize()
    vis = _u64(vis)
    col = col.cpu().numpy()
    off = vs.offsets()
    ref = [O.forward(wl.scene, v, oo) for v in wl.views]
    for i, v in enumerate(wl.views):
        a, b = off[i], off[i + 1]
        rv, rc, rl, _ = ref[i]
        gv = vis[a:b].reshape(v.height, v.width)
        mism = np.argwhere(gv != rv)
        assert mism.size == 0, f"view {i}: {len(mism)} visibility mismatches, first {mism[0]}"
        assert_colours(col[a:b].reshape(v.height, v.width, 3), rc)
        if logp:
            gl = lp.cpu().numpy()[a:b].reshape(v.height, v.width)
            if mode == 0:
                assert np.max(np.abs(gl - rl) / np.maximum(1.0, np.abs(rl))) < 1e-5
            else:
                assert np.all(gl == 0)
    if not check_bwd:
        return
    targets = wl.targets or [np.full((v.height, v.width, 3), 0.5, np.float32) for v in wl.views]
    gcs, gls = l2_grads([r[1] for r in ref], targets, vs.pixels)
    gc_d = torch.from_numpy(np.concatenate([g.reshape(-1, 3) for g in gcs])).cuda()
    gl_d = torch.from_numpy(np.concatenate([g.ravel() for g in gls])).cuda()
    gpu = R.rasterize_bwd(ds, vs, opts, torch.from_numpy(vis.view(np.int64)).cuda(),
                          torch.from_numpy(col).cuda(), gc_d, gl_d if mode == 0 else None)
    torch.cuda.synchronize()
    gpu = [g.cpu().numpy() for g in gpu]
    rv = np.zeros_like(gpu[0], np.float64)
    rf = np.zeros_like(gpu[1], np.float64)
    rm = np.zeros_like(gpu[2], np.float64)
    for i, v in enumerate(wl.views):
        a, b, c = O.backward(wl.scene, v, oo, ref[i][0], ref[i][1], gcs[i], gls[i] if mode == 0 else None)
        rv += a
        rf += b
        rm += c
    assert_grads(gpu, (rv, rf, rm))


def test_tiny_parity():
    _fwd_bwd_case(W.tiny())


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_single_view_parity(tile):
    _fwd_bwd_case(W.single(), tile=tile, check_bwd=(tile == 16))


def test_single_view_threshold_and_background():
    _fwd_bwd_case(W.single(), mode=1, bg=(0.2, 0.4, 0.6))


@pytest.mark.parametrize("edge_pairs", [1, 2])
def test_edge_pair_modes(edge_pairs):
    _fwd_bwd_case(W.tiny(), edge_pairs=edge_pairs)


def test_alpha_one_reduces_to_z_buffer():
    wl = W.tiny()
    wl.scene.mlp[-1] = 30.0          # opacity bias: sigmoid rounds to 1
    _fwd_bwd_case(wl)


def test_ragged_views_and_multiview():
    """Several views of odd sizes (ragged tiles) in one call."""
    wl = W.tiny()
    sizes = [(37, 23), (1, 1), (128, 3), (65, 130)]
    wl.views = [W.View(w, h, 10 + i, W.view_proj(W.fibonacci_sphere(4)[i], w, h)) for i, (w, h) in enumerate(sizes)]
    wl.targets = None
    for tile in (8, 16, 32):
        _fwd_bwd_case(wl, tile=tile, check_bwd=(tile == 16))


def test_tile_list_longer_than_sort_block():
    """3000 large triangles cover every pixel of a 32x32 view, so every tile
    list is longer than one sort block (lists are sorted block by block) and,
    with a low opacity, every pixel walks deep into its list."""
    wl = W.tiny()
    rng = np.random.default_rng(2048)
    T = 3000
    centres = W.uniform_ball(rng, T, 0.5)
    ang = rng.uniform(0.0, 2.0 * np.pi, T)[:, None] + np.array([0.0, 2.0 * np.pi / 3.0, 4.0 * np.pi / 3.0])
    verts = np.stack([4.0 * np.cos(ang), 4.0 * np.sin(ang), rng.uniform(-0.2, 0.2, (T, 3))], axis=2)
    verts = (verts + centres[:, None, :]).astype(np.float32)
    wl.scene = W.random_scene(rng, verts, 4, 8, [8, 16, 4])
    wl.scene.mlp[-1] = -3.0          # opacity bias: about one fragment in twenty passes
    wl.views = [W.View(32, 32, 3, W.view_proj((0.0, 0.0, 3.0), 32, 32))]
    wl.targets = None
    for tile in (8, 16, 32):
        _fwd_bwd_case(wl, tile=tile, check_bwd=(tile == 16))


@pytest.mark.parametrize("T", [63, 64, 65, 127, 128, 129, 255, 256, 257])
def test_tile_lists_at_the_wave_sort_sizes(T):
    """T large triangles cover every pixel of a 32x32 view, so every tile list
    holds exactly T entries: the sizes around the one-wave sorts' 64, 128 and
    256 entries and the workgroup sort past them. With a low opacity every pixel
    walks deep into its list, and its early exit trusts the sorted order."""
    wl = W.tiny()
    rng = np.random.default_rng(4000 + T)
    centres = W.uniform_ball(rng, T, 0.5)
    ang = rng.uniform(0.0, 2.0 * np.pi, T)[:, None] + np.array([0.0, 2.0 * np.pi / 3.0, 4.0 * np.pi / 3.0])
    verts = np.stack([4.0 * np.cos(ang), 4.0 * np.sin(ang), rng.uniform(-0.2, 0.2, (T, 3))], axis=2)
    verts = (verts + centres[:, None, :]).astype(np.float32)
    wl.scene = W.random_scene(rng, verts, 4, 8, [8, 16, 4])
    wl.scene.mlp[-1] = -3.0          # opacity bias: about one fragment in twenty passes
    wl.views = [W.View(32, 32, 5, W.view_proj((0.0, 0.0, 3.0), 32, 32))]
    wl.targets = None
    _fwd_bwd_case(wl, tile=16, check_bwd=(T in (64, 257)))


def test_empty_and_culled_scenes():
    R = _raster()
    wl = W.tiny()
    # everything behind the camera: all culled
    wl.scene.verts = (wl.scene.verts + np.float32(10.0)).astype(np.float32)
    _fwd_bwd_case(wl)
    # zero triangles
    wl0 = W.tiny()
    wl0.scene = W.Scene(np.zeros((0, 3, 3), np.float32), np.zeros((0, 4, 4, 8), np.float32), wl0.scene.mlp,
                        wl0.scene.dims)
    ds = _dev_scene(wl0.scene)
    vs = _views(wl0.views)
    vis, col, _ = R.rasterize_fwd(ds, vs, _opts(1, 0, 0, (0.1, 0.2, 0.3)))
    assert np.all(_u64(vis) == np.uint64(0xFFFFFFFFFFFFFFFF))
    assert np.allclose(col.cpu().numpy(), [0.1, 0.2, 0.3])


def test_invalid_arguments_are_rejected():
    R = _raster()
    from paper_2603_27151_amd import _lib
    wl = W.tiny()
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    with pytest.raises(_lib.SoupError, match="UNSUPPORTED"):
        bad = R.DeviceScene(ds.verts, ds.feats, ds.mlp, [8, 24, 4])
        R.rasterize_fwd(bad, vs, _opts())
    with pytest.raises(_lib.SoupError, match="INVALID"):
        R.rasterize_fwd(ds, vs, _opts(mode=3))
    with pytest.raises(_lib.SoupError, match="INVALID"):
        R.context().set_tile(12)
    # a texture grid whose backward gradient grid would not fit one workgroup's LDS
    # (11 x 11 x 32 floats per wave with the 32->64->64->4 MLP) is refused, not launched
    rng = np.random.default_rng(3)
    big = W.random_scene(rng, wl.scene.verts, 11, 32, [32, 64, 64, 4])
    dsb = _dev_scene(big)
    vis, col, _ = R.rasterize_fwd(dsb, vs, _opts())
    gc = torch.zeros_like(col)
    with pytest.raises(_lib.SoupError, match="UNSUPPORTED"):
        R.rasterize_bwd(dsb, vs, _opts(), vis, col, gc, None)


def test_batching_invariance():
    """A view rendered alone, or inside a batch in any order, gives the same
    visibility buffer (the draws depend on view_id, not batch position)."""
    R = _raster()
    wl = W.batched(with_targets=False, n_views=6, T=20000)
    ds = _dev_scene(wl.scene)
    opts = _opts(wl.seed)
    alone = []
    for v in wl.views:
        vis, _, _ = R.rasterize_fwd(ds, _views([v]), opts)
        alone.append(_u64(vis))
    perm = [3, 0, 5, 1, 4, 2]
    vs = _views([wl.views[i] for i in perm])
    vis, _, _ = R.rasterize_fwd(ds, vs, opts)
    vis = _u64(vis)
    off = vs.offsets()
    for k, i in enumerate(perm):
        assert np.array_equal(vis[off[k]:off[k + 1]], alone[i])


# --------------------------------------------------------------------------
# full-size workloads: sampled outputs
# --------------------------------------------------------------------------

def _sampled_case(wl, n_pix=300, tile=16, seed=0, check_bwd=True):
    R = _raster()
    ctx = R.context()
    ctx.set_tile(tile)
    _say(f"sampled {wl.name} T={wl.scene.T} V={len(wl.views)} P={wl.pixels} tile={tile}")
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    opts = _opts(wl.seed, wl.step)
    oo = _oopts(wl.seed, wl.step)
    vis_d, col_d, lp_d = R.rasterize_fwd(ds, vs, opts, want_logp=True)
    torch.cuda.synchronize()
    vis = _u64(vis_d)
    col = col_d.cpu().numpy()
    lp = lp_d.cpu().numpy()
    off = vs.offsets()
    rng = np.random.default_rng(seed)
    views_pick = rng.choice(len(wl.views), min(4, len(wl.views)), replace=False)
    sparse_c = np.zeros((vs.pixels, 3), np.float32)
    sparse_l = np.zeros(vs.pixels, np.float32)
    ref_grads = None
    for vi in views_pick:
        v = wl.views[vi]
        # sample covered pixels preferentially
        a = off[vi]
        cov = np.flatnonzero(vis[a:a + v.width * v.height] != np.uint64(0xFFFFFFFFFFFFFFFF))
        pick = rng.choice(cov, min(n_pix, cov.size), replace=False) if cov.size else np.array([], np.int64)
        pick = np.unique(np.concatenate([pick, rng.integers(0, v.width * v.height, 20)]))
        xy = np.stack([pick % v.width, pick // v.width], 1).astype(np.int32)
        rv, rc, rl = O.forward_pixels(wl.scene, v, oo, xy)
        assert np.array_equal(vis[a + pick], rv), f"view {vi}: visibility mismatch"
        assert_colours(col[a + pick], rc)
        assert np.max(np.abs(lp[a + pick] - rl) / np.maximum(1.0, np.abs(rl))) < 1e-5
        if check_bwd:
            gc = rng.normal(0, 1e-3, (len(pick), 3)).astype(np.float32)
            gl = rng.normal(0, 1e-3, len(pick)).astype(np.float32)
            sparse_c[a + pick] = gc
            sparse_l[a + pick] = gl
            g = O.backward_pixels(wl.scene, v, oo, xy, gc, gl)
            ref_grads = g if ref_grads is None else tuple(x + y for x, y in zip(ref_grads, g))
    if not check_bwd:
        return
    gpu = R.rasterize_bwd(ds, vs, opts, vis_d, col_d, torch.from_numpy(sparse_c).cuda(),
                          torch.from_numpy(sparse_l).cuda())
    torch.cuda.synchronize()
    assert_grads([g.cpu().numpy() for g in gpu], ref_grads)


@pytest.mark.slow
def test_batched_full_size_sampled():
    _sampled_case(W.batched(with_targets=False))


@pytest.mark.slow
def test_large_full_size_sampled():
    _sampled_case(W.large(with_targets=False), n_pix=150)


# --------------------------------------------------------------------------
# serving render and autograd plumbing
# --------------------------------------------------------------------------

def test_render_matches_oracle_threshold():
    R = _raster()
    rng = np.random.default_rng(3)
    scenes = [W.single(with_targets=False, T=t).scene for t in (3000, 6000)]
    vlist = [W.View(160, 90, 0, W.view_proj((0.0, 0.5, 3.0), 160, 90)),
             W.View(96, 96, 1, W.view_proj((1.0, -2.0, 2.0), 96, 96)),
             W.View(64, 36, 2, W.view_proj((-3.0, 0.0, 0.2), 64, 36))]
    which = [0, 1, 0]
    ds = [_dev_scene(s) for s in scenes]
    opts = _opts(mode=1, bg=(0.1, 0.1, 0.1))
    outs = R.render([ds[w] for w in which], _views(vlist), opts)
    torch.cuda.synchronize()
    for r, (w, v) in enumerate(zip(which, vlist)):
        _, rc, _, _ = O.forward(scenes[w], v, _oopts(mode=1, bg=(0.1, 0.1, 0.1)))
        assert np.array_equal(outs[r].cpu().numpy(), rc)


def test_autograd_function_matches_direct_calls():
    R = _raster()
    wl = W.tiny()
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    opts = _opts(wl.seed)
    verts = ds.verts.clone().requires_grad_(True)
    feats = ds.feats.clone().requires_grad_(True)
    mlp = ds.mlp.clone().requires_grad_(True)
    color, logp, vis = R.rasterize(verts, feats, mlp, ds.dims, vs, opts)
    target = torch.from_numpy(wl.targets[0].reshape(-1, 3)).cuda()
    per_pix = ((color - target) ** 2).sum(-1) / (3 * color.shape[0])
    loss = per_pix.sum() + (per_pix.detach() * logp).sum()
    loss.backward()
    loss_d, gc, gl = R.loss_l2(color.detach(), target)
    gv, gf, gm = R.rasterize_bwd(ds, vs, opts, vis, color.detach(), gc, gl)
    for a, b in ((verts.grad, gv), (feats.grad, gf), (mlp.grad, gm)):
        assert normwise(a.cpu().numpy(), b.cpu().numpy()) < 1e-5
    assert abs(float(loss_d) - float(per_pix.sum())) < 1e-6


def test_backward_reuses_forward_bins_only_when_valid():
    """reuse_bins=1 gives the gradients of a rebuilding backward; when another
    call on the context rebinned other views in between, the library
    rebuilds instead of reusing."""
    R = _raster()
    from paper_2603_27151_amd import _lib
    wl = W.batched(with_targets=True, n_views=4, T=20000)
    _say("case: batched 4 views, 20000 triangles, reuse_bins")
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    other = _views(W.batched(with_targets=False, n_views=2, T=20000).views)
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    ctx = _lib.Ctx(0)
    o = _opts(wl.seed)
    o_r = R.Opts(seed=wl.seed, reuse_bins=1)
    vis, col, _ = R.rasterize_fwd(ds, vs, o, ctx=ctx)
    _, gc, gl = R.loss_l2(col, target, ctx=ctx)
    ref = R.rasterize_bwd(ds, vs, o, vis, col, gc, gl, ctx=ctx)
    R.rasterize_fwd(ds, vs, o, ctx=ctx)
    got = R.rasterize_bwd(ds, vs, o_r, vis, col, gc, gl, ctx=ctx)
    R.rasterize_fwd(ds, other, o, ctx=ctx)          # rebins other views
    got2 = R.rasterize_bwd(ds, vs, o_r, vis, col, gc, gl, ctx=ctx)
    torch.cuda.synchronize()
    for a, b, c in zip(ref, got, got2):
        assert normwise(b.cpu().numpy(), a.cpu().numpy()) < 1e-5
        assert normwise(c.cpu().numpy(), a.cpu().numpy()) < 1e-5
    ctx.close()


def test_backward_from_forward_log_matches_replay():
    """A forward that keeps its fragment log (reuse_bins=1) lets the backward
    filter the log instead of replaying coverage: same gradients, same log p."""
    R = _raster()
    from paper_2603_27151_amd import _lib
    wl = W.batched(with_targets=True, n_views=4, T=20000)
    _say("case: batched 4 views, 20000 triangles, backward from the forward's log")
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).cuda()
    ctx = _lib.Ctx(0)
    o = _opts(wl.seed)
    o_k = R.Opts(seed=wl.seed, reuse_bins=1)
    vis, col, lp = R.rasterize_fwd(ds, vs, o, want_logp=True, ctx=ctx)
    _, gc, gl = R.loss_l2(col, target, ctx=ctx)
    ref = R.rasterize_bwd(ds, vs, o, vis, col, gc, gl, ctx=ctx)
    vis2, col2, lp2 = R.rasterize_fwd(ds, vs, o_k, want_logp=True, ctx=ctx)
    got = R.rasterize_bwd(ds, vs, o_k, vis2, col2, gc, gl, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(vis, vis2) and torch.equal(col, col2)
    assert normwise(lp2.cpu().numpy(), lp.cpu().numpy()) < 1e-6
    for a, b in zip(ref, got):
        assert normwise(b.cpu().numpy(), a.cpu().numpy()) < 1e-5
    ctx.close()


@pytest.mark.parametrize("from_log", [False, True])
def test_partial_upstream_gradients(from_log):
    """Upstream gradients that vanish on parts of the image: no colour gradient
    on the left half, no score weight on a checkerboard. Winners are then kept
    with or without any gradient (from the forward's log) or only with one
    (replay); either way the gradients match the oracle's."""
    R = _raster()
    from paper_2603_27151_amd import _lib
    wl = W.single(T=3000, res=400)
    _say(f"case: single view 400x400, 3000 triangles, partial upstream gradients, from_log={from_log}")
    ds = _dev_scene(wl.scene)
    vs = _views(wl.views)
    oo = _oopts(wl.seed, wl.step)
    o = R.Opts(seed=wl.seed, step=wl.step, reuse_bins=1 if from_log else 0)
    ctx = _lib.Ctx(0)
    vis, col, _ = R.rasterize_fwd(ds, vs, o, ctx=ctx)
    torch.cuda.synchronize()
    v = wl.views[0]
    ref = O.forward(wl.scene, v, oo)
    assert np.array_equal(_u64(vis).reshape(v.height, v.width), ref[0])
    gcs, gls = l2_grads([ref[1]], wl.targets, vs.pixels)
    gc, gl = gcs[0].copy(), gls[0].copy()
    gc[:, : v.width // 2] = 0.0
    yy, xx = np.mgrid[0 : v.height, 0 : v.width]
    gl[((yy // 8) + (xx // 8)) % 2 == 0] = 0.0
    gpu = R.rasterize_bwd(ds, vs, o, vis, col, torch.from_numpy(gc.reshape(-1, 3)).cuda(),
                          torch.from_numpy(gl.ravel()).cuda(), ctx=ctx)
    torch.cuda.synchronize()
    gpu = [g.cpu().numpy() for g in gpu]
    rv, rf, rm = O.backward(wl.scene, v, oo, ref[0], ref[1], gc, gl)
    assert_grads(gpu, (rv, rf, rm))
    ctx.close()


@pytest.mark.parametrize("P,offset", [(1001, 0), (4096, 1), (7, 0)])
def test_loss_l2_vector_and_tail_paths(P, offset):
    """The L2 loss kernel (16-byte path plus scalar tail; scalar throughout for
    unaligned buffers) against the float64 definition."""
    R = _raster()
    g = torch.Generator().manual_seed(P)
    base_c = torch.rand(P + offset, 3, generator=g).cuda()
    base_t = torch.rand(P + offset, 3, generator=g).cuda()
    col, tgt = base_c[offset:], base_t[offset:]
    _say(f"case: loss P={P} offset={offset}")
    loss, gc, gl = R.loss_l2(col, tgt)
    torch.cuda.synchronize()
    c64, t64 = col.double().cpu(), tgt.double().cpu()
    d = c64 - t64
    ref_gc = 2.0 * d / (3.0 * P)
    ref_gl = (d * d).sum(-1) / (3.0 * P)
    assert torch.allclose(gc.double().cpu(), ref_gc, rtol=1e-6, atol=1e-12)
    assert torch.allclose(gl.double().cpu(), ref_gl, rtol=1e-6, atol=1e-12)
    assert abs(float(loss) - float(ref_gl.sum())) <= 1e-6 * float(ref_gl.sum())
