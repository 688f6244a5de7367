"""GPU parity of the adaptive control of primitives (Section 3.4; Supplement
B) against the oracle: coverage counts bit-exact, screen-space edge lengths
to 1e-6 relative with identical split decisions, applied plans with
bit-exact vertices and resampled textures to 1e-6."""
import numpy as np
import pytest

from oracle import adaptive as A
from paper_2603_27151_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-adaptive]", *a, flush=True)


def _R():
    from paper_2603_27151_amd import raster as R
    return R


def _run_keys(rng, n, T, bg_frac=0.3, max_run=40, out_of_range=0.01):
    """Visibility keys in runs of equal winners, like image rows."""
    keys = np.empty(n, np.uint64)
    i = 0
    while i < n:
        r = int(rng.integers(1, max_run + 1))
        u = rng.random()
        if u < bg_frac:
            keys[i:i + r] = np.uint64(A.BG_KEY)
        else:
            t = int(rng.integers(T, T + 100)) if u > 1 - out_of_range else int(rng.integers(0, T))
            depth = rng.integers(0, 1 << 31, size=min(r, n - i)).astype(np.uint64)
            keys[i:i + r] = (depth << np.uint64(32)) | np.uint64(t)
        i += r
    return keys


@pytest.mark.parametrize("n,T", [(0, 5), (1, 3), (63, 7), (64, 1), (200_003, 5_000), (131_072, 1)])
def test_coverage_counts_match_the_oracle(n, T):
    _say("coverage", n, T)
    rng = np.random.default_rng(n + T)
    keys = _run_keys(rng, n, T)
    vis = torch.from_numpy(keys.view(np.int64)).cuda()
    c = _R().coverage_count(vis, T)
    torch.cuda.synchronize()
    ref = A.coverage_counts(keys, T)
    assert c.cpu().numpy().astype(np.int64).tolist() == ref.tolist()
    _R().coverage_count(vis, T, counts=c)          # adds into the counts
    assert c.cpu().numpy().astype(np.int64).tolist() == (2 * ref).tolist()


def test_coverage_counts_of_a_batched_forward():
    """The 64-view, 50k-triangle workload's visibility buffer (27.75 Mpixel):
    every covered pixel counted once, per triangle equal to a histogram of the
    keys' triangle indices."""
    R = _R()
    wl = W.batched(with_targets=False)
    _say("coverage batched", wl.pixels)
    sc = R.DeviceScene.from_host(wl.scene)
    views = R.Views.from_list(wl.views)
    vis, color, _ = R.rasterize_fwd(sc, views, R.Opts(seed=wl.seed), want_logp=False)
    c = R.coverage_count(vis, sc.T)
    keys = vis.cpu().numpy().view(np.uint64)
    ids = (keys[keys != np.uint64(A.BG_KEY)] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    got = c.cpu().numpy().astype(np.int64)
    assert got.sum() == ids.size
    assert np.array_equal(got, np.bincount(ids, minlength=sc.T))


def _views_for_lengths(rng, V):
    out = []
    eyes = W.fibonacci_sphere(V, 3.0)
    for v in range(V):
        w, h = [(256, 256), (320, 180), (97, 211), (1920, 1080)][v % 4]
        eye = eyes[v] if v % 5 else eyes[v] * 0.2      # every fifth camera sits inside the soup
        out.append(W.View(w, h, v, W.view_proj(eye, w, h)))
    return out


@pytest.mark.parametrize("T,V", [(1, 1), (1500, 40), (777, 32)])
def test_edge_lengths_match_the_oracle(T, V):
    _say("edge lengths", T, V)
    rng = np.random.default_rng(T * 100 + V)
    verts = W.equilateral_soup(rng, W.uniform_ball(rng, T), ) if T > 1 else \
        np.array([[[0, 0, 0], [0.3, 0, 0], [0, 0.3, 0]]], np.float32)
    verts = np.ascontiguousarray(verts, np.float32)
    views = _views_for_lengths(rng, V)
    R = _R()
    rel = R.edge_lengths(torch.from_numpy(verts).cuda(), R.Views.from_list(views), 0.1).cpu().numpy()
    ref = A.edge_lengths(verts, np.stack([v.M for v in views]), [v.width for v in views],
                         [v.height for v in views], 0.1)
    assert np.array_equal(rel == 0, ref == 0)
    np.testing.assert_allclose(rel, ref, rtol=1e-6, atol=0)
    assert np.array_equal(rel > np.float32(0.2), ref > np.float32(0.2))
    _say("exact", float(np.mean(rel == ref)))


@pytest.mark.parametrize("T,G,C,target,flags", [(700, 5, 3, 900, 0), (700, 8, 16, 500, 1),
                                                 (300, 8, 16, 600, 3), (64, 2, 1, 64, 0), (1, 4, 32, 2, 2)])
def test_apply_matches_the_oracle(T, G, C, target, flags):
    _say("apply", T, G, C, target, flags)
    rng = np.random.default_rng(T + G + C + target)
    verts = rng.standard_normal((T, 3, 3)).astype(np.float32)
    feats = rng.standard_normal((T, G, G, C)).astype(np.float32)
    counts = rng.integers(0, 6, size=T)
    rel = (rng.random((T, 3)) * 0.4).astype(np.float32)
    act, off, n = A.plan(counts, rel, 0.2, target, prune_zero=bool(flags & 1), fill=bool(flags & 2))
    R = _R()
    dims = [C, 4] if C != 16 else [16, 32, 32, 4]
    mlp = np.zeros(W.mlp_param_count(dims), np.float32)
    sc = R.DeviceScene(torch.from_numpy(verts).cuda(), torch.from_numpy(feats).cuda(),
                       torch.from_numpy(mlp).cuda(), dims)
    out = R.adaptive_apply(sc, act, off, n)
    torch.cuda.synchronize()
    ov, of = A.apply(verts, feats, act, off, n)
    assert out.T == n
    assert np.array_equal(out.verts.cpu().numpy(), ov)
    np.testing.assert_allclose(out.feats.cpu().numpy(), of, rtol=1e-6, atol=1e-6)


def test_apply_with_nothing_left():
    R = _R()
    verts = torch.zeros(3, 3, 3, device="cuda")
    feats = torch.zeros(3, 2, 2, 4, device="cuda")
    sc = R.DeviceScene(verts, feats, torch.zeros(W.mlp_param_count([4, 4]), device="cuda"), [4, 4])
    out = R.adaptive_apply(sc, np.zeros(3, np.int32), np.zeros(3, np.int32), 0)
    torch.cuda.synchronize()
    assert out.T == 0


def test_adaptive_round_trip_renders():
    """Measure, plan and rebuild a soup from a forward, then render the new soup."""
    R = _R()
    wl = W.single(with_targets=False, T=4000, res=400)
    sc = R.DeviceScene.from_host(wl.scene)
    views = R.Views.from_list(wl.views)
    vis, _, _ = R.rasterize_fwd(sc, views, R.Opts(seed=wl.seed), want_logp=False)
    counts = R.coverage_count(vis, sc.T)
    rel = R.edge_lengths(sc.verts, views, 0.1)
    act, off, n = R.adaptive_plan(counts, rel, 0.02, target=sc.T)
    assert n <= sc.T and (act >= 2).any() and (act == 0).any()
    new = R.adaptive_apply(sc, act, off, n)
    vis2, color2, _ = R.rasterize_fwd(new, views, R.Opts(seed=wl.seed), want_logp=False)
    torch.cuda.synchronize()
    assert torch.isfinite(color2).all()
    # the split halves cover what their parents covered: coverage is not lost wholesale
    assert int((vis2 != -1).sum()) > 0.9 * int((vis != -1).sum())


def test_adaptive_at_full_size_on_sampled_triangles():
    """The batched workload's soup (50,000 triangles, 8 x 8 x 16 textures):
    coverage over its 64 views, edge lengths over 20 of them, the plan of a
    random initialisation, and the applied soup, checked against the oracle
    on sampled triangles (edge lengths; each sampled source's outputs)."""
    R = _R()
    wl = W.batched(with_targets=False)
    sc = R.DeviceScene.from_host(wl.scene)
    views = R.Views.from_list(wl.views)
    vis, _, _ = R.rasterize_fwd(sc, views, R.Opts(seed=wl.seed), want_logp=False)
    counts = R.coverage_count(vis, sc.T)
    pick = np.sort(np.random.default_rng(20).choice(len(wl.views), size=20, replace=False))
    sample = [wl.views[i] for i in pick]
    rel = R.edge_lengths(sc.verts, R.Views.from_list(sample)).cpu().numpy()
    act, off, n = R.adaptive_plan(counts, rel, 0.2, target=sc.T, prune_zero=True, fill=True)
    assert n == sc.T
    new = R.adaptive_apply(sc, act, off, n)
    torch.cuda.synchronize()
    nv, nf = new.verts.cpu().numpy(), new.feats.cpu().numpy()
    rng = np.random.default_rng(21)
    split_ids = np.nonzero(act >= A.SPLIT0)[0]
    keep_ids = np.nonzero(act == A.KEEP)[0]
    ids = np.concatenate([rng.choice(split_ids, size=min(20, split_ids.size), replace=False),
                          rng.choice(keep_ids, size=20, replace=False)])
    _say("full size: splits", split_ids.size, "sampled", ids.size)
    ref_rel = A.edge_lengths(wl.scene.verts[ids], np.stack([v.M for v in sample]),
                             [v.width for v in sample], [v.height for v in sample], 0.1)
    np.testing.assert_allclose(rel[ids], ref_rel, rtol=1e-6, atol=0)
    for t in ids:
        kids = 2 if act[t] >= A.SPLIT0 else 1
        ov, of = A.apply(wl.scene.verts[t:t + 1], wl.scene.feats[t:t + 1], act[t:t + 1], np.zeros(1, np.int32), kids)
        o = int(off[t])
        assert np.array_equal(nv[o:o + kids], ov)
        np.testing.assert_allclose(nf[o:o + kids], of, rtol=1e-6, atol=1e-6)
