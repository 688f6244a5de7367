"""GPU parity of the paper form (Section 3.3: mesh-colour texture, opacity
outside the MLP, deferred shading; Supplement B.3, B.6) against the oracle,
through the C ABI: texture assembly and its gradient, the forward (visibility
bit-exact, colours and log p), the backward (score term, colour path, edge
term), ragged and degenerate views, and the paper-form training step at full
size on sampled pixels. The bar is that of tests/parity.py."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_27151_amd import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    PT.say("gpu-paper", *a)


def _R():
    from paper_2603_27151_amd import raster as R
    return R


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _soup(seed, T, R=3, ball=1.0):
    rng = np.random.default_rng(seed)
    verts = W.equilateral_soup(rng, W.uniform_ball(rng, T, ball))
    return W.random_pscene(rng, verts, R)


# the staged forward takes four triangles per workgroup for small levels, two
# for (3, 5, 5), one for (1, 5, 5); (6, 6, 7) does not fit and gathers
@pytest.mark.parametrize("Rmin,Rtop,Rmax", [(0, 0, 0), (0, 1, 2), (2, 4, 5), (1, 5, 5), (3, 5, 5), (3, 3, 6),
                                            (6, 6, 7)])
def test_assembly_matches_oracle(Rmin, Rtop, Rmax):
    _say("assembly", Rmin, Rtop, Rmax)
    R = _R()
    rng = np.random.default_rng(10 * Rmin + Rtop + Rmax)
    T = 37
    lv = W.random_levels(rng, T, Rmin, Rtop, Rmax, sd=1.0)
    raw = [torch.from_numpy(r).cuda() for r in lv.raw]
    tex = R.mc_assemble(raw, Rmin, Rmax)
    torch.cuda.synchronize()
    ref = O.mc_assemble(lv.raw, Rmin, Rmax)
    # the same float32 operations in the same order: bit for bit
    assert np.array_equal(tex.cpu().numpy(), ref)
    gt = rng.normal(size=ref.shape).astype(np.float32)
    g = R.mc_assemble_bwd(tex, torch.from_numpy(gt).cuda(), Rmin, len(raw), Rmax)
    g2 = R.mc_assemble_bwd(tex, torch.from_numpy(gt).cuda(), Rmin, len(raw), Rmax, out=[x.clone() for x in g],
                           accumulate=1)
    torch.cuda.synchronize()
    gref = O.mc_assemble_bwd(ref, gt, Rmin, len(raw), Rmax)
    PT.assert_grads([x.cpu().numpy() for x in g], gref, names=[f"level{Rmin + l}" for l in range(len(raw))],
                    tag="gpu-paper")
    PT.assert_grads([x.cpu().numpy() for x in g2], [2 * x for x in gref],
                    names=[f"level{Rmin + l}+" for l in range(len(raw))], tag="gpu-paper")


def _views(sizes, seed=0):
    eyes = W.fibonacci_sphere(max(2, len(sizes)), 3.0)
    return [W.View(w, h, 7 + i, W.view_proj(eyes[i], w, h)) for i, (w, h) in enumerate(sizes)]


def _oracle_forward(ps, views, o):
    out = []
    for v in views:
        vis, col, logp, st = O.pforward(ps, v, W.inv_view_proj(v.M), o)
        out.append((vis.ravel(), col.reshape(-1, 3), logp.ravel(), st))
    return out


CASES = [
    dict(seed=1, T=400, R=3, sizes=[(97, 61)], mode=0),
    dict(seed=2, T=300, R=5, sizes=[(64, 64), (13, 40), (1, 1)], mode=0),
    dict(seed=3, T=500, R=2, sizes=[(80, 48)], mode=1),
    dict(seed=4, T=0, R=3, sizes=[(16, 9)], mode=0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"T{c['T']}R{c['R']}m{c['mode']}v{len(c['sizes'])}")
def test_paper_forward_matches_oracle(case):
    _say("forward", case)
    R = _R()
    ps = _soup(case["seed"], case["T"], case["R"])
    views = _views(case["sizes"])
    o = O.Opts(seed=0xC0FFEE + case["seed"], step=3, mode=case["mode"], background=(0.1, 0.2, 0.3))
    ds = R.PDeviceScene.from_host(ps)
    rv = R.Views.from_list(views)
    ro = R.Opts(seed=o.seed, step=3, mode=case["mode"], background=(0.1, 0.2, 0.3))
    vis, col, logp = R.pforward(ds, rv, ro, want_logp=True)
    torch.cuda.synchronize()
    ref = _oracle_forward(ps, views, o)
    rvis = np.concatenate([r[0] for r in ref])
    rcol = np.concatenate([r[1] for r in ref])
    rlp = np.concatenate([r[2] for r in ref])
    assert np.array_equal(_u64(vis), rvis)
    PT.assert_colours(col.cpu().numpy(), rcol)
    if case["mode"] == 0:
        np.testing.assert_allclose(logp.cpu().numpy(), rlp, rtol=1e-5, atol=1e-5)
    _say("covered", int((rvis != O.BG_KEY).sum()), "of", rvis.size)


# R = 6: a texture row (2,145 vertices x 8 channels) too large for the sorted path's
# LDS row, so the backward takes the per-pixel path with global atomics
BWD_CASES = CASES + [dict(seed=6, T=80, R=6, sizes=[(56, 40)], mode=0)]   # CASES[3]: an empty soup


@pytest.mark.parametrize("case", BWD_CASES, ids=lambda c: f"T{c['T']}R{c['R']}m{c['mode']}v{len(c['sizes'])}")
@pytest.mark.parametrize("from_log", [False, True])
def test_paper_backward_matches_oracle(case, from_log):
    _say("backward", case, "from_log", from_log)
    R = _R()
    ps = _soup(case["seed"], case["T"], case["R"])
    views = _views(case["sizes"])
    o = O.Opts(seed=0xC0FFEE + case["seed"], step=3, mode=case["mode"])
    ds = R.PDeviceScene.from_host(ps)
    rv = R.Views.from_list(views)
    ro = R.Opts(seed=o.seed, step=3, mode=case["mode"], reuse_bins=1 if from_log else 0)
    vis, col, _ = R.pforward(ds, rv, ro)
    rng = np.random.default_rng(case["seed"] + 100)
    P = rv.pixels
    gc = rng.normal(size=(P, 3)).astype(np.float32)
    gl = rng.normal(size=P).astype(np.float32)
    gpu = R.pbackward(ds, rv, ro, vis, col, torch.from_numpy(gc).cuda(), torch.from_numpy(gl).cuda())
    torch.cuda.synchronize()
    T, V = ps.tex.shape[0], ps.tex.shape[1]
    out = (np.zeros((T, 3, 3)), np.zeros((T, V, 8)), np.zeros(O.pmlp_params()))
    off = 0
    vis_h, col_h = _u64(vis), col.cpu().numpy()
    for v in views:
        n = v.width * v.height
        O.pbackward(ps, v, W.inv_view_proj(v.M), o, vis_h[off:off + n].reshape(v.height, v.width),
                    col_h[off:off + n].reshape(v.height, v.width, 3), gc[off:off + n].reshape(v.height, v.width, 3),
                    gl[off:off + n].reshape(v.height, v.width), out=out)
        off += n
    PT.assert_grads([g.cpu().numpy() for g in gpu], out, names=("verts", "tex", "mlp"), tag="gpu-paper")
    # accumulate = 1 adds into the outputs
    ro2 = R.Opts(seed=o.seed, step=3, mode=case["mode"], accumulate=1)
    gpu2 = R.pbackward(ds, rv, ro2, vis, col, torch.from_numpy(gc).cuda(), torch.from_numpy(gl).cuda(),
                       out=[g.clone() for g in gpu])
    torch.cuda.synchronize()
    PT.assert_grads([g.cpu().numpy() for g in gpu2], [2 * x for x in out], names=("verts+", "tex+", "mlp+"),
                    tag="gpu-paper")


# (seed, T, R, Rmin, Rtop, view sizes, from_log): the paper's levels 2..4 onto 5;
# the finest grid learnable too; one level; R = 6, whose sorted path does not
# exist, through the texture-gradient workspace and the assembly's backward
LEVEL_CASES = [
    dict(seed=21, T=300, R=5, Rmin=2, Rtop=4, sizes=[(64, 64), (13, 40), (1, 1)], from_log=False),
    dict(seed=22, T=400, R=3, Rmin=0, Rtop=3, sizes=[(97, 61)], from_log=True),
    dict(seed=23, T=200, R=2, Rmin=1, Rtop=1, sizes=[(48, 40)], from_log=False),
    dict(seed=24, T=80, R=6, Rmin=3, Rtop=5, sizes=[(56, 40)], from_log=False),
    dict(seed=25, T=150, R=3, Rmin=3, Rtop=3, sizes=[(40, 30)], from_log=False),   # the finest level alone
    dict(seed=26, T=0, R=5, Rmin=2, Rtop=4, sizes=[(16, 9)], from_log=False),      # an empty soup
]


@pytest.mark.parametrize("case", LEVEL_CASES, ids=lambda c: f"R{c['R']}L{c['Rmin']}-{c['Rtop']}")
def test_paper_levels_backward_matches_oracle(case):
    """soup_pbackward_levels against the oracle's backward followed by its
    assembly backward, on a texture assembled from random levels; then with
    accumulate = 1. Many fragments per wave in the first case put triangles
    on both sides of wave boundaries (the restricted parts are added)."""
    _say("levels backward", case)
    R = _R()
    rng = np.random.default_rng(case["seed"])
    ps = _soup(case["seed"], case["T"], case["R"])
    lv = W.random_levels(rng, case["T"], case["Rmin"], case["Rtop"], case["R"], sd=1.0)
    ps.tex = O.mc_assemble(lv.raw, case["Rmin"], case["R"])
    views = _views(case["sizes"])
    o = O.Opts(seed=0xBEEF + case["seed"], step=5, mode=0)
    ds = R.PDeviceScene.from_host(ps)
    rv = R.Views.from_list(views)
    ro = R.Opts(seed=o.seed, step=5, mode=0, reuse_bins=1 if case["from_log"] else 0)
    vis, col, _ = R.pforward(ds, rv, ro)
    P = rv.pixels
    gc = rng.normal(size=(P, 3)).astype(np.float32)
    gl = rng.normal(size=P).astype(np.float32)
    n_lv = case["Rtop"] - case["Rmin"] + 1
    gv, gr, gm = R.pbackward_levels(ds, rv, ro, vis, col, torch.from_numpy(gc).cuda(), case["Rmin"], n_lv,
                                    grad_logp=torch.from_numpy(gl).cuda())
    torch.cuda.synchronize()
    T, V = ps.tex.shape[0], ps.tex.shape[1]
    out = (np.zeros((T, 3, 3)), np.zeros((T, V, 8)), np.zeros(O.pmlp_params()))
    off = 0
    vis_h, col_h = _u64(vis), col.cpu().numpy()
    for v in views:
        n = v.width * v.height
        O.pbackward(ps, v, W.inv_view_proj(v.M), o, vis_h[off:off + n].reshape(v.height, v.width),
                    col_h[off:off + n].reshape(v.height, v.width, 3), gc[off:off + n].reshape(v.height, v.width, 3),
                    gl[off:off + n].reshape(v.height, v.width), out=out)
        off += n
    ref_lv = O.mc_assemble_bwd(ps.tex, out[1].astype(np.float32), case["Rmin"], n_lv, case["R"])
    names = ["verts"] + [f"level{case['Rmin'] + l}" for l in range(n_lv)] + ["mlp"]
    PT.assert_grads([gv.cpu().numpy()] + [g.cpu().numpy() for g in gr] + [gm.cpu().numpy()],
                    [out[0]] + list(ref_lv) + [out[2]], names=names, tag="gpu-paper")
    ro2 = R.Opts(seed=o.seed, step=5, mode=0, accumulate=1)
    gv2, gr2, gm2 = R.pbackward_levels(ds, rv, ro2, vis, col, torch.from_numpy(gc).cuda(), case["Rmin"], n_lv,
                                       grad_logp=torch.from_numpy(gl).cuda(),
                                       out=(gv.clone(), [g.clone() for g in gr], gm.clone()))
    torch.cuda.synchronize()
    PT.assert_grads([gv2.cpu().numpy()] + [g.cpu().numpy() for g in gr2] + [gm2.cpu().numpy()],
                    [2 * out[0]] + [2 * x for x in ref_lv] + [2 * out[2]], names=[n + "+" for n in names],
                    tag="gpu-paper")


def test_paper_levels_backward_rejects_bad_levels():
    from paper_2603_27151_amd import _lib
    R = _R()
    ps = _soup(5, 10, 3)
    ds = R.PDeviceScene.from_host(ps)
    rv = R.Views.from_list(_views([(8, 8)]))
    vis, col, _ = R.pforward(ds, rv, R.Opts())
    gc = torch.zeros(rv.pixels, 3, device="cuda")
    with pytest.raises(_lib.SoupError):   # Rtop above the scene's level
        R.pbackward_levels(ds, rv, R.Opts(), vis, col, gc, 2, 3)


def test_paper_opacity_one_is_a_z_buffer_and_blend_limits():
    """Opacity 1 everywhere: the winner is the nearest covering fragment
    whatever the draws (two seeds give the same buffer); A = 1 gives the RGB
    features, A = 0 the MLP output."""
    R = _R()
    ps = _soup(9, 600, 2)
    ps.tex[..., 7] = 1.0
    views = _views([(72, 56)])
    rv = R.Views.from_list(views)
    outs = []
    for A in (1.0, 0.0):
        ps.tex[..., 3] = A
        ds = R.PDeviceScene.from_host(ps)
        v1, c1, _ = R.pforward(ds, rv, R.Opts(seed=1))
        v2, c2, _ = R.pforward(ds, rv, R.Opts(seed=2))
        torch.cuda.synchronize()
        assert np.array_equal(_u64(v1), _u64(v2))
        ref = _oracle_forward(ps, views, O.Opts(seed=1))[0]
        assert np.array_equal(_u64(v1), ref[0])
        PT.assert_colours(c1.cpu().numpy(), ref[1])
        outs.append(c1.cpu().numpy())
    assert not np.allclose(outs[0], outs[1])


def test_paper_invalid_arguments_are_rejected():
    from paper_2603_27151_amd import _lib
    R = _R()
    ps = _soup(5, 10, 3)
    ds = R.PDeviceScene.from_host(ps)
    rv = R.Views.from_list(_views([(8, 8)]))
    with pytest.raises(ValueError):
        R.pforward(ds, rv, R.Opts(), minv=np.zeros((2, 4, 4), np.float32))
    bad = R.PDeviceScene(ds.verts, ds.tex, ds.mlp, 3)
    bad.R = 8
    with pytest.raises((ValueError, _lib.SoupError)):
        R.pforward(bad, rv, R.Opts())
    with pytest.raises(_lib.SoupError):
        R.mc_assemble([torch.zeros(2, 3, 8, device="cuda")], 0, 9)


def test_paper_step_at_full_size_on_sampled_pixels():
    """The paper-form step the benchmark times (levels 2..4 assembled onto the
    level-5 grid, four 800 x 800 views, L1 + D-SSIM loss): the assembled
    texture bit for bit on sampled triangles, the visibility, colours and
    log p at sampled pixels, and every gradient of the loss terms of sampled
    pixels against the oracle's per-pixel backward."""
    R = _R()
    wl = W.paper()
    _say("paper workload", wl.T, "triangles", len(wl.views), "views")
    raw = [torch.from_numpy(r).cuda() for r in wl.levels.raw]
    tex = R.mc_assemble(raw, wl.levels.Rmin, wl.levels.Rmax)
    ds = R.PDeviceScene(torch.from_numpy(wl.verts).cuda(), tex, torch.from_numpy(wl.mlp).cuda(), wl.levels.Rmax)
    rv = R.Views.from_list(wl.views)
    ro = R.Opts(seed=wl.seed, step=wl.step, reuse_bins=1)
    vis, col, logp = R.pforward(ds, rv, ro, want_logp=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    tsample = rng.choice(wl.T, 64, replace=False)
    tex_ref = O.mc_assemble([r[tsample] for r in wl.levels.raw], wl.levels.Rmin, wl.levels.Rmax)
    tex_h = tex.cpu().numpy()
    assert np.array_equal(tex_h[tsample], tex_ref)
    ps = W.PScene(wl.verts, tex_h, wl.mlp, wl.levels.Rmax)
    vis_h, col_h, lp_h = _u64(vis), col.cpu().numpy(), logp.cpu().numpy()
    o = O.Opts(seed=wl.seed, step=wl.step)
    off = 0
    n_checked = 0
    for v in wl.views:
        n = v.width * v.height
        xy = np.stack([rng.integers(0, v.width, 500), rng.integers(0, v.height, 500)], 1).astype(np.int32)
        xy = np.unique(xy, axis=0)
        rvis, rcol, rlp = O.pforward_pixels(ps, v, W.inv_view_proj(v.M), o, xy)
        lin = off + xy[:, 1] * v.width + xy[:, 0]
        assert np.array_equal(vis_h[lin], rvis)
        PT.assert_colours(col_h[lin], rcol)
        np.testing.assert_allclose(lp_h[lin], rlp, rtol=1e-5, atol=1e-5)
        n_checked += len(xy)
        off += n
    _say("forward sampled pixels", n_checked, "covered", int((vis_h != O.BG_KEY).sum()), "of", vis_h.size)
    # backward of the loss terms of sampled pixels
    P = rv.pixels
    gc = np.zeros((P, 3), np.float32)
    gl = np.zeros(P, np.float32)
    samples = []
    off = 0
    for v in wl.views:
        xy = np.stack([rng.integers(0, v.width, 300), rng.integers(0, v.height, 300)], 1).astype(np.int32)
        xy = np.unique(xy, axis=0)
        lin = off + xy[:, 1] * v.width + xy[:, 0]
        gc[lin] = rng.normal(size=(len(xy), 3)).astype(np.float32)
        gl[lin] = rng.normal(size=len(xy)).astype(np.float32)
        samples.append((v, xy, lin))
        off += v.width * v.height
    gpu = R.pbackward(ds, rv, ro, vis, col, torch.from_numpy(gc).cuda(), torch.from_numpy(gl).cuda())
    torch.cuda.synchronize()
    gpu = [g.cpu().numpy() for g in gpu]
    refs = [np.zeros((wl.T, 3, 3)), np.zeros(tex_h.shape), np.zeros(O.pmlp_params())]
    for v, xy, lin in samples:
        a = O.pbackward_pixels(ps, v, W.inv_view_proj(v.M), o, xy, gc[lin], gl[lin])
        for r, x in zip(refs, a):
            r += x
    PT.assert_grads(gpu, refs, names=("verts", "tex", "mlp"), tag="gpu-paper")
    # the bench's own backward: the levels' gradients straight from the sorted pass,
    # against the oracle's assembly backward of its texture gradient (on the
    # triangles that the sampled pixels reach; every other row must stay zero)
    Rmin, n_lv = wl.levels.Rmin, len(wl.levels.raw)
    gv, glv, gm = R.pbackward_levels(ds, rv, ro, vis, col, torch.from_numpy(gc).cuda(), Rmin, n_lv,
                                     grad_logp=torch.from_numpy(gl).cuda())
    torch.cuda.synchronize()
    touched = np.nonzero(np.abs(refs[1]).reshape(wl.T, -1).max(1) > 0)[0]
    _say("levels backward: triangles reached by the sampled pixels", len(touched))
    ref_lv = O.mc_assemble_bwd(tex_h[touched], refs[1][touched].astype(np.float32), Rmin, n_lv, wl.levels.Rmax)
    glv = [g.cpu().numpy() for g in glv]
    PT.assert_grads([gv.cpu().numpy()] + [g[touched] for g in glv] + [gm.cpu().numpy()],
                    [refs[0]] + list(ref_lv) + [refs[2]],
                    names=["verts"] + [f"level{Rmin + l}" for l in range(n_lv)] + ["mlp"], tag="gpu-paper")
    rest = np.ones(wl.T, bool)
    rest[touched] = False
    for g in glv:
        assert not np.any(g[rest]), "a level gradient row outside the sampled pixels' triangles is not zero"
