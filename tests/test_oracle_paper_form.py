"""Pins of the oracle's paper form (Section 3.3, learnable multi-resolution
triangle texture and neural deferred shading; Supplement B.3 and B.6) against
what the paper and the mathematics fix: the grid-vertex count (561 at R = 5),
the micro-triangle lookup against a brute-force search with exact
barycentrics, the assembly of coarse levels against hand-sampled values and
affine fields, the spherical harmonics by quadrature and the addition
theorem, the deferred colour against a float64 model built from ray casting,
the opacity mask against Eq. (5) and Eq. (6), colour gradients by finite
differences and the score term's unbiasedness (Eq. (8), (9)).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_27151_amd import workloads as W
from tests import geometry as geo
from tests import scenes as S
from tests.test_oracle_pins import _bary_screen, _rand_snapped_tris, _ray_bary


# --------------------------------------------------------------------------
# mesh-colour grid: layout and lookup
# --------------------------------------------------------------------------

def _grid(R):
    """Grid vertices (i, j), i + j <= n, in storage order: rows of constant j
    from j = 0, i ascending within a row."""
    n = 1 << R
    return [(i, j) for j in range(n + 1) for i in range(n + 1 - j)]


def _micro_triangles(n):
    """Every micro-triangle of the level with n segments per edge, as three
    (i, j) grid vertices."""
    out = []
    for j in range(n):
        for i in range(n - j):
            out.append(((i, j), (i + 1, j), (i, j + 1)))
            if i + j <= n - 2:
                out.append(((i + 1, j + 1), (i + 1, j), (i, j + 1)))
    return out


def _brute_weights(n, b1, b2):
    """Vertices and float64 barycentric weights of a micro-triangle that
    contains (b1, b2), found by trying all of them."""
    p = np.array([b1 * n, b2 * n], np.float64)
    best = None
    for tri in _micro_triangles(n):
        a, b, c = (np.array(v, np.float64) for v in tri)
        Mt = np.stack([b - a, c - a], 1)
        l = np.linalg.solve(Mt, p - a)
        w = np.array([1 - l[0] - l[1], l[0], l[1]])
        if best is None or w.min() > best[1].min():
            best = (tri, w)
    return best


def test_grid_vertex_count_is_the_closed_form_and_561_at_level_5():
    # Section 3.3 gives (2^(R-1) + 1)(2^R + 1) vertices per level; Supplement B.6 561 at R = 5
    assert O.mc_count(5) == 561
    for R in range(0, 8):
        assert O.mc_count(R) == len(_grid(R)) == W.mc_vertices(R)
        if R >= 1:
            assert O.mc_count(R) == (2 ** (R - 1) + 1) * (2 ** R + 1)
    assert O.mc_count(0) == 3                       # the triangle's own vertices


@pytest.mark.parametrize("R", [0, 1, 2, 3, 5])
def test_lookup_weights_match_a_brute_force_search(R):
    n = 1 << R
    table = _grid(R)
    rng = np.random.default_rng(100 + R)
    pts = []
    for _ in range(300):
        b = rng.dirichlet([1, 1, 1])
        pts.append((b[1], b[2]))
    # points on micro-triangle edges and on the triangle's boundary
    for _ in range(100):
        i = int(rng.integers(0, n + 1))
        t = float(rng.random())
        pts += [(i / n, t * (n - i) / n), (t * (n - i) / n, i / n), (t, 1 - t)]
    for b1, b2 in pts:
        b1, b2 = float(np.float32(b1)), float(np.float32(b2))
        if b1 + b2 > 1.0:
            continue
        idx, w = O.mc_lookup(R, b1, b2)
        assert len(set(idx.tolist())) == 3
        verts = [table[k] for k in idx]
        # the three vertices form a micro-triangle of this level
        assert tuple(sorted(verts)) in {tuple(sorted(t)) for t in _micro_triangles(n)}
        w = w.astype(np.float64)
        assert w.min() >= -1e-6 and abs(w.sum() - 1) < 1e-6
        # the weights reconstruct the point
        rec = sum(wk * np.array(v, np.float64) for wk, v in zip(w, verts)) / n
        assert np.allclose(rec, [b1, b2], atol=2e-7)
        # same interpolation as the brute-force micro-triangle (equal on shared edges)
        tri, wb = _brute_weights(n, b1, b2)
        f = {v: float(rng.normal()) for v in table}
        got = sum(wk * f[v] for wk, v in zip(w, verts))
        want = sum(wk * f[v] for wk, v in zip(wb, tri))
        assert abs(got - want) < 1e-5


def test_lookup_is_exact_at_grid_vertices():
    for R in (1, 3, 5):
        n = 1 << R
        for k, (i, j) in enumerate(_grid(R)):
            idx, w = O.mc_lookup(R, i / n, j / n)
            pos = [int(q) for q in np.flatnonzero(w == 1.0)]
            assert len(pos) == 1 and idx[pos[0]] == k
            assert np.all(w[np.arange(3) != pos[0]] == 0.0)


def test_interpolated_field_is_continuous():
    """Piecewise linear on the micro-triangles and continuous across their
    edges: along a segment, no jump larger than the steepest micro-triangle
    slope allows."""
    R = 3
    n = 1 << R
    table = _grid(R)
    rng = np.random.default_rng(3)
    vals = rng.normal(size=len(table))
    slope = 4 * n * np.abs(vals).max()
    for _ in range(20):
        a, b = rng.dirichlet([1, 1, 1]), rng.dirichlet([1, 1, 1])
        ts = np.linspace(0, 1, 2001)
        f = []
        for t in ts:
            p = (1 - t) * a + t * b
            idx, w = O.mc_lookup(R, float(p[1]), float(p[2]))
            f.append(float(np.dot(w.astype(np.float64), vals[idx])))
        step = np.linalg.norm(b - a) / 2000
        assert np.abs(np.diff(f)).max() <= slope * step + 1e-5


# --------------------------------------------------------------------------
# multi-resolution assembly (Section 3.3)
# --------------------------------------------------------------------------

def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def test_single_level_assembly_is_the_sigmoid():
    rng = np.random.default_rng(1)
    lv = W.random_levels(rng, 3, 2, 2, 2)
    tex = O.mc_assemble(lv.raw, 2)
    assert np.allclose(tex, _sig(lv.raw[0].astype(np.float64)), rtol=0, atol=2e-7)


@pytest.mark.parametrize("Rmin,Rtop,Rmax", [(0, 1, 2), (0, 2, 2), (1, 2, 3)])
def test_coarse_levels_are_sampled_at_the_fine_vertices(Rmin, Rtop, Rmax):
    rng = np.random.default_rng(Rmin * 10 + Rtop + Rmax)
    T = 2
    lv = W.random_levels(rng, T, Rmin, Rtop, Rmax)
    tex = O.mc_assemble(lv.raw, Rmin, Rmax)
    n = 1 << Rmax
    for t in range(T):
        for k, (i, j) in enumerate(_grid(Rmax)):
            z = np.zeros(8)
            for l, R in enumerate(range(Rmin, Rtop + 1)):
                tri, w = _brute_weights(1 << R, i / n, j / n)
                tab = {v: q for q, v in enumerate(_grid(R))}
                z += sum(wk * lv.raw[l][t, tab[v]].astype(np.float64) for wk, v in zip(w, tri))
            assert np.allclose(tex[t, k], _sig(z), rtol=0, atol=5e-7)


def test_affine_levels_assemble_to_the_sigmoid_of_an_affine_field():
    Rmin, Rtop, Rmax = 1, 3, 4
    rng = np.random.default_rng(7)
    coef = rng.normal(size=(Rtop - Rmin + 1, 3, 8))
    raw = []
    for l, R in enumerate(range(Rmin, Rtop + 1)):
        n = 1 << R
        g = np.array([[1.0, i / n, j / n] for (i, j) in _grid(R)])
        raw.append((g @ coef[l])[None].astype(np.float32))
    # the float32 rounding of the raw values is part of the input
    tex = O.mc_assemble(raw, Rmin, Rmax)
    n = 1 << Rmax
    g = np.array([[1.0, i / n, j / n] for (i, j) in _grid(Rmax)])
    want = _sig(g @ coef.sum(0))
    assert np.abs(tex[0] - want).max() < 2e-6


def test_assembly_backward_matches_finite_differences():
    Rmin, Rtop, Rmax = 0, 1, 2
    rng = np.random.default_rng(5)
    lv = W.random_levels(rng, 2, Rmin, Rtop, Rmax)
    gt = rng.normal(size=(2, O.mc_count(Rmax), 8)).astype(np.float32)
    tex = O.mc_assemble(lv.raw, Rmin, Rmax)
    grads = O.mc_assemble_bwd(tex, gt, Rmin, len(lv.raw), Rmax)

    def loss(raw):
        return float((O.mc_assemble(raw, Rmin, Rmax).astype(np.float64) * gt).sum())

    for l in range(len(lv.raw)):
        for _ in range(12):
            idx = tuple(int(rng.integers(0, s)) for s in lv.raw[l].shape)
            rp = [r.copy() for r in lv.raw]
            rm = [r.copy() for r in lv.raw]
            h = 1e-2
            rp[l][idx] += h
            rm[l][idx] -= h
            num = (loss(rp) - loss(rm)) / (float(rp[l][idx]) - float(rm[l][idx]))
            assert abs(num - grads[l][idx]) < 2e-3 * (abs(num) + 1e-2), (l, idx, num, grads[l][idx])


# --------------------------------------------------------------------------
# spherical harmonics of the view direction (Supplement B.3)
# --------------------------------------------------------------------------

def test_harmonics_are_orthonormal_on_the_sphere():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for degree <= 4 products
    xg, wg = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((9, 9))
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            y = O.sh2([st * math.cos(ph), st * math.sin(ph), ct]).astype(np.float64)
            G += np.outer(y, y) * w * (2 * math.pi / nphi)
    assert np.abs(G - np.eye(9)).max() < 2e-6


def test_harmonics_addition_theorem_and_degree():
    """sum over m of Y_lm(d)^2 = (2l + 1) / (4 pi) for every direction, and
    each degree-l block is a homogeneous polynomial of degree l (checked by
    Y(-d) = (-1)^l Y(d))."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        y = O.sh2(d).astype(np.float64)
        for l, sl in [(0, slice(0, 1)), (1, slice(1, 4)), (2, slice(4, 9))]:
            assert abs((y[sl] ** 2).sum() - (2 * l + 1) / (4 * math.pi)) < 1e-6
        ym = O.sh2(-d).astype(np.float64)
        assert np.allclose(ym[1:4], -y[1:4], atol=1e-7) and np.allclose(ym[4:], y[4:], atol=1e-7)


def test_view_direction_is_the_pixel_ray_from_the_eye():
    Wd, Hd = 37, 29
    eye = np.array([0.4, -0.3, 2.6])
    M = W.view_proj(eye, Wd, Hd)
    view = W.View(Wd, Hd, 0, M)
    Minv = W.inv_view_proj(M)
    M64 = np.linalg.inv(M.astype(np.float64))
    for (x, y) in [(18, 14), (0, 0), (36, 28), (5, 20)]:
        d = O.view_dir(view, Minv, x, y).astype(np.float64)
        ndc = np.array([(x + 0.5) / (Wd / 2) - 1, 1 - (y + 0.5) / (Hd / 2), 0.3, 1.0])
        q = M64 @ ndc
        ref = q[:3] / q[3] - eye
        ref /= np.linalg.norm(ref)
        assert np.allclose(d, ref, atol=2e-5), (x, y, d, ref)
    # the centre pixel of an odd-sized image looks at the target (the origin)
    d = O.view_dir(view, Minv, 18, 14).astype(np.float64)
    assert np.allclose(d, -eye / np.linalg.norm(eye), atol=2e-5)


# --------------------------------------------------------------------------
# forward: mask (Eq. (2), (3), (5), (6)) and deferred colour
# --------------------------------------------------------------------------

def _pscene(tris, R, tex_fn, mlp=None):
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    T = tris.shape[0]
    tex = np.zeros((T, O.mc_count(R), 8), np.float32)
    for t in range(T):
        tex[t] = tex_fn(t)
    if mlp is None:
        mlp = np.zeros(O.pmlp_params(), np.float32)
    return W.PScene(tris, tex, mlp, R)


def test_opacity_one_is_an_ordinary_z_buffer():
    rng = np.random.default_rng(13)
    Wd = Hd = 20
    view = S.ortho_view(Wd, Hd)
    n = 8
    zs = rng.permutation(np.linspace(-0.7, 0.7, n))
    tris, verts = [], []
    for (v, z) in zip(_rand_snapped_tris(rng, n, Wd, Hd, lo=0, hi=Wd), zs):
        tris.append(v)
        verts.append(S.tri_world([(x / 256.0, y / 256.0) for x, y in v], z, Wd, Hd))

    def tex(t):
        a = rng.uniform(0, 1, (O.mc_count(2), 8))
        a[:, 7] = 1.0
        return a
    ps = _pscene(verts, 2, tex)
    vis, _, logp, _ = O.pforward(ps, view, np.eye(4, dtype=np.float32), O.Opts(seed=4))
    covers = [geo.coverage_rational([tuple(p) for p in v], Wd, Hd) for v in tris]
    for y in range(Hd):
        for x in range(Wd):
            cand = [t for t in range(n) if (x, y) in covers[t]]
            if not cand:
                assert vis[y, x] == O.BG_KEY
                continue
            assert int(vis[y, x]) & 0xFFFFFFFF == min(cand, key=lambda t: zs[t])
            assert abs(logp[y, x]) < 1e-6       # the interpolated 1 is within rounding of 1


def _layers(n, R, rng, zs=None, A=None):
    """Full-screen fronto-parallel squares (two triangles each) at increasing
    depth with random textures."""
    zs = np.linspace(-0.5, 0.5, n) if zs is None else zs
    q = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
    tris = []
    for k in range(n):
        for (a, b, c) in [(0, 1, 2), (0, 2, 3)]:
            tris.append(np.array([[*q[a], zs[k]], [*q[b], zs[k]], [*q[c], zs[k]]], np.float32))

    def tex(t):
        v = rng.uniform(0.0, 1.0, (O.mc_count(R), 8))
        v[:, 7] = rng.uniform(0.15, 0.85, O.mc_count(R))
        if A is not None:
            v[:, 3] = A
        return v
    return tris, tex


def _texel(ps, t, x, y, Wd, Hd):
    """float64 interpolated texture of triangle t at pixel (x, y) of the
    orthographic view: screen barycentrics are the perspective-correct ones."""
    xy = [((v[0] + 1) * Wd / 2, (1 - v[1]) * Hd / 2) for v in ps.verts[t]]
    b = _bary_screen(xy, x + 0.5, y + 0.5)
    if min(b) < 0:
        return None, None, None
    tri, w = _brute_weights(1 << ps.R, b[1], b[2])
    tab = {v: q for q, v in enumerate(_grid(ps.R))}
    ids = [tab[v] for v in tri]
    val = sum(wk * ps.tex[t, q].astype(np.float64) for wk, q in zip(w, ids))
    return val, ids, w


def test_stochastic_mask_takes_the_first_fragment_under_its_opacity():
    rng = np.random.default_rng(17)
    Wd, Hd = 16, 12
    tris, tex = _layers(3, 2, rng)
    ps = _pscene(tris, 2, tex)
    view = S.ortho_view(Wd, Hd, view_id=5)
    o = O.Opts(seed=0xABCD, step=3)
    vis, _, logp, st = O.pforward(ps, view, np.eye(4, dtype=np.float32), o)
    checked = 0
    for y in range(Hd):
        for x in range(Wd):
            frs = []
            for t in range(len(tris)):
                val, _, _ = _texel(ps, t, x, y, Wd, Hd)
                if val is not None and t // 2 not in [f[0] // 2 for f in frs]:
                    frs.append((t, val[7]))
            assert len(frs) == 3
            u = [O.uniform(o.seed, y * Wd + x, t, 5, 3) for t, _ in frs]
            if min(abs(uk - a) for uk, (_, a) in zip(u, frs)) < 1e-5:
                continue
            win = next((k for k, (uk, (_, a)) in enumerate(zip(u, frs)) if uk < a), None)
            a = np.array([f[1] for f in frs])
            if win is None:
                assert vis[y, x] == O.BG_KEY
                lp = np.log1p(-a).sum()
            else:
                assert int(vis[y, x]) & 0xFFFFFFFF == frs[win][0]
                lp = np.log1p(-a[:win]).sum() + math.log(a[win])
            assert abs(logp[y, x] - lp) < 1e-5
            checked += 1
    assert checked > 150
    assert st["covered_pixels"] == Wd * Hd


def test_threshold_mode_takes_the_first_fragment_above_one_half():
    rng = np.random.default_rng(19)
    Wd, Hd = 16, 12
    tris, tex = _layers(3, 3, rng)
    ps = _pscene(tris, 3, tex)
    view = S.ortho_view(Wd, Hd)
    vis, _, _, _ = O.pforward(ps, view, np.eye(4, dtype=np.float32), O.Opts(mode=1))
    for y in range(Hd):
        for x in range(Wd):
            best = None
            for t in range(len(tris)):
                val, _, _ = _texel(ps, t, x, y, Wd, Hd)
                if val is not None and abs(val[7] - 0.5) > 1e-6 and val[7] > 0.5:
                    z = ps.verts[t, 0, 2]
                    if best is None or z < best[1]:
                        best = (t, z)
            got = int(vis[y, x])
            if best is None:
                assert got == int(O.BG_KEY)
            else:
                assert got & 0xFFFFFFFF in (best[0], best[0] ^ 1) and ps.verts[got & 0xFFFFFFFF, 0, 2] == best[1]


def _persp_scene(rng, R=3):
    tris = np.array([[[-0.9, -0.8, 0.2], [0.8, -0.6, -0.5], [-0.1, 0.9, 0.1]],
                     [[-0.5, -0.2, 0.9], [0.6, 0.1, 0.7], [0.0, 0.7, 1.1]]], np.float32)
    ps = W.random_pscene(rng, tris, R)
    ps.tex[..., 7] = 1.0                          # opaque: the nearest fragment wins
    return ps


def _mlp_f64(mlp, x):
    d = W.PF_MLP_DIMS
    at = 0
    h = np.asarray(x, np.float64)
    for l in range(3):
        Wl = mlp[at:at + d[l + 1] * d[l]].reshape(d[l + 1], d[l]).astype(np.float64)
        at += d[l + 1] * d[l]
        b = mlp[at:at + d[l + 1]].astype(np.float64)
        at += d[l + 1]
        h = Wl @ h + b
        if l < 2:
            h = np.maximum(h, 0)
    return h


def test_deferred_colour_matches_a_float64_model():
    """Colour of the winner = A RGB + (1 - A) sigmoid(MLP(features, SH(view)))
    with features interpolated in the micro-triangle that contains the
    ray-cast barycentrics."""
    rng = np.random.default_rng(23)
    ps = _persp_scene(rng)
    Wd = Hd = 40
    eye = (0.2, 0.1, 3.0)
    M = W.view_proj(eye, Wd, Hd)
    view = W.View(Wd, Hd, 0, M)
    Minv = W.inv_view_proj(M)
    vis, color, _, _ = O.pforward(ps, view, Minv, O.Opts(seed=1))
    tab = {v: q for q, v in enumerate(_grid(ps.R))}
    checked = 0
    for y in range(0, Hd, 2):
        for x in range(0, Wd, 2):
            if vis[y, x] == O.BG_KEY:
                assert np.all(color[y, x] == 0.0)
                continue
            t = int(vis[y, x]) & 0xFFFFFFFF
            l = _ray_bary(M, ps.verts[t], x, y, Wd, Hd)
            tri, w = _brute_weights(1 << ps.R, l[0], l[1])
            if w.min() < 1e-3:
                continue                     # on a micro-triangle edge: either side is right
            sh = O.sh2(O.view_dir(view, Minv, x, y)).astype(np.float64)

            def model(b1, b2):
                _, ww = _brute_weights(1 << ps.R, b1, b2)
                f = sum(wk * ps.tex[t, tab[v]].astype(np.float64) for wk, v in zip(ww, tri))
                m = _sig(_mlp_f64(ps.mlp, np.concatenate([f[:7], sh])))
                return f[3] * f[:3] + (1 - f[3]) * m
            want = model(l[0], l[1])
            # the rasterizer samples at vertices snapped to 1/256 pixel: its barycentrics
            # are within 2e-4 of the ray-cast ones (the barycentric pin), so allow the
            # colour's slope times that
            h = 1e-6
            slope = np.abs(model(l[0] + h, l[1]) - want) / h + np.abs(model(l[0], l[1] + h) - want) / h
            tol = 2e-4 * slope + 2e-6
            assert np.all(np.abs(color[y, x] - want) <= tol), (x, y, color[y, x], want, tol)
            checked += 1
    assert checked > 40


# --------------------------------------------------------------------------
# backward: colour path by finite differences, score term (Eq. (8), (9))
# --------------------------------------------------------------------------

def test_colour_gradients_match_finite_differences():
    rng = np.random.default_rng(29)
    ps = _persp_scene(rng)
    Wd = Hd = 48
    M = W.view_proj((0.2, 0.1, 3.0), Wd, Hd)
    view = W.View(Wd, Hd, 0, M)
    Minv = W.inv_view_proj(M)
    o = O.Opts(seed=5, edge_pairs=2, analysis=1)
    vis, color, _, _ = O.pforward(ps, view, Minv, o)
    g = np.array([0.7, -0.4, 1.1])
    tested = 0
    for (x, y) in [(24, 24), (20, 30), (30, 18), (14, 26), (27, 27), (22, 16), (18, 20)]:
        key = int(vis[y, x])
        if key == int(O.BG_KEY):
            continue
        t = key & 0xFFFFFFFF
        l = _ray_bary(M, ps.verts[t], x, y, Wd, Hd)
        _, w = O.mc_lookup(ps.R, l[0], l[1])
        if w.min() < 0.03:
            continue                                  # finite steps would cross a micro-triangle edge
        gc = np.zeros((Hd, Wd, 3), np.float32)
        gc[y, x] = g
        gv, gt, gm = O.pbackward(ps, view, Minv, o, vis, color, gc, None)
        assert np.all(gt[..., 7] == 0.0)              # the colour path never reaches the opacity

        def f(p):
            rgb, _ = O.pcolor_f64(p, view, Minv, o, t, x, y)
            return float(np.dot(g, rgb))

        def fd(name, idx, h):
            p = W.PScene(ps.verts.copy(), ps.tex.copy(), ps.mlp.copy(), ps.R)
            arr = getattr(p, name)
            base = float(arr[idx])
            arr[idx] = np.float32(base + h)
            hp = float(arr[idx]) - base
            fp = f(p)
            arr[idx] = np.float32(base - h)
            hm = base - float(arr[idx])
            fm = f(p)
            return (fp - fm) / (hp + hm)

        for i in range(3):
            for k in range(3):
                num = fd("verts", (t, i, k), 1e-3)
                assert abs(num - gv[t, i, k]) < 2e-3 * (abs(num) + 1e-3), ("v", t, i, k, num, gv[t, i, k])
        nz = np.argwhere(np.abs(gt[t]) > 0)
        assert len(nz) == 3 * 7
        for idx in nz:
            num = fd("tex", (t, *idx), 1e-3)
            assert abs(num - gt[(t, *idx)]) < 1e-4 * (abs(num) + 1e-3), ("tex", idx, num, gt[(t, *idx)])
        for j in range(len(ps.mlp)):
            if j % 7:
                continue
            num = fd("mlp", (j,), 1e-4)
            assert abs(num - gm[j]) < 1e-4 * (abs(num) + 1e-3), ("mlp", j, num, gm[j])
        tested += 1
    assert tested >= 3


def test_score_estimator_is_unbiased_on_textured_opacity():
    """Mean over draws of the estimator's texture gradients = the exact
    derivative of E_p[L] (Eq. (6), (7)) for layers whose opacity and colour
    vary over the mesh-colour grid; with A = 1 the colour is the RGB feature
    and the MLP output m enters only through d colour / d A = RGB - m."""
    Wd, Hd, R = 16, 12, 2
    rng = np.random.default_rng(31)
    tris, tex = _layers(2, R, rng, zs=[-0.4, 0.3], A=1.0)
    mlp = np.zeros(O.pmlp_params(), np.float32)
    mlp[-3:] = [0.4, -0.7, 1.3]                        # MLP output = sigmoid(bias), constant
    m = _sig(mlp[-3:].astype(np.float64))
    ps = _pscene(tris, R, tex, mlp)
    view = S.ortho_view(Wd, Hd)
    I = np.eye(4, dtype=np.float32)
    target = np.array([0.2, 0.7, 0.4])
    T = len(tris)
    exact = np.zeros((T, O.mc_count(R), 8))
    for py in range(Hd):
        for px in range(Wd):
            layer = []
            for t in range(T):
                val, ids, w = _texel(ps, t, px, py, Wd, Hd)
                if val is not None and t // 2 not in [l[0] // 2 for l in layer]:
                    layer.append((t, ids, w, val[7], val[:3]))
            assert len(layer) == 2
            al = [l[3] for l in layer]
            p = [np.prod([1 - al[j] for j in range(k)]) * al[k] for k in range(2)] + [np.prod([1 - a for a in al])]
            Lf = [float(((l[4] - target) ** 2).sum()) for l in layer] + [float((target ** 2).sum())]
            for k, (t, ids, w, a, c) in enumerate(layer):
                dE = Lf[k] * p[k] / a - sum(Lf[f] * p[f] / (1 - a) for f in range(k + 1, 3))
                for q, wq in zip(ids, w):
                    exact[t, q, 7] += dE * wq
                    exact[t, q, 0:3] += p[k] * 2 * (c - target) * wq
                    exact[t, q, 3] += p[k] * float(np.dot(2 * (c - target), c - m)) * wq
    samples = []
    for step in range(40):
        o = O.Opts(seed=77, step=step, edge_pairs=2)
        vis, color, _, _ = O.pforward(ps, view, I, o)
        c = color.astype(np.float64)
        gC = (2 * (c - target)).astype(np.float32)
        gL = ((c - target) ** 2).sum(-1).astype(np.float32)
        gv, gt, gm = O.pbackward(ps, view, I, o, vis, color, gC, gL)
        samples.append(gt[..., [0, 1, 2, 3, 7]].ravel())
        gv_s, _, gm_s = O.pbackward(ps, view, I, o, vis, color, np.zeros_like(gC), gL)
        assert np.all(gv_s == 0.0) and np.all(gm_s == 0.0)       # the score term moves no vertex
    sm = np.array(samples)
    se = sm.std(0, ddof=1) / math.sqrt(len(sm))
    want = exact[..., [0, 1, 2, 3, 7]].ravel()
    assert np.abs(want).max() > 1e-2
    assert np.all(np.abs(sm.mean(0) - want) < 5 * se + 1e-6), np.abs(sm.mean(0) - want) / (se + 1e-12)


def test_pixel_entry_points_agree_with_full_image():
    rng = np.random.default_rng(37)
    ps = _persp_scene(rng)
    ps.tex[..., 7] = rng.uniform(0.2, 0.9, ps.tex[..., 7].shape)
    Wd, Hd = 40, 33
    M = W.view_proj((0.2, 0.1, 3.0), Wd, Hd)
    view = W.View(Wd, Hd, 3, M)
    Minv = W.inv_view_proj(M)
    o = O.Opts(seed=11, step=2)
    vis, color, logp, _ = O.pforward(ps, view, Minv, o)
    xy = np.array([(x, y) for y in range(0, Hd, 4) for x in range(1, Wd, 3)], np.int32)
    v2, c2, l2 = O.pforward_pixels(ps, view, Minv, o, xy)
    assert np.array_equal(v2, vis[xy[:, 1], xy[:, 0]])
    assert np.array_equal(c2, color[xy[:, 1], xy[:, 0]])
    assert np.array_equal(l2, logp[xy[:, 1], xy[:, 0]])
    gc = rng.normal(size=(len(xy), 3)).astype(np.float32)
    gl = rng.normal(size=len(xy)).astype(np.float32)
    full_gc = np.zeros((Hd, Wd, 3), np.float32)
    full_gl = np.zeros((Hd, Wd), np.float32)
    full_gc[xy[:, 1], xy[:, 0]] = gc
    full_gl[xy[:, 1], xy[:, 0]] = gl
    a = O.pbackward(ps, view, Minv, o, vis, color, full_gc, full_gl)
    b = O.pbackward_pixels(ps, view, Minv, o, xy, gc, gl)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-14 * max(1.0, np.abs(x).max()))
    assert np.abs(a[0]).max() > 0 and np.abs(a[1]).max() > 0 and np.abs(a[2]).max() > 0
