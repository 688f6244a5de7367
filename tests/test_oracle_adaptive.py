"""Pins of the adaptive-control oracle (Section 3.4, "Adaptive control of
primitives"; Supplement B, resampling of a random initialisation).

CPU only. Each test checks the oracle against something fixed outside it:
hand-counted answers, projected lengths in closed form for orthographic and
pinhole cameras, worked plans, and the geometry of a split (the halves
tile the parent; an affine texture is reproduced at the half's texels, whose
parent coordinates come from solving for them in 3-D, not from the oracle's
slot mapping).
"""
import numpy as np
import pytest

from oracle import adaptive as A

BG = A.BG_KEY


def _key(depth_bits: int, tri: int) -> int:
    return (depth_bits << 32) | tri


# --------------------------------------------------------------------------
# coverage counts
# --------------------------------------------------------------------------

def test_coverage_counts_hand_counted():
    vis = np.array([_key(7, 3), _key(9, 3), _key(1, 1), BG, _key(0, 3), _key(5, 0),
                    _key(2, 9), BG, _key(3, 1)], dtype=np.uint64)
    # triangle 9 is out of range for T = 4 and is skipped; background is skipped
    assert A.coverage_counts(vis, 4).tolist() == [1, 2, 0, 3]


def test_coverage_counts_sum_to_covered_pixels():
    rng = np.random.default_rng(1)
    ids = rng.integers(0, 50, size=4000)
    vis = (rng.integers(0, 1 << 31, size=4000).astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)
    bg = rng.random(4000) < 0.3
    vis[bg] = np.uint64(BG)
    c = A.coverage_counts(vis, 50)
    assert c.sum() == int((~bg).sum())
    assert c.tolist() == np.bincount(ids[~bg], minlength=50).tolist()


# --------------------------------------------------------------------------
# screen-space edge lengths
# --------------------------------------------------------------------------

def _ortho(sx, sy):
    return np.array([[sx, 0, 0, 0], [0, sy, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]], dtype=np.float32)


def _pinhole(f):
    # clip w = z: a camera looking down +z with focal f in NDC units
    return np.array([[f, 0, 0, 0], [0, f, 0, 0], [0, 0, 1, 0], [0, 0, 1, 0]], dtype=np.float32)


def test_edge_lengths_orthographic_closed_form():
    W, H = 200, 100
    a, b = 0.5, 0.25
    tri = np.array([[[0, 0, 0], [a, 0, 0], [0, b, 0]]], dtype=np.float32)
    M = _ortho(1.0, 1.0)
    r = A.edge_lengths(tri, M[None], [W], [H], 0.1)
    ex = W / 2 * a          # pixels along x
    ey = H / 2 * b          # pixels along y
    np.testing.assert_allclose(r[0], [ex / H, np.hypot(ex, ey) / H, ey / H], rtol=1e-6)


def test_edge_lengths_pinhole_takes_the_nearest_view():
    W = H = 256
    L, f = 0.2, 2.0
    tri = np.array([[[0, 0, 0], [L, 0, 0], [0, L, 0]]], dtype=np.float32)
    # the same camera model at two distances: translate the triangle by d in z
    views = []
    for d in (4.0, 2.0):
        M = _pinhole(f).astype(np.float64)
        M[:, 3] += M[:, 2] * d     # x -> x + d e_z before projecting
        views.append(M.astype(np.float32))
    r = A.edge_lengths(tri, np.stack(views), [W, W], [H, H], 0.1)
    px = W / 2 * f * L / 2.0       # the nearer view (d = 2) projects the longer edge
    np.testing.assert_allclose(r[0], [px / H, np.sqrt(2) * px / H, px / H], rtol=1e-6)


def test_edge_lengths_relative_to_each_views_height():
    tri = np.array([[[0, 0, 0], [0.5, 0, 0], [0, 0.5, 0]]], dtype=np.float32)
    M = _ortho(1.0, 1.0)
    # 100 px tall view: edge 0 is 100/2 * 0.5 = 25 px wide on a 100-wide image -> 0.25;
    # 400 x 50 view: 400/2 * 0.5 = 100 px -> 100 / 50 = 2.0
    r = A.edge_lengths(tri, np.stack([M, M]), [100, 400], [100, 50], 0.1)
    assert r[0, 0] == pytest.approx(2.0, rel=1e-6)


def test_edge_lengths_cull_near_plane_and_off_screen():
    W = H = 64
    tri = np.array([[[0, 0, 1.0], [0.1, 0, 1.0], [0, 0.1, 0.05]],      # a vertex at w = 0.05 < near
                    [[5, 5, 1.0], [5.1, 5, 1.0], [5, 5.1, 1.0]],       # projects far right/up of the image
                    [[0, 0, 1.0], [0.1, 0, 1.0], [0, 0.1, 1.0]]],      # visible
                   dtype=np.float32)
    r = A.edge_lengths(tri, _pinhole(1.0)[None], [W], [H], 0.1)
    assert r[0].tolist() == [0.0, 0.0, 0.0]
    assert r[1].tolist() == [0.0, 0.0, 0.0]
    assert r[2, 0] == pytest.approx(W / 2 * 0.1 / H, rel=1e-6)


# --------------------------------------------------------------------------
# plans
# --------------------------------------------------------------------------

def _rel(longest):
    """[T, 3] lengths with the given longest edge length on edge 1, shorter ones elsewhere."""
    r = np.zeros((len(longest), 3), dtype=np.float32)
    for t, x in enumerate(longest):
        r[t] = [x / 2, x, x / 3]
    return r


def test_plan_split_then_prune_to_budget():
    counts = [5, 0, 3, 0, 9]
    rel = _rel([0.3, 0.1, 0.1, 0.1, 0.1])
    act, off, n = A.plan(counts, rel, 0.2, 4)
    # t0 splits (6 triangles), then the two zero-coverage ones go, lowest index first
    assert act.tolist() == [A.SPLIT0 + 1, A.REMOVE, A.KEEP, A.REMOVE, A.KEEP]
    assert off.tolist() == [0, 2, 2, 3, 3]
    assert n == 4


def test_plan_pruning_takes_the_split_with_it():
    counts = [0, 4, 7]
    rel = _rel([0.5, 0.05, 0.05])
    act, off, n = A.plan(counts, rel, 0.2, 2)
    assert act.tolist() == [A.REMOVE, A.KEEP, A.KEEP] and n == 2
    act, off, n = A.plan(counts, rel, 0.2, 1)
    assert act.tolist() == [A.REMOVE, A.REMOVE, A.KEEP] and n == 1


def test_plan_random_initialisation_prune_zero_then_fill():
    counts = [0, 4, 2, 1]
    rel = _rel([0.9, 0.1, 0.15, 0.01])
    # t0 goes (no coverage) with its split; 3 triangles remain, and fill splits the
    # longest edges first: t2 (0.15) -> 4, t1 (0.1) -> 5 = target, so t3 (0.01) stays
    act, off, n = A.plan(counts, rel, 0.2, 5, prune_zero=True, fill=True)
    assert n == 5
    assert act.tolist() == [A.REMOVE, A.SPLIT0 + 1, A.SPLIT0 + 1, A.KEEP]
    assert off.tolist() == [0, 0, 2, 4]


def test_plan_longest_edge_ties_take_the_lowest_index():
    rel = np.array([[0.3, 0.3, 0.1], [0.1, 0.3, 0.3], [0.3, 0.1, 0.3]], dtype=np.float32)
    act, _, n = A.plan([1, 1, 1], rel, 0.2, 100)
    assert act.tolist() == [A.SPLIT0 + 0, A.SPLIT0 + 1, A.SPLIT0 + 0] and n == 6


def test_plan_threshold_is_strict_in_float32():
    thr = np.float32(0.2)
    rel = np.array([[thr, 0, 0], [np.nextafter(thr, np.float32(1)), 0, 0]], dtype=np.float32)
    act, _, n = A.plan([1, 1], rel, 0.2, 100)
    assert act.tolist() == [A.KEEP, A.SPLIT0] and n == 3


def test_plan_invariants_on_random_input():
    rng = np.random.default_rng(7)
    for trial in range(20):
        T = int(rng.integers(1, 300))
        counts = rng.integers(0, 6, size=T)
        rel = rng.random((T, 3)).astype(np.float32) * 0.4
        target = int(rng.integers(0, 2 * T))
        act, off, n = A.plan(counts, rel, 0.2, target, prune_zero=bool(trial % 2), fill=bool(trial % 3 == 0))
        kids = np.where(act == A.REMOVE, 0, np.where(act == A.KEEP, 1, 2))
        assert off.tolist() == (np.cumsum(kids) - kids).tolist()
        assert n == kids.sum()
        assert n <= target
        # every removed triangle has coverage <= every kept one, unless removed for zero coverage
        if (act == A.REMOVE).any() and (act != A.REMOVE).any():
            assert counts[act == A.REMOVE].max() <= counts[act != A.REMOVE].min()


# --------------------------------------------------------------------------
# applying a plan
# --------------------------------------------------------------------------

def _parent_coords(parent, X):
    """(G-1)-free barycentrics (b1, b2) of 3-D point X in the parent triangle, by least squares."""
    P = parent.astype(np.float64)
    Mx = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)
    sol, *_ = np.linalg.lstsq(Mx, X - P[0], rcond=None)
    return sol


@pytest.mark.parametrize("k", [0, 1, 2])
def test_apply_split_tiles_the_parent_and_keeps_orientation(k):
    rng = np.random.default_rng(k)
    v = rng.standard_normal((1, 3, 3)).astype(np.float32)
    f = rng.standard_normal((1, 4, 4, 2)).astype(np.float32)
    ov, _ = A.apply(v, f, np.array([A.SPLIT0 + k]), np.array([0]), 2)
    P = v[0].astype(np.float64)
    n0 = np.cross(P[1] - P[0], P[2] - P[0])
    mid = 0.5 * (P[k] + P[(k + 1) % 3])
    area = 0.0
    for h in (0, 1):
        Q = ov[h].astype(np.float64)
        nh = np.cross(Q[1] - Q[0], Q[2] - Q[0])
        assert np.dot(nh, n0) > 0                          # same orientation
        np.testing.assert_allclose(nh / np.linalg.norm(nh), n0 / np.linalg.norm(n0), atol=1e-5)
        assert any(np.allclose(q, mid, atol=1e-6) for q in Q)
        assert np.allclose(Q[(k + 2) % 3], P[(k + 2) % 3])  # the opposite vertex stays in its slot
        area += 0.5 * np.linalg.norm(nh)
    np.testing.assert_allclose(area, 0.5 * np.linalg.norm(n0), rtol=1e-5)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_apply_split_reproduces_an_affine_texture(k):
    G, C = 6, 3
    rng = np.random.default_rng(10 + k)
    v = rng.standard_normal((1, 3, 3)).astype(np.float32)
    al, be, ga = rng.standard_normal(C), rng.standard_normal(C), rng.standard_normal(C)
    iy, ix = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")
    f = (al + be * ix[..., None] + ga * iy[..., None])[None].astype(np.float32)
    ov, of = A.apply(v, f, np.array([A.SPLIT0 + k]), np.array([0]), 2)
    checked = 0
    for h in (0, 1):
        Q = ov[h].astype(np.float64)
        for jy in range(G):
            for jx in range(G):
                b1, b2 = jx / (G - 1), jy / (G - 1)
                X = (1 - b1 - b2) * Q[0] + b1 * Q[1] + b2 * Q[2]
                u, w = _parent_coords(v[0], X) * (G - 1)
                if not (-1e-6 <= u <= G - 1 + 1e-6 and -1e-6 <= w <= G - 1 + 1e-6):
                    continue                                  # clamped texels: not affine
                np.testing.assert_allclose(of[h, jy, jx], al + be * u + ga * w, atol=1e-5)
                checked += 1
    assert checked >= G * (G + 1) // 2                        # at least the texels inside each half


def test_apply_keep_and_remove():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, 3, 3)).astype(np.float32)
    f = rng.standard_normal((3, 2, 2, 4)).astype(np.float32)
    ov, of = A.apply(v, f, np.array([A.REMOVE, A.KEEP, A.KEEP]), np.array([0, 0, 1]), 2)
    assert np.array_equal(ov, v[1:])
    assert np.array_equal(of, f[1:].astype(np.float64))
