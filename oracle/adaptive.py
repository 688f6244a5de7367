"""CPU oracle of the adaptive control of primitives.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline import this module; the library never does.

Section 3.4 ("Adaptive control of primitives"): every so many iterations,
edges whose projected length exceeds a fraction of the image height (1/5)
on a sample of training views are split, and triangles with the lowest
pixel coverage over the training views are pruned until the triangle budget
holds. Supplement B (initialisation from random triangles): triangles that
cover no pixel are removed first, then the longest edges are split until the
count reaches the target.

Readings (the paper leaves these open):
  * pixel coverage of a triangle = number of pixels whose visibility key
    names it as the winner, summed over the views given;
  * an edge's length is its screen-space length in pixels divided by that
    view's height, maximised over the views in which the triangle is in
    front of the near plane (every vertex at clip w >= near_w, the
    rasterizer's own cull) and its screen bounding box meets the image;
  * a triangle splits at most once per plan, on its longest edge (lowest
    edge index among equal lengths), at the edge's midpoint; the two halves
    keep the parent's vertex order;
  * pruning removes triangles in order of (coverage, index) ascending; a
    removed triangle takes its planned split with it;
  * the texture of a half is the parent's G x G grid resampled bilinearly at
    the half's texel positions mapped into the parent's barycentrics (the
    mapping sends texel (ix, iy) of the half to grid coordinates that are
    multiples of 1/2 in the parent, so the resampling weights are exact).

Plain numpy; float64 geometry; loops where the definition is a loop.
"""
from __future__ import annotations

import numpy as np

BG_KEY = 0xFFFFFFFFFFFFFFFF

REMOVE, KEEP, SPLIT0 = 0, 1, 2  # action codes; SPLIT0 + k splits edge k (vertex k to vertex (k+1) mod 3)


def coverage_counts(vis: np.ndarray, T: int) -> np.ndarray:
    """Pixels won per triangle: the low 32 bits of a visibility key are the
    winner's triangle index (the key is depth bits << 32 | triangle, Eq. (1)'s
    nearest passing fragment); background keys and indices >= T are skipped."""
    v = np.asarray(vis, dtype=np.uint64).ravel()
    ids = (v[v != np.uint64(BG_KEY)] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    ids = ids[ids < T]
    counts = np.zeros(T, dtype=np.int64)
    for t in ids:  # the definition: one count per pixel
        counts[t] += 1
    return counts


def _project(M: np.ndarray, p: np.ndarray):
    """Clip coordinates of point p under the row-major 4x4 M, each row's dot
    product summed left to right in float64 (products of float32 values are
    exact in float64)."""
    M = M.astype(np.float64)
    x, y, z = (float(np.float64(c)) for c in p)
    out = []
    for r in range(4):
        acc = M[r, 0] * x
        acc = acc + M[r, 1] * y
        acc = acc + M[r, 2] * z
        acc = acc + M[r, 3]
        out.append(acc)
    return out


def edge_lengths(verts: np.ndarray, view_proj: np.ndarray, width, height, near_w: float) -> np.ndarray:
    """[T, 3] float32: for edge k of triangle t (vertex k to vertex (k+1) mod 3)
    the largest screen-space length in units of the image height over the
    views where the triangle is in front of the near plane and its screen
    bounding box meets the image; 0 where no view qualifies.
    Screen x = W/2 (c_x/c_w + 1), y = H/2 (1 - c_y/c_w) (the rasterizer's
    projection)."""
    verts = np.asarray(verts, dtype=np.float32).reshape(-1, 3, 3)
    T = verts.shape[0]
    V = len(width)
    best = np.zeros((T, 3), dtype=np.float64)
    for v in range(V):
        M = np.asarray(view_proj, dtype=np.float32).reshape(V, 4, 4)[v]
        W, H = float(width[v]), float(height[v])
        for t in range(T):
            clip = [_project(M, verts[t, i]) for i in range(3)]
            if any(c[3] < float(np.float32(near_w)) for c in clip):
                continue
            sx = [W / 2 * (c[0] / c[3] + 1.0) for c in clip]
            sy = [H / 2 * (1.0 - c[1] / c[3]) for c in clip]
            if max(sx) < 0.0 or min(sx) > W or max(sy) < 0.0 or min(sy) > H:
                continue
            for k in range(3):
                j = (k + 1) % 3
                d = np.sqrt((sx[j] - sx[k]) ** 2 + (sy[j] - sy[k]) ** 2) / H
                best[t, k] = max(best[t, k], d)
    return best.astype(np.float32)


def plan(counts, rel_len, split_frac: float, target: int, prune_zero: bool = False, fill: bool = False):
    """Actions, output offsets and the new triangle count.

    1. split every triangle whose longest edge exceeds split_frac (compared in
       float32) on that edge;
    2. with prune_zero, remove every triangle of zero coverage;
    3. remove triangles by (coverage, index) ascending while the count after
       the splits exceeds target;
    4. with fill, split kept, unsplit triangles by (longest edge descending,
       index ascending) while the count is below target.
    Returns (actions int32 [T], offsets int32 [T], n_new)."""
    counts = np.asarray(counts, dtype=np.int64)
    T = counts.shape[0]
    rel = np.asarray(rel_len, dtype=np.float32).reshape(T, 3)
    thr = np.float32(split_frac)
    longest = [0] * T
    for t in range(T):
        k = 0
        for e in (1, 2):
            if rel[t, e] > rel[t, k]:
                k = e
        longest[t] = k
    split = [bool(rel[t, longest[t]] > thr) for t in range(T)]
    removed = [False] * T
    if prune_zero:
        for t in range(T):
            if counts[t] == 0:
                removed[t] = True
                split[t] = False
    n = sum((2 if split[t] else 1) for t in range(T) if not removed[t])
    for t in sorted(range(T), key=lambda t: (counts[t], t)):
        if n <= target:
            break
        if removed[t]:
            continue
        n -= 2 if split[t] else 1
        removed[t] = True
        split[t] = False
    if fill:
        cand = [t for t in range(T) if not removed[t] and not split[t]]
        cand.sort(key=lambda t: (-float(rel[t, longest[t]]), t))
        for t in cand:
            if n >= target:
                break
            split[t] = True
            n += 1
    actions = np.zeros(T, dtype=np.int32)
    offsets = np.zeros(T, dtype=np.int32)
    o = 0
    for t in range(T):
        offsets[t] = o
        if removed[t]:
            actions[t] = REMOVE
        elif split[t]:
            actions[t] = SPLIT0 + longest[t]
            o += 2
        else:
            actions[t] = KEEP
            o += 1
    assert o == n
    return actions, offsets, n


def _half_slots(k: int, half: int):
    """Parent barycentric vectors of the three vertex slots of one half of a
    triangle split on edge k: half 0 keeps vertex k and replaces vertex k+1
    by the edge midpoint; half 1 replaces vertex k by the midpoint."""
    P = np.eye(3)
    a, b = k, (k + 1) % 3
    mid = 0.5 * (P[a] + P[b])
    if half == 0:
        P[b] = mid
    else:
        P[a] = mid
    return P


def _bilinear(grid: np.ndarray, u: float, v: float) -> np.ndarray:
    """The rasterizer's fetch on a G x G x C grid at grid coordinates (u, v):
    cell (floor, clamped to G-2), weights from the fractions."""
    G = grid.shape[0]
    ix = min(max(int(np.floor(u)), 0), G - 2)
    iy = min(max(int(np.floor(v)), 0), G - 2)
    fx, fy = u - ix, v - iy
    g = grid.astype(np.float64)
    return ((1 - fx) * (1 - fy) * g[iy, ix] + fx * (1 - fy) * g[iy, ix + 1]
            + (1 - fx) * fy * g[iy + 1, ix] + fx * fy * g[iy + 1, ix + 1])


def apply(verts, feats, actions, offsets, n_new: int):
    """The new soup: kept triangles copied, split triangles replaced by their
    two halves (vertices at the exact edge midpoint, textures resampled).
    Returns (verts float32 [n_new,3,3], feats float64 [n_new,G,G,C])."""
    verts = np.asarray(verts, dtype=np.float32).reshape(-1, 3, 3)
    feats = np.asarray(feats, dtype=np.float32)
    T, G, _, C = feats.shape
    ov = np.zeros((n_new, 3, 3), dtype=np.float32)
    of = np.zeros((n_new, G, G, C), dtype=np.float64)
    for t in range(T):
        a, o = int(actions[t]), int(offsets[t])
        if a == REMOVE:
            continue
        if a == KEEP:
            ov[o] = verts[t]
            of[o] = feats[t]
            continue
        k = a - SPLIT0
        for half in (0, 1):
            P = _half_slots(k, half)
            ov[o + half] = (P @ verts[t].astype(np.float64)).astype(np.float32)
            for iy in range(G):
                for ix in range(G):
                    b = np.array([G - 1 - ix - iy, ix, iy], dtype=np.float64)  # (G-1) x barycentrics
                    pb = b @ P                                                  # (G-1) x parent barycentrics
                    u = min(max(pb[1], 0.0), G - 1.0)
                    v = min(max(pb[2], 0.0), G - 1.0)
                    of[o + half, iy, ix] = _bilinear(feats[t], u, v)
    return ov, of
