"""Exact-arithmetic geometry used by the oracle pins (test-only, independent
of the rasterizer's edge-function formulation).

* ``inside_rational``: point-in-triangle by solving for barycentric
  coordinates with Fractions; a sample exactly on an edge or vertex is
  classified as the point moved by an infinitesimal step along (1, eps),
  eps -> 0+ (the tie rule the rasterizer claims to implement).
* ``pixel_area``: area of a convex polygon inside each unit pixel square
  (Sutherland-Hodgman clipping), i.e. the box-filtered coverage image.
"""
from fractions import Fraction

import numpy as np


def _bary(v, p):
    (x0, y0), (x1, y1), (x2, y2) = v
    px, py = p
    a, b = x1 - x0, x2 - x0
    c, d = y1 - y0, y2 - y0
    det = a * d - b * c
    rx, ry = px - x0, py - y0
    l1 = (d * rx - b * ry) / det
    l2 = (-c * rx + a * ry) / det
    # derivative of (l1, l2) along x and along y
    dl1 = (Fraction(d) / det, Fraction(-b) / det)
    dl2 = (Fraction(-c) / det, Fraction(a) / det)
    l0 = 1 - l1 - l2
    dl0 = (-dl1[0] - dl2[0], -dl1[1] - dl2[1])
    return (l0, l1, l2), (dl0, dl1, dl2)


def _positive_after_nudge(val, grad):
    if val != 0:
        return val > 0
    if grad[0] != 0:
        return grad[0] > 0
    return grad[1] > 0


def inside_rational(v, p):
    """v: three (x, y) Fractions/ints, p: (x, y). Non-degenerate triangle."""
    lam, dlam = _bary(v, p)
    return all(_positive_after_nudge(l, g) for l, g in zip(lam, dlam))


def coverage_rational(v, width, height, snap=256):
    """Set of (x, y) pixels whose centre is covered; v in 1/snap units (ints)."""
    vf = [(Fraction(x, snap), Fraction(y, snap)) for x, y in v]
    xs = [p[0] for p in vf]
    ys = [p[1] for p in vf]
    out = set()
    for y in range(max(0, int(min(ys)) - 1), min(height, int(max(ys)) + 2)):
        for x in range(max(0, int(min(xs)) - 1), min(width, int(max(xs)) + 2)):
            if inside_rational(vf, (Fraction(2 * x + 1, 2), Fraction(2 * y + 1, 2))):
                out.add((x, y))
    return out


def _clip(poly, inside, inter):
    out = []
    n = len(poly)
    for i in range(n):
        cur, prev = poly[i], poly[i - 1]
        ci, pi = inside(cur), inside(prev)
        if ci:
            if not pi:
                out.append(inter(prev, cur))
            out.append(cur)
        elif pi:
            out.append(inter(prev, cur))
    return out


def clip_halfplane(poly, a, b, c):
    """Keep a*x + b*y + c >= 0."""
    f = lambda p: a * p[0] + b * p[1] + c

    def inter(p, q):
        t = f(p) / (f(p) - f(q))
        return (p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1]))

    return _clip(poly, lambda p: f(p) >= 0, inter)


def area(poly):
    if len(poly) < 3:
        return 0.0
    s = 0.0
    for i in range(len(poly)):
        x0, y0 = poly[i - 1]
        x1, y1 = poly[i]
        s += x0 * y1 - x1 * y0
    return abs(s) / 2.0


def pixel_area(poly, width, height):
    """[H, W] float64 image: area of the polygon inside each pixel square."""
    img = np.zeros((height, width))
    if len(poly) < 3:
        return img
    xs = [p[0] for p in poly]
    ys = [p[1] for p in poly]
    for y in range(max(0, int(np.floor(min(ys)))), min(height, int(np.ceil(max(ys))) + 1)):
        band = clip_halfplane(poly, 0, 1, -y)
        band = clip_halfplane(band, 0, -1, y + 1)
        if len(band) < 3:
            continue
        for x in range(max(0, int(np.floor(min(xs)))), min(width, int(np.ceil(max(xs))) + 1)):
            cell = clip_halfplane(band, 1, 0, -x)
            cell = clip_halfplane(cell, -1, 0, x + 1)
            img[y, x] = area(cell)
    return img
