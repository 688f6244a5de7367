"""Small hand-built scenes for the tests (inputs only, no rasterizer math).

``ortho_view`` is a camera whose matrix is the identity: clip = (x, y, z, 1),
so screen x = W/2 (x + 1), screen y = H/2 (1 - y) and depth01 = (z + 1) / 2.
With dyadic vertex coordinates every float32 operation of the projection is
exact, so a test can place vertices on exact subpixel positions.
"""
import numpy as np

from paper_2603_27151_amd import workloads as W


def ortho_view(width, height, view_id=0):
    return W.View(width, height, view_id, np.eye(4, dtype=np.float32))


def screen_to_world(sx, sy, width, height):
    """Inverse of the ortho camera's mapping (exact for dyadic inputs)."""
    return sx / (width / 2.0) - 1.0, 1.0 - sy / (height / 2.0)


def tri_world(pts_screen, z, width, height):
    """[3,3] float32 world triangle from three screen (x, y) points and depths z."""
    out = np.zeros((3, 3), np.float32)
    for i, (sx, sy) in enumerate(pts_screen):
        x, y = screen_to_world(sx, sy, width, height)
        out[i] = (x, y, z[i] if np.ndim(z) else z)
    return out


def passthrough_scene(tris, G=4, C=8, logit=None, rgb_logits=None):
    """Scene whose MLP passes features through: opacity logit = feature 0,
    RGB logits = features 1..3, constant over each triangle's grid."""
    tris = np.asarray(tris, np.float32).reshape(-1, 3, 3)
    T = tris.shape[0]
    feats = np.zeros((T, G, G, C), np.float32)
    if logit is not None:
        feats[..., 0] = np.asarray(logit, np.float32).reshape(T, 1, 1)
    if rgb_logits is not None:
        feats[..., 1:4] = np.asarray(rgb_logits, np.float32).reshape(T, 1, 1, 3)
    return W.Scene(verts=tris, feats=feats, mlp=W.passthrough_mlp(C, 16), dims=[C, 16, 4])


def logit(p):
    return float(np.log(p) - np.log1p(-p))
