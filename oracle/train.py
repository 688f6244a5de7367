"""CPU oracle of the training step around the rasterizer.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline import this module; the library never does.

* Photometric loss (Section 3.4, "Loss function"): lambda L1 + (1 - lambda)
  L_SSIM with lambda = 0.8, evaluated on the stochastic rendering. Readings:
  L1 = mean over pixels and channels of |C - T|; L_SSIM = 1 - mean over
  pixels and channels of the SSIM map of Wang et al. (2004) with an 11 x 11
  Gaussian window of standard deviation 1.5, C1 = 0.01^2, C2 = 0.03^2, the
  local statistics taken per channel with zero padding at the image border
  (the window is not renormalised there). The per-pixel weight of the score
  term is pixel p's share of the loss,
      g_L(p) = [lambda sum_c |C - T| + (1 - lambda) sum_c (1 - S_c(p))] / (3P),
  so that the weights of all pixels sum to the loss (as for the L2 loss).
  Its colour gradient: the L1 part is lambda sign(C - T) / (3P) (0 where
  C = T); the SSIM part is taken by torch's autograd in float64 through the
  direct definition below.
* Optimisers (Section 3.4 and Supplement "Hyperparameters"): Adam (Kingma
  and Ba 2015) for features and MLP weights, VectorAdam (Ling et al. 2022)
  for vertex positions: the second moment of a vertex is the running mean
  of the squared norm of its 3-vector gradient, shared by its three
  coordinates. beta1 = 0.9, beta2 = 0.999, eps = 1e-8; bias-corrected
  moments; the learning rate decays exponentially to 1/100 over training.

float64 throughout.
"""
from __future__ import annotations

import math

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WIN = 11
SIGMA = 1.5


def gaussian_window() -> np.ndarray:
    """11 x 11 window: the outer product of the normalised 1-D Gaussian."""
    x = np.arange(WIN, dtype=np.float64) - WIN // 2
    g = np.exp(-x * x / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def _filter(img: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Window-weighted local sum at every pixel of a 2-D map, zero outside."""
    H, Wd = img.shape
    r = WIN // 2
    pad = np.zeros((H + 2 * r, Wd + 2 * r))
    pad[r:r + H, r:r + Wd] = img
    out = np.zeros((H, Wd))
    for dy in range(WIN):
        for dx in range(WIN):
            out += w[dy, dx] * pad[dy:dy + H, dx:dx + Wd]
    return out


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """[H, W, 3] images -> [H, W, 3] SSIM map (per channel)."""
    w = gaussian_window()
    out = np.zeros(x.shape, dtype=np.float64)
    for c in range(x.shape[2]):
        a = x[..., c].astype(np.float64)
        b = y[..., c].astype(np.float64)
        mx, my = _filter(a, w), _filter(b, w)
        sxx = _filter(a * a, w) - mx * mx
        syy = _filter(b * b, w) - my * my
        sxy = _filter(a * b, w) - mx * my
        out[..., c] = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return out


def loss_l1_ssim(colors, targets, lam: float = 0.8):
    """colors, targets: lists of [H, W, 3] images (the views of one step).
    Returns (loss, grad_color [P, 3], grad_logp [P]) with pixels of all views
    concatenated in order, row-major."""
    import torch
    P = sum(c.shape[0] * c.shape[1] for c in colors)
    n = 3.0 * P
    loss = 0.0
    gcs, gls = [], []
    w = torch.from_numpy(gaussian_window())
    for col, tgt in zip(colors, targets):
        x = torch.tensor(np.asarray(col, np.float64), requires_grad=True)
        y = torch.from_numpy(np.asarray(tgt, np.float64))
        d = x - y
        l1 = d.abs()
        # SSIM through the same definition, differentiable
        S = []
        for c in range(3):
            a, b = x[..., c][None, None], y[..., c][None, None]
            k = w[None, None]
            f = lambda z: torch.nn.functional.conv2d(z, k, padding=WIN // 2)[0, 0]
            mx, my = f(a), f(b)
            sxx = f(a * a) - mx * mx
            syy = f(b * b) - my * my
            sxy = f(a * b) - mx * my
            S.append(((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2)))
        S = torch.stack(S, dim=-1)
        part = lam * l1.sum() + (1.0 - lam) * (1.0 - S).sum()
        part = part / n
        # the L1 part's gradient is lam sign(d) / (3P); autograd gives the SSIM part
        ((1.0 - lam) * (1.0 - S).sum() / n).backward()
        g = x.grad.numpy() + lam * np.sign(d.detach().numpy()) / n
        gl = (lam * l1.detach().numpy().sum(-1) + (1.0 - lam) * (1.0 - S.detach().numpy()).sum(-1)) / n
        loss += float(part)
        gcs.append(g.reshape(-1, 3))
        gls.append(gl.reshape(-1))
    return loss, np.concatenate(gcs), np.concatenate(gls)


def adam(p, g, m, v, lr: float, t: int, b1=0.9, b2=0.999, eps=1e-8, vec: int = 1):
    """One Adam (vec = 1) or VectorAdam (vec = 3) step at iteration t >= 1.
    p, g, m: [n]; v: [n / vec]. Returns new (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    g2 = (g * g).reshape(-1, vec).sum(axis=1)
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g2
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    p = p - lr * mhat / (np.repeat(np.sqrt(vhat), vec) + eps)
    return p, m, v


def lr_at(lr0: float, t: int, iters: int) -> float:
    """Exponential decay to lr0 / 100 at the last iteration (t = 0 .. iters-1)."""
    if iters <= 1:
        return lr0
    return lr0 * math.pow(0.01, t / (iters - 1))
