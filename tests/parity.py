"""Comparison rules of the GPU parity tests (the bar the HIP path is held to
against the oracle).

* visibility buffer: bit-exact;
* colours: |gpu - ref| <= 1e-5 max(|ref|, 1e-3) element by element;
* gradients: each tensor within 1e-4 normwise (||gpu - ref|| / ||ref||) AND
  every element within |gpu_i - ref_i| <= 1e-4 |ref_i| + 1e-6 max|ref|.
  The second term is the float32 summation floor: an element that is a sum
  of many terms of both signs keeps about 1e-7 of the largest term as
  rounding noise, so an element far below the tensor's scale cannot be held
  to 1e-4 of itself.
"""
import sys

import numpy as np

GRAD_RTOL = 1e-4
GRAD_FLOOR = 1e-6
COLOUR_RTOL = 1e-5


def say(tag, *a):
    print(f"[{tag}]", *a, flush=True)
    sys.stdout.flush()


def normwise(gpu, ref):
    gpu = np.asarray(gpu, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    den = np.linalg.norm(ref)
    if den == 0:
        return float(np.linalg.norm(gpu))
    return float(np.linalg.norm(gpu - ref) / den)


def grad_violations(gpu, ref, rtol=GRAD_RTOL, floor=GRAD_FLOOR):
    """Indices (flat) of elements outside |d_i| <= rtol |r_i| + floor max|r|."""
    g = np.asarray(gpu, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    if r.size == 0:
        return np.zeros(0, np.int64), 0.0
    scale = float(np.abs(r).max())
    bound = rtol * np.abs(r) + floor * scale
    d = np.abs(g - r)
    bad = np.flatnonzero(~(d <= bound))
    worst = float((d / np.maximum(bound, 1e-300)).max())
    return bad, worst


def assert_grads(gpu, ref, tol=GRAD_RTOL, names=("verts", "feats", "mlp"), tag="parity"):
    bad = []
    for n, g, r in zip(names, gpu, ref):
        e = normwise(g, r)
        g64 = np.asarray(g, np.float64).ravel()
        r64 = np.asarray(r, np.float64).ravel()
        mx = float(np.max(np.abs(g64 - r64))) if r64.size else 0.0
        idx, worst = grad_violations(g64, r64, tol)
        say(tag, f"grad {n}: normwise {e:.3e} max-abs {mx:.3e} |ref| {np.linalg.norm(r64):.3e} "
                 f"element bound use {worst:.3f} ({idx.size} of {r64.size} outside)")
        if not e <= tol:
            bad.append(f"grad_{n} normwise error {e:.3e} > {tol} (max-abs {mx:.3e})")
        if idx.size:
            i = int(idx[np.argmax(np.abs(g64[idx] - r64[idx]))])
            bad.append(f"grad_{n}: {idx.size} elements outside {tol}|ref| + {GRAD_FLOOR} max|ref| "
                       f"(worst at {i}: gpu {g64[i]:.6e} ref {r64[i]:.6e})")
    assert not bad, "; ".join(bad)


def assert_colours(gpu, ref, rtol=COLOUR_RTOL):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-3)
    assert err.max() <= rtol, f"colour relative error {err.max():.3e}"
