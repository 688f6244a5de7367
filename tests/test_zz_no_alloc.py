"""soup_loss_l1_ssim_noalloc, the entry point for callers that cannot
allocate device memory, against soup_loss_l1_ssim (the same kernels with a
context workspace), through the C ABI: two calls in a row, the second on a
smaller input; the device's free memory does not drop across them; a view
too large for the static scratch is rejected before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)


def _views(_lib, h, sizes):
    n = len(sizes)
    return _lib.make_views(h, np.array([w for w, _ in sizes], np.int32), np.array([hh for _, hh in sizes], np.int32),
                           np.zeros(n, np.uint32), np.tile(np.eye(4, dtype=np.float32), (n, 1, 1)))


def _inputs(rng, sizes):
    P = sum(w * h for w, h in sizes)
    c = torch.from_numpy(rng.random((P, 3)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.random((P, 3)).astype(np.float32)).cuda()
    return c, t


def _outputs(P):
    return (torch.full((P, 3), float("nan"), device="cuda"), torch.full((P,), float("nan"), device="cuda"),
            torch.full((1,), float("nan"), device="cuda"))


def _run(_lib, ctx, fn, c, t, views, lam, out=None):
    gc, gl, loss = out if out is not None else _outputs(c.shape[0])
    fn(ctx, c, t, views, lam, gc, gl, loss)
    return gc, gl, loss


def test_noalloc_loss_matches_the_allocating_entry_point():
    from paper_2603_27151_amd import _lib
    ctx = _lib.Ctx(0)
    rng = np.random.default_rng(5)
    h = _lib._Holder()
    warm = [(8, 8)]
    cases = [([(1000, 1000), (317, 211)], 0.8),   # 1.0 Mpixel view: 48 MB of the 64 MiB scratch
             ([(64, 48), (1, 1), (200, 13)], 0.2)]  # smaller: the scratch keeps the last call's records
    # the kernels' code loaded once before free memory is read
    cw, tw = _inputs(rng, warm)
    _run(_lib, ctx, _lib.soup_loss_l1_ssim_noalloc, cw, tw, _views(_lib, h, warm), 0.8)
    inputs = [(_inputs(rng, sizes), _views(_lib, h, sizes), lam, sizes) for sizes, lam in cases]
    outs = [_outputs(c.shape[0]) for (c, _), _, _, _ in inputs]   # every output before free memory is read
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for ((c, t), views, lam, sizes), out in zip(inputs, outs):
        _say(f"noalloc call: views {sizes}, lambda {lam}")
        _run(_lib, ctx, _lib.soup_loss_l1_ssim_noalloc, c, t, views, lam, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    # the allocating entry point would have taken a 48 MB workspace on this fresh context
    _say(f"device free memory across the calls: {free0} -> {free1}")
    assert free1 == free0
    for ((c, t), views, lam, sizes), got in zip(inputs, outs):
        _say(f"allocating call: views {sizes}, lambda {lam}")
        ref = _run(_lib, ctx, _lib.soup_loss_l1_ssim, c, t, views, lam)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0]), "grad_color differs"
        assert torch.equal(got[1], ref[1]), "grad_logp differs"
        assert float(got[2]) == pytest.approx(float(ref[2]), rel=1e-6)   # float atomics: order may differ
        assert torch.isfinite(got[0]).all() and torch.isfinite(got[1]).all()
    ctx.close()


def test_noalloc_loss_rejects_views_beyond_the_scratch():
    from paper_2603_27151_amd import _lib
    ctx = _lib.Ctx(0)
    h = _lib._Holder()
    sizes = [(1400, 1000)]          # 1.4 Mpixel > 1,398,101
    views = _views(_lib, h, sizes)
    c = torch.zeros((1, 3), device="cuda")   # never read: the call fails before any launch
    gc = torch.zeros((1, 3), device="cuda")
    gl = torch.zeros((1,), device="cuda")
    with pytest.raises(_lib.SoupError, match="static scratch"):
        _lib.soup_loss_l1_ssim_noalloc(ctx, c, c, views, 0.8, gc, gl, None)
    ctx.close()
