"""The measured-ceiling probes leave exact results: a copy is the source, a
read sums it, the scattered atomics land where their hash sends them, and
the FMA and matrix-core chains end at their closed forms."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-probe]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2603_27151_amd import _lib
    c = _lib.Ctx(0)
    yield c
    c.close()


def test_copy_and_read(ctx):
    from paper_2603_27151_amd import _lib
    g = torch.Generator().manual_seed(3)
    n = (1 << 20) + 4 * 37                    # a ragged tail past the four-per-step loop
    src = torch.rand(n, generator=g).cuda()
    dst = torch.empty_like(src)
    _say("case: copy and read of", n, "floats")
    _lib.soup_probe_copy(ctx, src, dst)
    ones = torch.ones(n, device="cuda")
    partial = torch.zeros(8192, device="cuda")
    _lib.soup_probe_read(ctx, ones, partial)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert float(partial.double().sum()) == n   # per-workgroup sums of ones are exact


def test_scattered_atomics_land_by_their_hash(ctx):
    from paper_2603_27151_amd import _lib
    n_slots, n_ops = 1009, 250_003
    slots = torch.zeros(n_slots, device="cuda")
    _say("case: atomics", n_ops, "ops into", n_slots, "slots")
    _lib.soup_probe_atomic(ctx, slots, n_ops)
    torch.cuda.synchronize()
    k = np.arange(n_ops, dtype=np.uint64)
    want = np.bincount(((k * np.uint64(2654435761)) % np.uint64(n_slots)).astype(np.int64), minlength=n_slots)
    assert np.array_equal(slots.cpu().numpy(), want.astype(np.float32))


def test_fma_and_mfma_chains_end_at_their_closed_forms(ctx):
    from paper_2603_27151_amd import _lib
    out = torch.zeros(256 * 6, device="cuda")
    _lib.soup_probe_fma(ctx, out, 1000)
    torch.cuda.synchronize()
    assert torch.all(out == 8 * 1000 + 28)
    out2 = torch.zeros(256 * 3, device="cuda")
    _lib.soup_probe_mfma(ctx, out2, 100)
    torch.cuda.synchronize()
    assert torch.all(out2 == 64 * 100)


def test_bad_arguments_are_rejected(ctx):
    from paper_2603_27151_amd import _lib
    with pytest.raises(_lib.SoupError):
        _lib.soup_probe_fma(ctx, torch.zeros(100, device="cuda"), 10)   # not a multiple of 256 threads
    with pytest.raises(_lib.SoupError):
        _lib.soup_probe_atomic(ctx, torch.zeros(0, device="cuda"), 10)
