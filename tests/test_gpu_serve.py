"""GPU checks of the serving loop: a request renders to the same colours
inside a mixed batch (different soups and resolutions in one launch) as
alone, and an open-loop run completes every request with sane latencies."""
import sys

import numpy as np
import pytest

from paper_2603_27151_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def server():
    from paper_2603_27151_amd import raster as R
    from paper_2603_27151_amd import serve as SV
    soups = [R.DeviceScene.from_host(s) for s in W.serving_soups()]
    return SV.Server(soups, tile=16, n_streams=2, max_batch=8, keep_colors=True)


def test_batched_render_equals_alone(server):
    from paper_2603_27151_amd import serve as SV
    reqs = W.serving_requests(200.0, 0.05, seed=77)[:6]
    _say(f"case: {len(reqs)} requests, soups {[r.soup for r in reqs]}, "
         f"sizes {[(r.view.width, r.view.height) for r in reqs]}")
    sched = server.sched
    for i, r in enumerate(reqs):
        sched.submit(SV.Ticket(i, r.soup, r.view, 0.0, server.need(r.soup, r.view)))
    done = []
    while sched.busy:
        done += sched.poll()
    assert len(done) == len(reqs)
    for t in done:
        alone = server.render_alone(t.soup, t.view)
        assert torch.equal(t.color, alone), f"request {t.rid} differs from its lone render"


def test_open_loop_run_completes(server):
    from paper_2603_27151_amd import serve as SV
    reqs = W.serving_requests(100.0, 1.0, seed=5)
    _say(f"case: open loop, {len(reqs)} requests at 100/s")
    st = SV.run(server, reqs)
    _say(st)
    assert st["requests"] == len(reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["p99_ms"] < 1000.0


def test_tuned_tiles_keep_results():
    """With tiles tuned per resolution, a batch renders with the tile of its
    largest request; colours do not depend on the tile side, so every request
    still equals its lone render at the default tile."""
    from paper_2603_27151_amd import raster as R
    from paper_2603_27151_amd import serve as SV
    soups = [R.DeviceScene.from_host(s) for s in W.serving_soups()[:2]]
    srv = SV.Server(soups, tile=None, n_streams=2, max_batch=4, keep_colors=True)
    sizes = [(160, 90), (320, 180)]
    tuned = srv.tune_tiles([W.View(w, h, 0, W.view_proj((0.0, 0.3, 3.0), w, h)) for w, h in sizes], reps=1)
    _say(f"case: tuned tiles {srv.tile_by_res}")
    assert set(srv.tile_by_res) == set(sizes)
    assert all(t in (8, 16, 32) for t in srv.tile_by_res.values())
    assert all(set(e["ms"]) == {"8", "16", "32"} for e in tuned.values())
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(6):
        w, h = sizes[i % 2]
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        reqs.append(SV.Ticket(i, i % 2, W.View(w, h, 100 + i, W.view_proj(3.0 * d, w, h)), 0.0, 0))
    for t in reqs:
        t.need = srv.need(t.soup, t.view)
        srv.sched.submit(t)
    done = []
    while srv.sched.busy:
        done += srv.sched.poll()
    assert len(done) == len(reqs)
    ref = SV.Server(soups, tile=16, n_streams=1, max_batch=1)
    for t in done:
        assert torch.equal(t.color, ref.render_alone(t.soup, t.view)), f"request {t.rid} differs"
