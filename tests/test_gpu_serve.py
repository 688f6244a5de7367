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


def test_request_bytes_bounds_what_a_render_allocates():
    """request_bytes (the admission's per-request charge) against the bytes a
    render really allocates: its colour buffer plus the workspaces it grows
    a fresh context to, for every soup and resolution of the workload."""
    from paper_2603_27151_amd import raster as R
    from paper_2603_27151_amd import serve as SV
    soups = [R.DeviceScene.from_host(s) for s in W.serving_soups()]
    srv = SV.Server(soups, tile=16, n_streams=1, max_batch=1)
    for soup in range(len(soups)):
        for (w, h) in W.SERVING_RES:
            v = W.View(w, h, 3, W.view_proj((0.4, 0.2, 3.0), w, h))
            actual = srv.measure_request(soup, v)
            est = srv.need(soup, v)
            _say(f"soup {soup} ({soups[soup].T} triangles) {w}x{h}: allocated {actual} B, charged {est} B "
                 f"({actual / est:.2f})")
            assert actual <= est
            assert actual >= 0.4 * est


def test_admission_budget_binds_and_results_hold():
    """A budget that fits about two requests: a burst of 24 requests is
    admitted at most two at a time, the charged bytes in flight never exceed
    the budget, and every request still equals its lone render."""
    from paper_2603_27151_amd import raster as R
    from paper_2603_27151_amd import serve as SV
    soups = [R.DeviceScene.from_host(s) for s in W.serving_soups()]
    rng = np.random.default_rng(21)
    views = []
    for i in range(24):
        w, h = W.SERVING_RES[i % 2]                # 640x360 and 1280x720
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        views.append((int(rng.integers(0, len(soups))), W.View(w, h, 500 + i, W.view_proj(3.0 * d, w, h))))
    needs = [SV.request_bytes(v.width, v.height, soups[s].T) for s, v in views]
    budget = int(max(needs) * 2.05)
    srv = SV.Server(soups, tile=16, n_streams=2, max_batch=16, keep_colors=True, budget_bytes=budget)
    _say(f"case: burst of {len(views)} requests, budget {budget} B, largest request {max(needs)} B")
    for i, (s, v) in enumerate(views):
        srv.sched.submit(SV.Ticket(i, s, v, 0.0, srv.need(s, v)))
    done = []
    while srv.sched.busy:
        done += srv.sched.poll()
        assert srv.sched.in_use <= budget
    assert len(done) == len(views)
    sizes = srv.sched.batch_sizes
    _say(f"batches {len(sizes)}, sizes {sizes}, peak in flight {srv.sched.peak_in_flight}, "
         f"peak charged {srv.sched.peak_in_use} B")
    assert srv.sched.peak_in_use <= budget
    assert 2 <= srv.sched.peak_in_flight <= 3       # about two requests' worth at a time
    assert len(sizes) > len(views) / 3              # admission split the burst
    for t in done:
        assert torch.equal(t.color, srv.render_alone(t.soup, t.view)), f"request {t.rid} differs"
