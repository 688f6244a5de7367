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
