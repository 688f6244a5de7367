"""CPU checks of the boundary and host logic (no compute calls without a GPU).

* libdiffsoup.so loads and exports every function include/diffsoup.h declares;
* the ctypes structs have the C layout the header defines;
* the Python binding fails loudly when the library is missing (no fallback);
* bench.py refuses more than one GPU;
* the input generators are deterministic and have the stated shapes.
"""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diffsoup.h")
LIB = os.path.join(ROOT, "paper_2603_27151_amd", "libdiffsoup.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(soup_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("soup_rasterize_fwd", "soup_rasterize_bwd", "soup_render", "soup_ctx_create",
                 "soup_ctx_destroy", "soup_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (soup_[a-z0-9_]+)", out))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_export():
    from paper_2603_27151_amd import _lib
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_struct_layouts_match_the_header():
    from paper_2603_27151_amd import _lib
    # soup_scene: 4 int32 + 4 pointers
    assert ctypes.sizeof(_lib.soup_scene) == 16 + 4 * 8
    # soup_views: int32 (+pad) + 4 pointers
    assert ctypes.sizeof(_lib.soup_views) == 8 + 4 * 8
    # soup_opts: u64, u32, i32, float[3], i32, float, i32, i32
    assert ctypes.sizeof(_lib.soup_opts) == 48
    assert _lib.soup_opts.accumulate.offset == 36
    assert _lib.soup_opts.reuse_bins.offset == 40
    assert ctypes.sizeof(_lib.soup_stats) == 6 * 8


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2603_27151_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        _lib.lib()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_bench_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    # roofline.traffic comes from the committed FETCH_SIZE / WRITE_SIZE summary, scaled by
    # its copy calibration, and only while the kernel sources hash to the recorded value
    # and the workload and tile side are the profiled ones
    sys.path.insert(0, ROOT)
    import bench
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_batched.txt").write_text(
        "# a summary\ncsrc_sha1: 0123456789abcdef\nworkload: batched\ntile: 16\n"
        "fetch_scale: 2.0\nwrite_scale: 1.0\ndecode_bwd.fetch_kb: 1000\ndecode_bwd.write_kb: 300\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "csrc_sha1", lambda: "0123456789abcdef")
    assert bench.measured_traffic("decode_bwd", "batched", 16) == 1000 * 1024 * 2 + 300 * 1024
    assert bench.measured_traffic("raster_fwd", "batched", 16) is None      # not in the summary
    assert bench.measured_traffic("decode_bwd", "large", 16) is None        # another workload
    assert bench.measured_traffic("decode_bwd", "batched", 8) is None       # another tile side
    monkeypatch.setattr(bench, "csrc_sha1", lambda: "fedcba9876543210")
    assert bench.measured_traffic("decode_bwd", "batched", 16) is None      # the kernels changed


def test_bench_source_hash_follows_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.csrc_sha1()
    assert re.fullmatch(r"[0-9a-f]{16}", h) and bench.csrc_sha1() == h


def test_generators_are_deterministic_and_shaped():
    from paper_2603_27151_amd import workloads as W
    a, b = W.tiny(), W.tiny()
    assert np.array_equal(a.scene.verts, b.scene.verts) and np.array_equal(a.scene.mlp, b.scene.mlp)
    assert a.scene.verts.shape == (64, 3, 3) and a.scene.feats.shape == (64, 4, 4, 8)
    assert a.scene.mlp.size == W.mlp_param_count([8, 16, 4]) == 212
    s = W.single(with_targets=False)
    assert s.scene.feats.shape == (10000, 8, 8, 16) and s.scene.mlp.size == 1732
    side = np.linalg.norm(s.scene.verts[:, 1] - s.scene.verts[:, 0], axis=1)
    assert abs(np.log(side).mean() + 3.0) < 0.02 and abs(np.log(side).std() - 0.5) < 0.02
    assert np.linalg.norm(s.scene.verts.mean(1), axis=1).max() <= 1.0 + 1e-6
    bt = W.batched(with_targets=False, n_views=64, T=1000)
    assert len(bt.views) == 64 and {v.width for v in bt.views} <= set(W.BATCHED_RES)
    assert all(v.width == v.height for v in bt.views)
    eyes = W.fibonacci_sphere(64)
    assert np.allclose(np.linalg.norm(eyes, axis=1), 3.0)
    req = W.serving_requests(200.0, 1.0)
    assert 120 < len(req) < 280 and all(r.view.width in (640, 1280, 1920) for r in req)


def test_camera_projects_origin_to_image_centre():
    from paper_2603_27151_amd import workloads as W
    M = W.view_proj((0.3, -1.2, 2.5), 200, 100).astype(np.float64)
    c = M @ np.array([0, 0, 0, 1.0])
    assert abs(c[0] / c[3]) < 1e-6 and abs(c[1] / c[3]) < 1e-6
