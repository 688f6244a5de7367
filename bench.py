"""Benchmark of one differentiable rasterization step on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
soup_rasterize_fwd (setup, tile binning, raster with stochastic opacity
masking, winner shading) -> soup_loss_l2 (L2 against a random target) ->
soup_rasterize_bwd (setup and bins recomputed, front-set replay with colour
and score gradients, edge term, vertex chain, MLP-gradient reduction), all on
one stream with inputs resident in HBM.

Workload (default): the batched configuration -- 50,000 triangles (centres
uniform in the unit ball, equilateral, side exp(N(-3, 0.5^2))), 8x8x16
features, MLP 16->32->32->4, 64 views on a Fibonacci sphere of radius 3 with
resolutions drawn from {256, 512, 800, 1024}^2, all views in one call.

The tile size is autotuned (every candidate runs the step), the step is run
eagerly with per-kernel HIP events recorded on its stream (the per-kernel
times and the roofline of the dominant kernel come from these steps), then
captured once into a HIP graph in static-capacity mode and replayed: the
timed steps of the metric are graph replays (--no-graph times eager calls).

Prints ONE JSON line. Besides the metric it reports the per-view path (a host
loop over the 64 views on the same GPU), the roofline of the dominant kernel
and the CPU oracle timed on a bounded sample on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published fp32 vector peak (packed FMA)
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X published dense fp32 matrix-core peak
PEAK_HBM_GBS = 8000.0
# non-packed fp32 FMA: 256 CUs x 4 SIMD16 x 16 lanes x 2 FLOP x 2.4 GHz (the library disables packed fp32)
PEAK_FP32_NON_PACKED_TFLOPS = 78.6


def mlp_macs(dims):
    return int(sum(i * o for i, o in zip(dims[:-1], dims[1:])))


def csrc_sha1() -> str:
    """Hash of the kernel sources (matches profiles/traffic_batched.txt when unchanged)."""
    import hashlib
    root = os.path.join(ROOT, "paper_2603_27151_amd", "csrc")
    h = hashlib.sha1()
    for f in sorted(f for f in os.listdir(root) if f.endswith((".hip", ".hpp"))):
        h.update(f.encode())
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, tile: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, scaled by its copy-kernel calibration; None when the
    kernel sources changed since the counters were taken, or when the summary
    covers another workload or tile side."""
    path = os.path.join(ROOT, "profiles", "traffic_batched.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("csrc_sha1") != csrc_sha1() or f"{kernel}.fetch_kb" not in kv:
        return None
    if kv.get("workload") != workload or kv.get("tile") != str(tile):
        return None
    return int(float(kv[f"{kernel}.fetch_kb"]) * 1024 * float(kv["fetch_scale"]) +
               float(kv[f"{kernel}.write_kb"]) * 1024 * float(kv["write_scale"]))


class Step:
    """One step of the hot path on one stream, into preallocated buffers:
    soup_rasterize_fwd (keeping its tile lists and fragment log) ->
    soup_loss_l2 -> soup_rasterize_bwd (reusing both). The same object is
    run eagerly, in static-capacity mode and under HIP-graph capture."""

    def __init__(self, R, ctx, ds, vs, target, seed, step=0):
        import torch
        self.R, self.ctx, self.ds, self.vs, self.target = R, ctx, ds, vs, target
        dev = ds.verts.device
        P = vs.pixels
        self.opts = R.Opts(seed=seed, step=step, reuse_bins=1)
        self.vis = torch.empty(P, dtype=torch.int64, device=dev)
        self.color = torch.empty(P, 3, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.gc = torch.empty(P, 3, dtype=torch.float32, device=dev)
        self.gl = torch.empty(P, dtype=torch.float32, device=dev)
        self.gv = torch.empty_like(ds.verts)
        self.gf = torch.empty_like(ds.feats)
        self.gm = torch.empty_like(ds.mlp)

    def __call__(self):
        R, ctx = self.R, self.ctx
        R.rasterize_fwd(self.ds, self.vs, self.opts, ctx=ctx, out=(self.vis, self.color, None))
        R.loss_l2(self.color, self.target, ctx=ctx, out=(self.loss, self.gc, self.gl))
        R.rasterize_bwd(self.ds, self.vs, self.opts, self.vis, self.color, self.gc, self.gl, ctx=ctx,
                        out=(self.gv, self.gf, self.gm))

    def capture(self, log=None):
        """Static-capacity mode, then one HIP-graph capture of the step; returns
        the graph (static mode stays on until the caller turns it off). A
        static step that overflows the workspaces sized by the eager calls is
        rerun eagerly (which grows them) and tried again."""
        import torch
        from paper_2603_27151_amd import _lib
        for attempt in range(3):
            self.ctx.set_static(True)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                self()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            try:
                self.ctx.check_overflow()
                break
            except _lib.SoupError as e:
                if log:
                    log(f"static step overflowed ({e}); growing the workspaces")
                self.ctx.set_static(False)
                self()
                torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self()
        return g


class PStep(Step):
    """One step of the paper form (Section 3.3; Supplement B.3, B.6) on one
    stream: soup_mc_assemble (levels Rmin..Rmax-1 onto the level-Rmax grid)
    -> soup_pforward (opacity-texture mask, deferred shading) ->
    soup_loss_l1_ssim (the paper's loss) -> soup_pbackward_levels (the
    backward with the assembly's restriction folded in), into preallocated
    buffers; with fused=False the last call is soup_pbackward followed by
    soup_mc_assemble_bwd through a texture-sized gradient."""

    def __init__(self, R, ctx, wl, target, dev, fused=True):
        import torch
        self.R, self.ctx, self.wl, self.target, self.fused = R, ctx, wl, target, fused
        lv = wl.levels
        self.Rmin, self.Rmax = lv.Rmin, lv.Rmax
        self.raw = [torch.from_numpy(r).to(dev) for r in lv.raw]
        self.graw = [torch.empty_like(r) for r in self.raw]
        T = wl.T
        tex = torch.empty(T, R.mc_vertices(lv.Rmax), 8, dtype=torch.float32, device=dev)
        self.ds = R.PDeviceScene(torch.from_numpy(wl.verts).to(dev), tex, torch.from_numpy(wl.mlp).to(dev), lv.Rmax)
        self.vs = R.Views.from_list(wl.views)
        self.minv = R.inv_view_proj(self.vs)
        P = self.vs.pixels
        self.opts = R.Opts(seed=wl.seed, step=wl.step, reuse_bins=1)
        self.vis = torch.empty(P, dtype=torch.int64, device=dev)
        self.color = torch.empty(P, 3, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.gc = torch.empty(P, 3, dtype=torch.float32, device=dev)
        self.gl = torch.empty(P, dtype=torch.float32, device=dev)
        self.gv = torch.empty_like(self.ds.verts)
        self.gt = torch.empty_like(tex)
        self.gm = torch.empty_like(self.ds.mlp)

    def __call__(self):
        R, ctx = self.R, self.ctx
        R.mc_assemble(self.raw, self.Rmin, self.Rmax, out=self.ds.tex, ctx=ctx)
        R.pforward(self.ds, self.vs, self.opts, minv=self.minv, ctx=ctx, out=(self.vis, self.color, None))
        R.loss_l1_ssim(self.color, self.target, self.vs, 0.8, ctx=ctx, out=(self.loss, self.gc, self.gl))
        self.backward()

    def backward(self):
        R, ctx = self.R, self.ctx
        if self.fused:
            R.pbackward_levels(self.ds, self.vs, self.opts, self.vis, self.color, self.gc, self.Rmin, len(self.raw),
                               grad_logp=self.gl, minv=self.minv, ctx=ctx, out=(self.gv, self.graw, self.gm))
        else:
            R.pbackward(self.ds, self.vs, self.opts, self.vis, self.color, self.gc, self.gl, minv=self.minv, ctx=ctx,
                        out=(self.gv, self.gt, self.gm))
            R.mc_assemble_bwd(self.ds.tex, self.gt, self.Rmin, len(self.raw), self.Rmax, out=self.graw, ctx=ctx)


def paper_form_bench(args, R, W, dev, timed):
    """The paper form's training step at the paper's second stage (levels
    2..4 onto level 5, 561 grid vertices per triangle) on four 800 x 800
    views of a 50,000-triangle soup: step time, per-kernel times, counts and
    the roofline of its dominant kernel."""
    import torch
    wl = W.paper()
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).to(dev)
    ctx = R._lib.Ctx(0)
    ctx.set_tile(16)
    st = PStep(R, ctx, wl, target, dev)
    for _ in range(max(2, args.warmup)):
        st()
    torch.cuda.synchronize()
    ctx.set_counting(True)
    R.pforward(st.ds, st.vs, st.opts, minv=st.minv, ctx=ctx, out=(st.vis, st.color, None))
    sf = ctx.stats()
    R.loss_l1_ssim(st.color, st.target, st.vs, 0.8, ctx=ctx, out=(st.loss, st.gc, st.gl))
    st.backward()
    ctx.set_counting(False)
    torch.cuda.synchronize()
    P = st.vs.pixels
    winners = int((st.vis != -1).sum().item())
    # the paper form's kernels under the timing kinds they share with the workloads' form
    names = {"decode_bwd": "winner_bwd", "grad_reduce": "score", "mlp_reduce": "reduce"}
    # the unfused backward (texture gradient through HBM, then the assembly's
    # backward) for comparison: eager with per-kernel times, and graph replays
    # (an eager call that synchronises now and then blocks for tens of
    # milliseconds; replays have no host synchronisation)
    st.fused = False
    st()
    ctx.read_timings()
    ctx.set_timing(True)
    unfused_ms = timed(st, args.steps)
    ctx.set_timing(False)
    kern_u = ctx.read_timings()
    per_kernel_u = {names.get(k, k): (v[0] / v[1] if v[1] else 0.0) for k, v in kern_u.items()}
    unfused_graph_ms = None
    if not args.no_graph:
        gu = st.capture(log)
        gu.replay()
        torch.cuda.synchronize()
        ctx.check_overflow()
        unfused_graph_ms = timed(gu.replay, args.steps)
        ctx.check_overflow()
        ctx.set_static(False)
        del gu
    st.fused = True
    st()
    ctx.read_timings()
    ctx.set_timing(True)
    eager_ms = timed(st, args.steps)
    ctx.set_timing(False)
    kern = ctx.read_timings()
    per_kernel = {names.get(k, k): (v[0] / v[1] if v[1] else 0.0) for k, v in kern.items()}
    ms, graph = eager_ms, False
    if not args.no_graph:
        ref = st.vis.clone()
        g = st.capture(log)
        g.replay()
        torch.cuda.synchronize()
        ctx.check_overflow()
        if not torch.equal(st.vis, ref):
            raise RuntimeError("paper-form graph replay changed the visibility buffer")
        ms = timed(g.replay, args.steps)
        torch.cuda.synchronize()
        ctx.check_overflow()
        ctx.set_static(False)
        graph = True
    T, V = wl.T, R.mc_vertices(wl.levels.Rmax)
    n_raw = sum(int(r.numel()) for r in st.raw)
    # algorithmic bytes per launch of each kernel (the data it must touch once)
    bytes_ = {
        # levels read once, the assembled texture written once
        "assemble": 4.0 * (n_raw + 8 * T * V),
        # the texture and its gradient read once, the levels' gradients written once
        "assemble_bwd": 4.0 * (n_raw + 2 * 8 * T * V),
        # per pixel: its key in, its colour out; per winner: the record (64 B), the three
        # grid vertices (96 B) and the view's inverse matrix is cached
        "shade": 8.0 * P + 12.0 * P + winners * (64.0 + 96.0),
    }
    log(f"paper form: {P} pixels, {winners} winners, fwd decodes {sf['decodes']}, eager {eager_ms:.3f} ms, "
        f"graph {ms:.3f} ms; unfused backward: eager {unfused_ms:.3f} ms, graph {unfused_graph_ms} ms")
    log("paper form per-kernel avg ms: " + ", ".join(f"{k}={v:.3f}" for k, v in per_kernel.items() if v > 0))
    out = {"workload": f"paper form: {T} triangles, texture levels {wl.levels.Rmin}..{wl.levels.Rtop} onto level "
                       f"{wl.levels.Rmax} ({V} grid vertices x 8 channels), MLP 16->16->16->3 deferred, "
                       f"{st.vs.V} views of 800x800, L1 + D-SSIM",
           "ms_per_step": round(ms, 4), "eager_ms_per_step": round(eager_ms, 4), "hip_graph": graph,
           "mpixel_s": round(P / (ms * 1e-3) / 1e6, 2), "pixels": P, "winners": winners,
           "forward_decodes": sf["decodes"], "covered_pixels": sf["covered_pixels"],
           "kernels_ms": {k: round(v, 4) for k, v in per_kernel.items() if v > 0},
           "hbm": {k: {"bytes": b, "gb_s": round(b / (pk[k] * 1e-3) / 1e9, 1),
                       "frac": round(b / (pk[k] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
                   for k, b in bytes_.items() for pk in [per_kernel if per_kernel.get(k, 0) > 0 else per_kernel_u]
                   if pk.get(k, 0) > 0},
           "unfused_backward": {"eager_ms_per_step": round(unfused_ms, 4),
                                "ms_per_step": None if unfused_graph_ms is None else round(unfused_graph_ms, 4),
                                "kernels_ms": {k: round(v, 4) for k, v in per_kernel_u.items() if v > 0}}}
    del st
    if graph:
        del g
    ctx.close()
    return out


def ceilings_bench(R, dev):
    """Measured ceilings on this GPU (the library's probe kernels, HIP events,
    best of several launches): HBM copy and read of 1 GiB, scattered float
    atomics, the non-packed float32 FMA rate and the float32 matrix-core
    rate, beside the published peaks."""
    import torch
    from paper_2603_27151_amd import _lib
    ctx = _lib.Ctx(0)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count

    def best_ms(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    out = {}
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    dst = torch.empty_like(src)
    ms = best_ms(lambda: _lib.soup_probe_copy(ctx, src, dst))
    out["hbm_copy"] = {"bytes": 2 * nbytes, "ms": round(ms, 4), "gb_s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
                       "frac": round(2 * nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    partial = torch.empty(n_cu * 64, dtype=torch.float32, device=dev)   # 64 workgroups per CU
    ms = best_ms(lambda: _lib.soup_probe_read(ctx, src, partial))
    out["hbm_read"] = {"bytes": nbytes, "ms": round(ms, 4), "gb_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                       "frac": round(nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    del src, dst
    slots = torch.zeros(1 << 26, dtype=torch.float32, device=dev)   # 256 MB: beyond the caches
    n_ops = 1 << 28
    ms = best_ms(lambda: _lib.soup_probe_atomic(ctx, slots, n_ops), reps=3)
    out["f32_atomics_scattered"] = {"ops": n_ops, "slots": int(slots.numel()), "ms": round(ms, 4),
                                    "gops": round(n_ops / (ms * 1e-3) / 1e9, 2)}
    del slots
    threads = n_cu * 4 * 8 * 64          # eight waves per SIMD
    iters = 8192
    o = torch.empty(threads, dtype=torch.float32, device=dev)
    ms = best_ms(lambda: _lib.soup_probe_fma(ctx, o, iters))
    tf = 16.0 * iters * threads / (ms * 1e-3) / 1e12
    out["valu_fp32_fma"] = {"ms": round(ms, 4), "tflops": round(tf, 2),
                            "frac_of_non_packed": round(tf / PEAK_FP32_NON_PACKED_TFLOPS, 4),
                            "frac_of_published": round(tf / PEAK_FP32_VECTOR_TFLOPS, 4)}
    threads = n_cu * 4 * 2 * 64          # two waves per SIMD
    o = torch.empty(threads, dtype=torch.float32, device=dev)
    ms = best_ms(lambda: _lib.soup_probe_mfma(ctx, o, iters))
    tf = 8192.0 * iters * (threads // 64) / (ms * 1e-3) / 1e12
    out["mfma_fp32"] = {"ms": round(ms, 4), "tflops": round(tf, 2), "frac_of_published": round(tf / PEAK_FP32_MFMA_TFLOPS, 4)}
    ctx.close()
    return out


def single_view_bench(args, R, W, dev, timed):
    """The single-view workload as configured (centres in the unit ball, depth
    complexity 2.97) and with the ball shrunk to a depth complexity of 8 (the
    figure the configuration quotes; both measured by the oracle's fragment
    statistics in tests/test_workload_depth.py): autotuned tile, eager and
    graph-replayed steps."""
    import torch
    from paper_2603_27151_amd import autotune
    out = {}
    for name, dc in (("single", 2.97), ("single_dc8", 8.0)):
        wl = W.by_name(name)
        ds = R.DeviceScene.from_host(wl.scene)
        vs = R.Views.from_list(wl.views)
        target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).to(dev)
        ctx = R._lib.Ctx(0)
        st = Step(R, ctx, ds, vs, target, wl.seed, wl.step)
        autotune.tune(st, ctx, name + "-" + autotune.signature(ds, vs))
        for _ in range(max(2, args.warmup)):
            st()
        eager = timed(st, max(10, args.steps))
        g = st.capture(log)
        g.replay()
        torch.cuda.synchronize()
        ctx.check_overflow()
        ms = timed(g.replay, max(10, args.steps))
        ctx.check_overflow()
        ctx.set_static(False)
        out[name] = {"depth_complexity": dc, "tile": ctx.tile, "ms_per_step": round(ms, 4),
                     "eager_ms_per_step": round(eager, 4), "mpixel_s": round(vs.pixels / (ms * 1e-3) / 1e6, 1),
                     "triangles_per_s": round(ds.T / (ms * 1e-3), 1)}
        del g, st
        ctx.close()
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched", choices=["batched", "single", "single_dc8", "large", "tiny"])
    ap.add_argument("--tile", type=int, default=0, help="tile side (0: autotuned)")
    ap.add_argument("--no-graph", action="store_true", help="time eager calls instead of HIP-graph replays")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-per-view", action="store_true")
    ap.add_argument("--cpu-pixels", type=float, default=8e6, help="oracle sample size in pixels (about 10 s of host work)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--skip-serve", action="store_true")
    ap.add_argument("--skip-adaptive", action="store_true")
    ap.add_argument("--skip-train", action="store_true")
    ap.add_argument("--skip-paper", action="store_true", help="skip the paper-form step")
    ap.add_argument("--skip-single", action="store_true", help="skip the single-view steps")
    ap.add_argument("--skip-ceilings", action="store_true", help="skip the measured ceilings")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first copy this many MiB device to device three times (a known-size kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="open-loop run at 200 req/s")
    ap.add_argument("--sweep-seconds", type=float, default=2.0, help="duration of each rate of the sweep")
    ap.add_argument("--serve-budget", type=float, default=0.25, help="admission budget: fraction of free HBM")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr, flush=True)
        sys.exit(2)
    import torch
    from paper_2603_27151_amd import raster as R
    from paper_2603_27151_amd import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = W.by_name(args.workload)
    ds = R.DeviceScene.from_host(wl.scene)
    vs = R.Views.from_list(wl.views)
    P = vs.pixels
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 3) for t in wl.targets])).to(dev)
    ctx = R.context()
    # the forward keeps its tile lists and a log of its decoded fragments; the backward reuses both
    step = Step(R, ctx, ds, vs, target, wl.seed, wl.step)
    opts_b = step.opts
    vis, color, loss, gc, gl = step.vis, step.color, step.loss, step.gc, step.gl
    gv, gf, gm = step.gv, step.gf, step.gm

    # tile size: given, or measured (every candidate runs the step)
    from paper_2603_27151_amd import autotune
    tuning = None
    if args.tile:
        ctx.set_tile(args.tile)
    else:
        tuning = autotune.tune(step, ctx, autotune.signature(ds, vs))
        log(f"autotune: {tuning}")
    tile = ctx.tile
    log(f"workload {args.workload}: T={ds.T} views={vs.V} pixels={P} tile={tile}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # work counts of the step (outside the timed region)
    ctx.set_counting(True)
    R.rasterize_fwd(ds, vs, opts_b, ctx=ctx, out=(vis, color, None))
    st_fwd = ctx.stats()
    R.loss_l2(color, target, ctx=ctx, out=(loss, gc, gl))
    R.rasterize_bwd(ds, vs, opts_b, vis, color, gc, gl, ctx=ctx, out=(gv, gf, gm))
    st_bwd = ctx.stats()
    ctx.set_counting(False)
    torch.cuda.synchronize()
    winners = int((vis != -1).sum().item())           # pixels where some fragment passes
    P_cov = st_fwd["covered_pixels"]                   # pixels that at least one fragment covers
    # winners that also carry a score weight: their colour logits get a data backward of their own
    W_s = int(((vis != -1) & (gl != 0)).sum().item())
    E = st_bwd["decodes"]          # front set + winner of every pixel: the method's decodes
    log(f"counts: bins={st_fwd['bin_entries']} fwd decodes={st_fwd['decodes']} E={E} winners={winners} "
        f"P_cov={P_cov} W_s={W_s}")

    def timed(fn, k):
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(k):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return max((t1 - t0) * 1e3 / k, ev0.elapsed_time(ev1) / k)

    # eager steps with per-kernel HIP events (recorded on the launch stream)
    ctx.read_timings()
    ctx.set_timing(True)
    eager_ms = timed(step, args.steps)
    ctx.set_timing(False)
    kern = ctx.read_timings()
    per_kernel = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern.items()}
    log(f"eager step {eager_ms:.3f} ms")
    log("per-kernel avg ms: " + ", ".join(f"{k}={v:.3f}" for k, v in per_kernel.items() if v > 0))

    # the step captured once into a HIP graph (static-capacity mode) and
    # replayed: the timed steps
    ms = eager_ms
    graph = False
    if not args.no_graph:
        ref = (vis.clone(), gv.clone())
        g = step.capture(log)
        g.replay()
        torch.cuda.synchronize()
        ctx.check_overflow()
        if not torch.equal(vis, ref[0]):
            raise RuntimeError("graph replay changed the visibility buffer")
        ms = timed(g.replay, args.steps)
        torch.cuda.synchronize()
        ctx.check_overflow()
        ctx.set_static(False)
        graph = True
        log(f"graph step {ms:.3f} ms")
    mpix = P / (ms * 1e-3) / 1e6
    log(f"batched step {ms:.3f} ms -> {mpix:.1f} Mpixel/s")

    # per-view path on the same GPU: a host loop of single-view calls with the
    # batched step's options (the forward keeps its tile lists and fragment
    # log, the backward reuses both), gradients summed in place (accumulate),
    # outputs written into slices of the batched step's buffers
    per_view = None
    if not args.skip_per_view:
        singles = [R.Views.from_list([v]) for v in wl.views]
        offs = vs.offsets()
        opts_f = R.Opts(seed=wl.seed, step=wl.step, reuse_bins=1)
        opts_acc = R.Opts(seed=wl.seed, step=wl.step, accumulate=1, reuse_bins=1)
        loss_i = torch.empty(1, dtype=torch.float32, device=dev)

        def step_pv():
            gv.zero_()
            gf.zero_()
            gm.zero_()
            for i, sv in enumerate(singles):
                a, b = int(offs[i]), int(offs[i + 1])
                vis_i, col_i, gc_i, gl_i = vis[a:b], color[a:b], gc[a:b], gl[a:b]
                R.rasterize_fwd(ds, sv, opts_f, ctx=ctx, out=(vis_i, col_i, None))
                R.loss_l2(col_i, target[a:b], ctx=ctx, out=(loss_i, gc_i, gl_i))
                R.rasterize_bwd(ds, sv, opts_acc, vis_i, col_i, gc_i, gl_i, ctx=ctx, out=(gv, gf, gm))

        step_pv()
        torch.cuda.synchronize()
        n_pv = max(2, args.steps // 3)
        t0 = time.perf_counter()
        for _ in range(n_pv):
            step_pv()
        torch.cuda.synchronize()
        pv_ms = (time.perf_counter() - t0) * 1e3 / n_pv
        per_view = {"ms_per_step": round(pv_ms, 3), "mpixel_s": round(P / (pv_ms * 1e-3) / 1e6, 1),
                    "options": "reuse_bins=1 on forward and backward, as the batched step",
                    "batched_speedup": round(pv_ms / ms, 3),
                    "batched_eager_speedup": round(pv_ms / eager_ms, 3)}
        log(f"per-view path {pv_ms:.3f} ms -> {per_view['mpixel_s']} Mpixel/s")

    # adaptive control of primitives on the same soup and visibility buffer
    # (not part of the step): coverage counts over every pixel, edge lengths
    # over a 20-view sample, the host plan of a random initialisation
    # (prune zero coverage, then split longest edges back to the triangle
    # count), and its application
    adaptive = None
    if not args.skip_adaptive:
        k_ad = max(3, args.steps)
        counts = torch.zeros(ds.T, dtype=torch.int32, device=dev)
        pick = np.sort(np.random.default_rng(20).choice(vs.V, size=min(20, vs.V), replace=False))
        sample = R.Views.from_list([wl.views[i] for i in pick])
        R.coverage_count(vis, ds.T, counts=counts, ctx=ctx)
        rel = R.edge_lengths(ds.verts, sample, ctx=ctx)
        torch.cuda.synchronize()
        ctx.read_timings()
        ctx.set_timing(True)
        for _ in range(k_ad):
            counts.zero_()
            R.coverage_count(vis, ds.T, counts=counts, ctx=ctx)
            rel = R.edge_lengths(ds.verts, sample, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        act, off, n_new = R.adaptive_plan(counts, rel, 0.2, target=ds.T, prune_zero=True, fill=True)
        plan_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(k_ad):
            new = R.adaptive_apply(ds, act, off, n_new, ctx=ctx)
        torch.cuda.synchronize()
        ctx.set_timing(False)
        kt = ctx.read_timings()
        avg = {k: kt[k][0] / kt[k][1] for k in ("coverage", "edge_lengths", "adaptive_apply") if kt[k][1]}
        n_split = int((act >= 2).sum())
        n_keep = int((act == 1).sum())
        per_tri = 4 * wl.scene.G * wl.scene.G * wl.scene.C + 36
        cov_bytes = 8 * P
        apply_bytes = (n_keep + n_split) * per_tri + n_new * per_tri + 8 * ds.T
        adaptive = {
            "coverage": {"ms": round(avg["coverage"], 4), "bytes": cov_bytes,
                         "gb_s": round(cov_bytes / (avg["coverage"] * 1e-3) / 1e9, 1),
                         "frac_hbm": round(cov_bytes / (avg["coverage"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
            "edge_lengths": {"ms": round(avg["edge_lengths"], 4), "views": int(sample.V),
                             "triangle_views_per_s": round(ds.T * sample.V / (avg["edge_lengths"] * 1e-3), 1)},
            "plan_host_ms": round(plan_ms, 3),
            "apply": {"ms": round(avg["adaptive_apply"], 4), "bytes": apply_bytes,
                      "gb_s": round(apply_bytes / (avg["adaptive_apply"] * 1e-3) / 1e9, 1),
                      "frac_hbm": round(apply_bytes / (avg["adaptive_apply"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                      "removed": int((act == 0).sum()), "split": n_split, "n_new": int(n_new)},
        }
        # the coverage kernel issues one device-scope atomic per distinct
        # triangle among each wave's 256 consecutive keys: count them
        keys = vis.cpu().numpy().view(np.uint64)
        tri = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
        valid = (keys != np.uint64(0xFFFFFFFFFFFFFFFF)) & (tri < ds.T)
        chunk = np.nonzero(valid)[0] // 256
        runs = int(np.unique(chunk * ds.T + tri[valid]).size)
        adaptive["coverage"]["atomics"] = runs
        adaptive["coverage"]["atomics_per_s"] = round(runs / (avg["coverage"] * 1e-3), 1)
        del new, keys, tri, valid, chunk
        log("adaptive: " + json.dumps(adaptive))

    # the training step's own kernels (not part of the step timed above): the
    # L1 + D-SSIM loss on a batch of four views (the paper's batch) and one
    # optimiser step over every parameter (VectorAdam on vertices, Adam on
    # features and MLP), on copies of the parameters
    train = None
    if not args.skip_train:
        k_tr = max(3, args.steps)
        four = R.Views.from_list(wl.views[:4])
        P4 = four.pixels
        c4, t4 = color[:P4].contiguous(), target[:P4].contiguous()
        out4 = (torch.empty(1, device=dev), torch.empty_like(c4), torch.empty(P4, device=dev))
        R.loss_l1_ssim(c4, t4, four, 0.8, ctx=ctx, out=out4)
        pv, pf, pm = ds.verts.clone().view(-1), ds.feats.clone().view(-1), ds.mlp.clone()
        mv, mf, mm = torch.zeros_like(pv), torch.zeros_like(pf), torch.zeros_like(pm)
        vv, vf, vm = torch.zeros(pv.numel() // 3, device=dev), torch.zeros_like(pf), torch.zeros_like(pm)
        torch.cuda.synchronize()
        ctx.read_timings()
        ctx.set_timing(True)
        for it in range(1, k_tr + 1):
            R.loss_l1_ssim(c4, t4, four, 0.8, ctx=ctx, out=out4)
            R.adam_step(pv, gv.view(-1), mv, vv, 1e-3, it, vec=3, ctx=ctx)
            R.adam_step(pf, gf.view(-1), mf, vf, 5e-2, it, ctx=ctx)
            R.adam_step(pm, gm, mm, vm, 1e-2, it, ctx=ctx)
        torch.cuda.synchronize()
        ctx.set_timing(False)
        kt = ctx.read_timings()
        loss_ms = kt["train_loss"][0] / kt["train_loss"][1]
        adam_ms = kt["adam"][0] / k_tr                        # the three launches of one step
        n_par = pv.numel() + pf.numel() + pm.numel()
        adam_bytes = 28 * (pf.numel() + pm.numel()) + 24 * pv.numel() + 8 * vv.numel()
        train = {"loss_l1_ssim": {"ms": round(loss_ms, 4), "views": 4, "pixels": int(P4),
                                  "mpixel_s": round(P4 / (loss_ms * 1e-3) / 1e6, 1)},
                 "adam_step": {"ms": round(adam_ms, 4), "params": int(n_par), "bytes": int(adam_bytes),
                               "gb_s": round(adam_bytes / (adam_ms * 1e-3) / 1e9, 1),
                               "frac_hbm": round(adam_bytes / (adam_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}}
        del pv, pf, pm, mv, mf, mm, vv, vf, vm
        # whole training iterations as the paper runs them: four random views
        # of the 64, stochastic forward, loss, backward, three optimiser
        # launches (one host synchronisation per iteration, for the loss value)
        from paper_2603_27151_amd import train as TRN
        student = R.DeviceScene(ds.verts.clone(), ds.feats.clone(), ds.mlp.clone(), list(ds.dims))
        trainer = TRN.Trainer(student, wl.views, wl.targets, TRN.TrainConfig(iters=1000), ctx=ctx)
        for _ in range(2):
            trainer.step()
        torch.cuda.synchronize()
        n_it = max(5, args.steps)
        t0 = time.perf_counter()
        for _ in range(n_it):
            trainer.step()
        torch.cuda.synchronize()
        it_ms = (time.perf_counter() - t0) * 1e3 / n_it
        train["iteration"] = {"ms": round(it_ms, 3), "iters_per_s": round(1e3 / it_ms, 1), "views": 4,
                              "mean_pixels": int(np.mean([v.width * v.height for v in wl.views]) * 4)}
        del student, trainer
        log("train: " + json.dumps(train))

    # roofline of the dominant kernel: the MLP kernels are bound by float32
    # ALU work; their algorithmic FLOPs count the decodes the method needs
    # (E = front set + winner per pixel, counted exactly by the backward's
    # decode). The forward shades a winner from the decode that tests it, so
    # it needs E decodes and no re-shade; the backward recomputes, back-
    # propagates and forms the weight gradient of every one of the E, plus a
    # second data backward for the colour logits of each winner that also
    # carries a score weight (its vertices move with those alone)
    macs = mlp_macs(ds.dims)
    work = {
        "decode_bwd": 6.0 * macs * E + 2.0 * macs * W_s,
        "raster_fwd": 2.0 * macs * E,
    }
    dom = max(work, key=lambda k: per_kernel.get(k, 0.0))
    t_dom = per_kernel[dom]
    fl = work[dom]
    achieved = fl / (t_dom * 1e-3) / 1e12
    # the decode's contractions run on the matrix cores (dense fp32 MFMA peak);
    # the forward's bit-exact MLP runs on the vector ALU (fp32 vector peak)
    bound, peak = ("mfma", PEAK_FP32_MFMA_TFLOPS) if dom == "decode_bwd" else ("alu", PEAK_FP32_VECTOR_TFLOPS)
    roofline = {"kernel": dom, "bound": bound, "achieved": round(achieved, 3),
                "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(dom, args.workload, tile),
                "flops_per_launch": fl, "avg_launch_ms": round(t_dom, 4)}
    # the other MLP kernel's standing, on the same terms (the forward's bit-exact MLP
    # runs on the vector ALU: its ceiling with packed FP32 disabled is 78.6 TFLOP/s)
    other = "raster_fwd" if dom == "decode_bwd" else "decode_bwd"
    o_bound, o_peak = ("mfma", PEAK_FP32_MFMA_TFLOPS) if other == "decode_bwd" else ("alu", PEAK_FP32_VECTOR_TFLOPS)
    o_achieved = work[other] / (per_kernel[other] * 1e-3) / 1e12 if per_kernel.get(other) else 0.0
    roofline_other = {"kernel": other, "bound": o_bound, "achieved": round(o_achieved, 3), "peak": o_peak,
                      "unit": "TFLOP/s", "frac": round(o_achieved / o_peak, 4),
                      "traffic": measured_traffic(other, args.workload, tile),
                      "flops_per_launch": work[other], "avg_launch_ms": round(per_kernel.get(other, 0.0), 4)}
    if o_bound == "alu":
        roofline_other["frac_of_non_packed_peak"] = round(o_achieved / PEAK_FP32_NON_PACKED_TFLOPS, 4)
    step_flops = work["decode_bwd"] + work["raster_fwd"]
    step_roofline = {"flops": step_flops, "achieved_tflops": round(step_flops / (ms * 1e-3) / 1e12, 3),
                     "frac": round(step_flops / (ms * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4)}

    # serving: forward-only renders of four resident soups, Poisson arrivals,
    # continuous batching over two streams
    serving = None
    if not args.skip_serve:
        from paper_2603_27151_amd import serve as SV
        soups = [R.DeviceScene.from_host(sc) for sc in W.serving_soups()]
        srv = SV.Server(soups, tile=None, n_streams=2, max_batch=16, budget_fraction=args.serve_budget)
        tuned = srv.tune_tiles([W.View(w, h, 0, W.view_proj((0.0, 0.3, 3.0), w, h)) for w, h in W.SERVING_RES])
        log(f"serving tiles: {srv.tile_by_res}")
        SV.run(srv, W.serving_requests(200.0, 1.0, seed=99))   # warm-up: workspaces, allocator
        log(f"serving: {args.serve_seconds:.0f} s at 200 req/s")
        main_st = SV.run(srv, W.serving_requests(200.0, args.serve_seconds))
        log(f"serving 200/s: {main_st}")
        sweep = []
        for rate in (100, 200, 400, 800, 1600, 3200, 6400, 12800):
            st = SV.run(srv, W.serving_requests(float(rate), args.sweep_seconds, seed=rate))
            sweep.append({"rate_hz": rate, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                          "throughput_rps": st["throughput_rps"], "mean_batch": st["mean_batch"]})
            log(f"serving sweep {rate}/s: {sweep[-1]}")
            if st["throughput_rps"] is None or st["throughput_rps"] < 0.9 * rate:
                break   # saturated
        # the same arrivals with a memory budget that fits two of the largest requests
        # (1920x1080 on the 100k-triangle soup), so that admission binds
        big = max(SV.request_bytes(w, h, sc.T) for w, h in W.SERVING_RES for sc in soups)
        srv_b = SV.Server(soups, tile=None, n_streams=2, max_batch=16, budget_bytes=2 * big)
        srv_b.tile_by_res = dict(srv.tile_by_res)
        SV.run(srv_b, W.serving_requests(200.0, 1.0, seed=98))
        bind_st = SV.run(srv_b, W.serving_requests(200.0, args.serve_seconds / 2, seed=97))
        burst = SV.run(srv_b, [W.Request(0.0, r.soup, r.view) for r in W.serving_requests(200.0, 0.5, seed=96)])
        log(f"serving 200/s, budget of two requests: {bind_st}; burst: {burst}")
        serving_bind = {"budget_bytes": srv_b.budget, "largest_request_bytes": big, "rate_hz": 200, **bind_st,
                        "burst_of_100": burst}
        del srv_b
        serving = {"workload": "4 soups (20k/40k/70k/100k triangles), 8x8x16 features, MLP 16->32->32->4, "
                               "threshold mode, 640x360/1280x720/1920x1080 uniform, Poisson arrivals",
                   "budget_of_two_requests": serving_bind,
                   "rate_hz": 200, "duration_s": args.serve_seconds, "streams": 2, "max_batch": 16,
                   "budget_fraction": args.serve_budget, "budget_bytes": srv.budget,
                   "tiles": {f"{w}x{h}": t for (w, h), t in srv.tile_by_res.items()},
                   "slo_p99_ms": 16.7, **main_st, "sweep": sweep}

    # the single-view workload, literal and at depth complexity 8
    single_view = None
    if not args.skip_single:
        single_view = single_view_bench(args, R, W, dev, timed)
        log("single view: " + json.dumps(single_view))

    # the paper form (Section 3.3): mesh-colour texture, opacity outside the
    # MLP, deferred shading; its own step on its own workload
    paper_form = None
    if not args.skip_paper:
        paper_form = paper_form_bench(args, R, W, dev, timed)
        log("paper form: " + json.dumps(paper_form))

    # measured ceilings of this GPU (probe kernels beside the published peaks)
    ceilings = None
    if not args.skip_ceilings:
        ceilings = ceilings_bench(R, dev)
        log("ceilings: " + json.dumps(ceilings))
        if roofline["bound"] == "mfma":
            roofline["measured_peak_mfma_fp32"] = ceilings["mfma_fp32"]["tflops"]
            roofline["frac_of_measured_peak"] = round(roofline["achieved"] / ceilings["mfma_fp32"]["tflops"], 4)
        else:
            roofline["measured_peak_valu_fp32"] = ceilings["valu_fp32_fma"]["tflops"]
            roofline["frac_of_measured_peak"] = round(roofline["achieved"] / ceilings["valu_fp32_fma"]["tflops"], 4)

    # CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.skip_cpu:
        from oracle import oracle as O
        oo = O.Opts(seed=wl.seed, step=wl.step)
        sample, npx = [], 0
        for v in wl.views:
            if npx >= args.cpu_pixels and sample:
                break
            sample.append(v)
            npx += v.width * v.height
        t0 = time.perf_counter()
        Ptot = P
        for i, v in enumerate(sample):
            rv, rc, _, _ = O.forward(wl.scene, v, oo, want_logp=False)
            d = rc - wl.targets[i]
            g_c = (2 * d / np.float32(3 * Ptot)).astype(np.float32)
            g_l = ((d * d).sum(-1) / np.float32(3 * Ptot)).astype(np.float32)
            O.backward(wl.scene, v, oo, rv, rc, g_c, g_l)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(npx / cpu_s / 1e6, 4), "unit": "Mpixel/s", "cores": O.threads(),
               "kind": "oracle",
               "sample": f"fwd+bwd of the first {len(sample)} of {vs.V} views ({npx} pixels) in {cpu_s:.1f} s"}
        log(f"cpu oracle {cpu['value']} Mpixel/s on {cpu['cores']} threads")

    out = {
        "metric": "fwd+bwd Mpixel/s (batched vs per-view) at <=1e-4 grad rel err; render p50/p99 ms",
        "value": round(mpix, 2),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {ds.T} triangles, {vs.V} views, {P} pixels, "
                               f"features {wl.scene.G}x{wl.scene.G}x{wl.scene.C}, MLP "
                               + "->".join(str(d) for d in ds.dims),
                   "tile": tile, "autotune_ms": None if tuning is None else tuning["ms"],
                   "hip_graph": graph, "eager_ms_per_step": round(eager_ms, 4),
                   "triangles_per_s": round(ds.T * vs.V / (ms * 1e-3), 1),
                   "decodes_E": E, "winners": winners, "covered_pixels_P_cov": P_cov,
                   "winners_with_score_weight": W_s, "forward_decodes": st_fwd["decodes"],
                   "bin_entries": st_fwd["bin_entries"]},
        "per_view": per_view,
        "kernels_ms": {k: round(v, 4) for k, v in per_kernel.items() if v > 0},
        "roofline": roofline,
        "step_roofline": step_roofline,
        "roofline_other": roofline_other,
        "cpu_baseline": cpu,
        "serving": serving,
        "adaptive": adaptive,
        "train": train,
        "paper_form": paper_form,
        "single_view": single_view,
        "ceilings": ceilings,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
