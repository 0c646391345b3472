"""Benchmark of the integral-histogram hot path on one MI355X.

One step = one pass of the whole path over the 8192x8192 uint16 aerial-style
frame (64 bins, a 17.2 GB int32 integral histogram):
  1. ih_build (binning, row/column scans, carries, write-out);
  2. 1,000,000 plain four-corner rectangle histograms (sides 4-200 px);
  3. the 3-level pyramid descriptor of a 32x32 template and the pyramid
     chi-square search over a 129 x 129 grid of candidate origins.
Inputs are resident in HBM before timing.  Prints one JSON line whose value is
that step's throughput; the headline layout is planes innermost (the one the
queries read fast) and the bin-major layout is reported beside it.

The line also carries the other workloads ("workloads": the 640x480 frame,
the 1920x1080 7-channel frame with 100k weighted windows, the 64-frame batch
and the further rows), the tracker workload ("tracker": a 1280x720, 300-frame
synthetic video, exhaustive 65x65 search against the learned proposal), and
for every workload the oracle timed on the host's cores.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "integral-hist Gpx·bins/s (% HBM peak); queries/s; tracker fps learned vs exhaustive"
# kernel sources whose hash keys the committed traffic figures (a counter
# figure is reported only while the kernels it was taken from are unchanged)
KERNEL_SOURCES = ("paper_1711_01656_amd/csrc/ih_build_dev.h", "paper_1711_01656_amd/csrc/ih_build.hip",
                  "paper_1711_01656_amd/csrc/ih_onepass.hip", "paper_1711_01656_amd/csrc/ih_internal.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 summaries (lines `traffic: <kernel> | <workload> | <sources
    hash> | <bytes>`), or None when none was taken from the current sources."""
    want = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                parts = [x.strip() for x in line[len("traffic:"):].split("|")]
                if len(parts) == 4 and parts[0] == kernel and parts[1] == workload and parts[2] == want:
                    return int(parts[3])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--trials", type=int, default=5, help="graph-replay trials of --steps steps; median reported")
    ap.add_argument("--layout", choices=["hwb", "bhw"], default="hwb",
                    help="memory layout of the integral histogram for the headline step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--no-other", action="store_true", help="skip timing the other layout")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run one device fill and one copy of this many MiB (counter calibration)")
    ap.add_argument("--no-tracker", action="store_true", help="skip the tracker workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (640x480, 1920x1080x112, 64-frame batch, further rows)")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the further rows' legs (PHoG, median, SWIH kernels, CAMSHIFT) among the workloads")
    ap.add_argument("--fixed-tiles", action="store_true",
                    help="other workloads: use the tile shapes the autotuners chose on an MI355X instead of tuning")
    ap.add_argument("--workloads-only", action="store_true",
                    help="run only the other workloads and print their JSON object (for profiling)")
    ap.add_argument("--tracker-only", action="store_true",
                    help="run only the tracker workload and print its JSON object (for profiling)")
    ap.add_argument("--phog-only", action="store_true",
                    help="run only the magnitude-weighted orientation histogram and print its JSON object")
    ap.add_argument("--median-only", action="store_true",
                    help="run only the spatio-temporal median and print its JSON object")
    ap.add_argument("--camshift-only", action="store_true",
                    help="run only the colour likelihood + CAMSHIFT workload and print its JSON object")
    ap.add_argument("--kernels-only", action="store_true",
                    help="run only the spatial-kernel accuracy/time comparison and print its JSON object")
    ap.add_argument("--train-videos", type=int, default=800)
    ap.add_argument("--train-steps", type=int, default=8000)
    ap.add_argument("--tile", type=str, default="",
                    help="tile_h,tile_w,planes_per_wave[,passes] of the headline layout (default: the library's)")
    return ap.parse_args()


def _host():
    return platform.processor() or platform.machine()


def cpu_config3(w, min_seconds=10.0, threads=0):
    """The oracle on the 8192^2 workload, streamed one plane at a time (the
    17 GB histogram does not fit the host comfortably): planes are built by
    the Alg. 5 recurrence and their 1M rectangle queries answered until
    `min_seconds` have passed, then the full 129x129 search runs once by
    direct counting; the step time scales the per-plane times to 64 planes."""
    import oracle
    oracle.set_threads(threads)
    t_b = t_q = 0.0
    planes = 0
    t0 = time.perf_counter()
    while planes == 0 or (time.perf_counter() - t0 < min_seconds and planes < w.P):
        a = time.perf_counter()
        pl = oracle.ih_plane(w.img, w.bins, w.bits, planes)
        b = time.perf_counter()
        oracle.query_rect(pl[None], w.rects)
        c = time.perf_counter()
        t_b += b - a
        t_q += c - b
        planes += 1
        del pl
    a = time.perf_counter()
    tmpl = oracle.pyramid_desc_direct(w.img, w.bins, w.bits, [w.tmpl_win], 3)[0]
    oracle.match_direct(w.img, w.bins, w.bits, tmpl, 32, 32, 3, w.origins, "chi2")
    t_m = time.perf_counter() - a
    cores = oracle.num_threads()
    oracle.set_threads(0)
    step = (t_b + t_q) / planes * w.P + t_m
    return {"value": round(w.H * w.W * w.P / step / 1e9, 4), "unit": "Gpx·bins/s", "cores": cores,
            "kind": "oracle",
            "sample": ("%d of %d planes of the 8192x8192 frame built by the Alg. 5 recurrence (one at a time) "
                       "with their 1M rectangle queries, scaled to %d planes, plus the 129x129 pyramid chi2 "
                       "search by direct counting; step %.2f s (build %.3f s/plane, 1M queries %.3f s/plane, "
                       "search %.3f s)" % (planes, w.P, w.P, step, t_b / planes, t_q / planes, t_m)),
            "host": _host()}


def cpu_config2(w, origins, tmpl_win, min_seconds=5.0, threads=0):
    """The oracle on the 1920x1080x112 step (count + moment IHs, 100k SWIH
    queries, 100k rect queries, 129x129 search), repeated for >= min_seconds."""
    import oracle
    oracle.set_threads(threads)
    reps, t_build, t_wq, t_rq, t_m = 0, 0.0, 0.0, 0.0, 0.0
    t_start = time.perf_counter()
    while reps == 0 or time.perf_counter() - t_start < min_seconds:
        t0 = time.perf_counter()
        ih = oracle.ih(w.img, w.bins, w.bits)
        mx, my = oracle.moments(w.img, w.bins, w.bits)
        t1 = time.perf_counter()
        oracle.weighted_swih(ih, mx, my, w.C, w.windows)
        t2 = time.perf_counter()
        oracle.query_rect(ih, w.windows)
        t3 = time.perf_counter()
        tmpl = oracle.pyramid_desc(ih, [tmpl_win], 3)[0]
        oracle.match_direct(w.img, w.bins, w.bits, tmpl, 32, 32, 3, origins, "chi2")
        t4 = time.perf_counter()
        del ih, mx, my
        reps += 1
        t_build += t1 - t0
        t_wq += t2 - t1
        t_rq += t3 - t2
        t_m += t4 - t3
    t_step = (t_build + t_wq + t_rq + t_m) / reps
    cores = oracle.num_threads()
    oracle.set_threads(0)
    return {"value": round(w.H * w.W * w.P / t_step / 1e9, 4), "unit": "Gpx·bins/s", "cores": cores,
            "kind": "oracle",
            "sample": ("the full step (count + moment IHs by the Alg. 5 recurrence, 100k SWIH queries, 100k "
                       "rect queries, 129x129 pyramid chi2 search) repeated %d times in %.1f s; per step: "
                       "build %.3f s, weighted %.3f s, rect %.3f s, match %.3f s"
                       % (reps, t_build + t_wq + t_rq + t_m, t_build / reps, t_wq / reps, t_rq / reps,
                          t_m / reps)),
            "host": _host()}


def cpu_config1(w, min_seconds=3.0, threads=0):
    """The oracle on the 640x480 frame: build and 10,000 rectangle queries."""
    import oracle
    oracle.set_threads(threads)
    reps, tb, tq = 0, 0.0, 0.0
    t0 = time.perf_counter()
    while reps == 0 or time.perf_counter() - t0 < min_seconds:
        a = time.perf_counter()
        h = oracle.ih(w.img, w.bins, w.bits)
        b = time.perf_counter()
        oracle.query_rect(h, w.rects)
        tq += time.perf_counter() - b
        tb += b - a
        reps += 1
    cores = oracle.num_threads()
    oracle.set_threads(0)
    return {"value": round(w.H * w.W * w.P / (tb / reps) / 1e9, 4), "unit": "Gpx·bins/s (build)", "cores": cores,
            "kind": "oracle", "build_ms": round(tb / reps * 1e3, 3), "rect_ms": round(tq / reps * 1e3, 3),
            "sample": "build + 10k rectangle queries repeated %d times" % reps, "host": _host()}


def cpu_config4(frames, min_seconds=6.0, threads=0):
    """The oracle on the 64-frame batch, one frame at a time (build by the Alg.
    5 recurrence, template descriptor, 4,096-candidate chi-square search by
    direct counting) until min_seconds have passed; the batch time scales the
    sampled frames' time by their share of the batch's histogram elements."""
    import oracle
    oracle.set_threads(threads)
    total = sum(f.img.shape[1] * f.img.shape[2] * f.bins for f in frames)
    done = 0
    t = 0.0
    n = 0
    t0 = time.perf_counter()
    for f in frames:
        if n and time.perf_counter() - t0 >= min_seconds:
            break
        a = time.perf_counter()
        h = oracle.ih(f.img, f.bins, f.bits)
        tmpl = oracle.pyramid_desc(h, [f.tmpl_win], 3)[0]
        oracle.match_direct(f.img, f.bins, f.bits, tmpl, 32, 32, 3, f.origins, "chi2")
        t += time.perf_counter() - a
        done += f.img.shape[1] * f.img.shape[2] * f.bins
        n += 1
        del h
    cores = oracle.num_threads()
    oracle.set_threads(0)
    batch_s = t * total / done
    return {"value": round(total / batch_s / 1e9, 4), "unit": "Gpx·bins/s", "cores": cores, "kind": "oracle",
            "batch_ms": round(batch_s * 1e3, 1),
            "sample": "%d of %d frames (build + template + 4,096-candidate search each), scaled by histogram size"
                      % (n, len(frames)), "host": _host()}


class Step3:
    """Preallocated buffers and the three calls of one step on the 8192^2
    frame, in one layout and build configuration."""

    def __init__(self, ih, torch, w, img, rects, origins, tmpl_win, layout, cfg):
        dev = img.device
        self.ih, self.torch, self.layout, self.cfg = ih, torch, layout, cfg
        self.img, self.rects, self.origins, self.tmpl_win = img, rects, origins, tmpl_win
        self.bins, self.bits, P = w.bins, w.bits, w.P
        self.out = torch.empty(ih.shape_of(P, w.H, w.W, layout), dtype=torch.int32, device=dev)
        self.ws = torch.empty(ih.workspace_size(w.H, w.W, 1, w.bins, False, cfg, layout), dtype=torch.uint8,
                              device=dev)
        self.q = torch.empty((rects.shape[0], P), dtype=torch.int32, device=dev)
        self.desc = torch.empty((1, 21, P), dtype=torch.int32, device=dev)
        self.dist = torch.empty(origins.shape[0], dtype=torch.float32, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev)

    def build(self):
        self.ih.ih_build(self.img, self.bins, self.bits, cfg=self.cfg, out=self.out, ws=self.ws, layout=self.layout)

    def rect(self):
        self.ih.ih_query_rect(self.out, self.rects, out=self.q, layout=self.layout)

    def match(self):
        self.ih.ih_pyramid_desc(self.out, self.tmpl_win, 3, out=self.desc, layout=self.layout)
        self.ih.ih_match_candidates(self.out, self.desc, 32, 32, self.origins, 3, "chi2", dist=self.dist,
                                    best=self.best, layout=self.layout)

    def after_build(self):
        self.rect()
        self.match()

    def __call__(self):
        self.build()
        self.after_build()

    def outputs(self):
        return (self.out, self.q, self.dist, self.best)

    def stages(self):
        return {"rect": self.rect, "match": self.match}


def measure_step(torch, ih, step, steps, warmup, trials, alg_bytes, workload):
    """Times a step: `warmup` eager steps, then `steps` eager steps with the
    build bracketed by events on its stream (whole build) and the dominant
    kernel by the library's events, then the step captured once as a HIP
    graph and replayed (`trials` trials of `steps` replays, median), every
    replayed result checked bit for bit against the eager one."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev_b = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    ev_k = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev_b + ev_k:          # torch creates the HIP event on first record
        a.record()
        b.record()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for k in range(steps):
        ih.ih_profile_events(*ev_k[k])
        ev_b[k][0].record()
        step.build()
        ev_b[k][1].record()
        step.after_build()
    t1.record()
    torch.cuda.synchronize()
    ih.ih_profile_events(None, None)
    eager_ms = t0.elapsed_time(t1) / steps
    build_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_b]))
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_k]))
    status = ih.status(step.ws)
    ref = [t.clone() for t in step.outputs()]
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        step()
    for _ in range(warmup):
        graph.replay()
    tr = []
    for _ in range(max(1, trials)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            graph.replay()
        b.record()
        torch.cuda.synchronize()
        tr.append(a.elapsed_time(b) / steps)
    same = all(torch.equal(x, y) for x, y in zip(ref, step.outputs()))
    if not same:
        raise SystemExit("graph replay results differ from the eager step")
    del ref, graph
    stages = {"build": round(build_ms, 4), "dominant_kernel": round(k_ms, 4)}
    for name, fn in step.stages().items():
        stages[name] = round(time_calls(torch, fn, 5), 4)
    one = ih.build_passes(step.layout, step.cfg) == 1
    kname = "single-pass band kernel" if one else "three-pass write-out"
    return {
        "layout": step.layout, "cfg": repr(step.cfg) if step.cfg is not None else "library default",
        "build": "one pass" if one else "three passes",
        "ms_per_step": float(np.median(tr)), "graph_trials_ms": [round(t, 4) for t in tr],
        "eager_ms_per_step": round(eager_ms, 4), "graph_replays_match_eager": same, "stages_ms": stages,
        "build_status_bits": status,
        "build_roofline": {"bound": "hbm", "kernel": "whole build (%s)" % ("init + band kernel" if one else
                                                                          "tile pass + carry scan + write-out"),
                           "achieved": round(alg_bytes / build_ms / 1e6, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(alg_bytes / build_ms / 1e6 / HBM_PEAK_GBS, 4),
                           "traffic": profiled_traffic("whole build", "%s %s %s" % (workload, step.layout,
                                                                                    repr(step.cfg)))},
        "dominant_kernel": {"kernel": kname, "ms": round(k_ms, 4),
                            "achieved": round(alg_bytes / k_ms / 1e6, 1),
                            "frac": round(alg_bytes / k_ms / 1e6 / HBM_PEAK_GBS, 4),
                            "traffic": profiled_traffic(kname, "%s %s %s" % (workload, step.layout,
                                                                             repr(step.cfg)))},
    }


class Step2:
    """Preallocated buffers and the calls of one step on the 1920x1080 frame
    with 7 channels x 16 bins: build with moments, 100k weighted and 100k
    plain window histograms, template descriptor and 129x129 search."""

    def __init__(self, ih, torch, w, img, wins, origins, tmpl_win, layout, cfg):
        dev = img.device
        self.ih, self.torch, self.layout, self.cfg = ih, torch, layout, cfg
        self.img, self.wins, self.origins, self.tmpl_win = img, wins, origins, tmpl_win
        self.C, self.bins, P = w.C, w.bins, w.P
        shp = ih.shape_of(P, w.H, w.W, layout)
        self.out = torch.empty(shp, dtype=torch.int32, device=dev)
        self.mx = torch.empty_like(self.out)
        self.my = torch.empty_like(self.out)
        self.ws = torch.empty(ih.workspace_size(w.H, w.W, w.C, w.bins, True, cfg, layout), dtype=torch.uint8,
                              device=dev)
        n = wins.shape[0]
        self.wq = torch.empty((n, P), dtype=torch.float32, device=dev)
        self.rq = torch.empty((n, P), dtype=torch.int32, device=dev)
        self.desc = torch.empty((1, 21, P), dtype=torch.int32, device=dev)
        self.dist = torch.empty(origins.shape[0], dtype=torch.float32, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev)

    def build(self):
        self.ih.ih_build(self.img, self.bins, moments=True, cfg=self.cfg, out=self.out, mom_out=(self.mx, self.my),
                         ws=self.ws, layout=self.layout)

    def weighted(self):
        self.ih.ih_query_weighted(self.out, self.mx, self.my, self.C, self.wins, out=self.wq, layout=self.layout)

    def rect(self):
        self.ih.ih_query_rect(self.out, self.wins, out=self.rq, layout=self.layout)

    def match(self):
        self.ih.ih_pyramid_desc(self.out, self.tmpl_win, 3, out=self.desc, layout=self.layout)
        self.ih.ih_match_candidates(self.out, self.desc, 32, 32, self.origins, 3, "chi2", dist=self.dist,
                                    best=self.best, layout=self.layout)

    def after_build(self):
        self.weighted()
        self.rect()
        self.match()

    def __call__(self):
        self.build()
        self.after_build()

    def outputs(self):
        return (self.out, self.mx, self.my, self.wq, self.rq, self.dist, self.best)

    def stages(self):
        return {"weighted": self.weighted, "rect": self.rect, "match": self.match}


def config2_leg(torch, ih, synth, args):
    """The 1920x1080 frame with 7 u8 channels x 16 bins (112 planes): build
    with both moment tensors, 100k Manhattan-weighted and 100k plain window
    histograms (16-256 px), a 129x129 pyramid chi2 search; per layout the
    step graph-replayed and the whole build and its dominant kernel timed."""
    dev = torch.device("cuda:0")
    w = synth.config2()
    rng_win = np.random.default_rng(205)
    H, W, P = w.H, w.W, w.P
    img = torch.from_numpy(w.img).to(dev)
    wins = torch.from_numpy(w.windows).to(dev)
    tr = int(rng_win.integers(64, H - 32 - 64))
    tc = int(rng_win.integers(64, W - 32 - 64))
    origins_np = synth.grid_origins(tr - 64, tc - 64, 129, 129)
    origins = torch.from_numpy(origins_np).to(dev)
    tmpl_win = torch.tensor([[tr, tc, 32, 32]], dtype=torch.int32, device=dev)
    alg = 3 * P * H * W * 4 + w.C * H * W
    res = {"workload": "1920x1080 frame, 7 u8 channels x 16 bins (112 planes), count + 2 moment IHs; 100k "
                       "weighted + 100k plain window queries (16-256 px); 129x129 pyramid chi2 search",
           "alg_bytes_per_build": alg, "layouts": {}}
    for layout in ("hwb", "bhw"):
        step = Step2(ih, torch, w, img, wins, origins, tmpl_win, layout, None)
        r = measure_step(torch, ih, step, min(args.steps, 20), 3, 3, alg, "1920x1080x112 moments")
        r["gpxbins_per_s"] = round(H * W * P / r["ms_per_step"] / 1e6, 2)
        r["weighted_queries_per_s"] = round(wins.shape[0] / r["stages_ms"]["weighted"] * 1e3, 1)
        res["layouts"][layout] = r
        del step
        torch.cuda.empty_cache()
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_config2(w, origins_np, (tr, tc, 32, 32))
    return res


def time_calls(torch, fn, n):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(n):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / n


# tile shapes the autotuners chose for the other workloads on one MI355X
FIXED_TILES = {"640x480": (16, 16, 64), "8192x8192": (128, 64, 64), "batch_hwb": (128, 32, 64),
               "batch_bhw": (64, 256, 2)}


def phog_leg(torch, ih, synth):
    """Magnitude-weighted orientation integral histogram (Alg. 2 step 4) of
    the 1920x1080 scene: gradient orientation in 16 bins, gradient magnitude
    as the weight, edge pixels only.  Whole build (graph-replayed, median of
    trials) and the write-out kernel alone (library events around its
    launch), both layouts with their default tiles, checked against the
    count build for the same frame."""
    dev = torch.device("cuda:0")
    go, gm, edge = synth.phog_inputs()
    img, wt, mask = (torch.from_numpy(a).to(dev) for a in (go, gm, edge))
    H, W, bins = go.shape[1], go.shape[2], 16
    P = bins
    alg = P * H * W * 4 + 3 * H * W
    res = {"workload": "1920x1080 gradient orientation, 16 bins, magnitude-weighted over edge pixels",
           "edge_fraction": round(float((edge != 0).mean()), 4), "algorithmic_bytes": alg, "layouts": {}}
    for layout in ("bhw", "hwb"):
        out = torch.empty(ih.shape_of(P, H, W, layout), dtype=torch.int32, device=dev)
        ws = torch.empty(ih.workspace_size(H, W, 1, bins, False, None, layout), dtype=torch.uint8, device=dev)

        def wbuild():
            ih.ih_build_weighted(img, bins, wt, mask, out=out, ws=ws, layout=layout)

        def cbuild():
            ih.ih_build(img, bins, out=out, ws=ws, layout=layout)

        wbuild()
        torch.cuda.synchronize()
        ref = out.clone()
        tw = graph_median(torch, wbuild, 20, per=20)
        same = bool(torch.equal(out, ref))
        tc = graph_median(torch, cbuild, 20, per=20)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        for a, b in ev:
            a.record()
            b.record()
        torch.cuda.synchronize()
        for a, b in ev:
            ih.ih_profile_events(a, b)
            wbuild()
        torch.cuda.synchronize()
        ih.ih_profile_events(None, None)
        k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        res["layouts"][layout] = {"build_ms": round(tw, 4), "build_gbs": round(alg / tw / 1e6, 1),
                                  "writeout_ms": round(k_ms, 4),
                                  "writeout_gbs": round(P * H * W * 4 / k_ms / 1e6, 1),
                                  "writeout_frac_of_peak": round(P * H * W * 4 / k_ms / 1e6 / HBM_PEAK_GBS, 4),
                                  "count_build_ms": round(tc, 4), "replays_match_eager": same}
        del out, ws
    return res


def median_leg(torch, ih, synth):
    """Spatio-temporal median background model (Alg. 4) of a 768x576 grey
    surveillance video: 256 bins, a window of T+1 = 17 frames, a 3x3 spatial
    window.  Per layout: the joint-IH update (head in, tail out, in place)
    and the local-median pass, each graph-replayed, and the whole per-frame
    push (update, ring copy, median) timed over a stream of frames; the
    replayed median is checked against the streamed one."""
    from paper_1711_01656_amd.median import SpatioTemporalMedian
    dev = torch.device("cuda:0")
    F, T, bins, wh, ww = 48, 16, 256, 3, 3
    v = synth.surveillance_video(600, F)
    H, W = v.shape[1], v.shape[2]
    frames = torch.from_numpy(v).to(dev)
    P = bins
    upd_bytes = 2 * P * H * W * 4 + 2 * H * W
    probes = int(np.ceil(np.log2(bins)))
    # bin-major median: a binary search, 4 corners of one cumulative plane per
    # probe, plus the output
    med_bytes = H * W * (probes * 4 * 4 + 4)
    res = {"workload": "768x576 u8 grey video, 256 bins, 17-frame window, 3x3 spatial median",
           "frames_streamed": F - (T + 1), "update_algorithmic_bytes": upd_bytes,
           "median_probe_bytes_bhw": med_bytes, "layouts": {}}
    for layout in ("bhw", "hwb"):
        model = SpatioTemporalMedian(1, H, W, bins, T, wh, ww, layout=layout)
        for f in range(T + 1):
            model.push(frames[f])
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for f in range(T + 1, F):
            model.push(frames[f])
        b.record()
        torch.cuda.synchronize()
        push_ms = a.elapsed_time(b) / (F - T - 1)
        med_ref = model.median.clone()
        jih_ref = model.jih.clone()
        out = torch.empty_like(model.median)
        tm = graph_median(torch, lambda: ih.ih_local_median(jih_ref, 1, bins, T + 1, wh, ww, out=out,
                                                             layout=layout), 20, per=5)
        same = bool(torch.equal(out, med_ref))
        J = jih_ref.clone()
        ws = model.ws
        tu = graph_median(torch, lambda: ih.ih_jih_update(frames[F - 1], frames[F - 2], bins, J, ws=ws,
                                                          layout=layout), 20, per=5)
        res["layouts"][layout] = {"push_ms_per_frame": round(push_ms, 4),
                                  "frames_per_s": round(1e3 / push_ms, 1),
                                  "update_ms": round(tu, 4), "update_gbs": round(upd_bytes / tu / 1e6, 1),
                                  "update_frac_of_peak": round(upd_bytes / tu / 1e6 / HBM_PEAK_GBS, 4),
                                  "median_ms": round(tm, 4), "median_pixels_per_s": round(H * W / tm * 1e3, 1),
                                  "median_replay_matches_stream": same}
        del model, J, jih_ref, med_ref, out
        torch.cuda.empty_cache()
    return res


def kernels_leg(torch, ih, synth, sample=400):
    """Accuracy against time of the spatially weighted local histograms on the
    1920x1080, 7-channel x 16-bin frame with 100,000 windows (sides 16-256):
    exact SWIH with the Manhattan and quadratic kernels (O(1) from the count,
    moment and second-moment integral histograms) and the wedding cake of
    Eq. 3.2 with 1-8 layers for the Manhattan, quadratic and Gaussian
    (sigma 0.5) kernels.  Each query batch is graph-replayed; its error is
    the relative L1 distance to the oracle's FP64 brute force of the same
    kernel on `sample` of the windows, whose CPU time is also reported."""
    import oracle
    dev = torch.device("cuda:0")
    w = synth.config2()
    img = torch.from_numpy(w.img).to(dev)
    rects = torch.from_numpy(w.windows).to(dev)
    n = rects.shape[0]
    P = w.P
    c, mx, my = ih.ih_build(img, w.bins, w.bits, moments=True, layout="hwb")
    mxx, myy = ih.ih_build_moments2(img, w.bins, w.bits, layout="hwb")
    t_build = graph_median(torch, lambda: ih.ih_build(img, w.bins, w.bits, moments=True, out=c, mom_out=(mx, my),
                                                      layout="hwb"), 5)
    t_m2 = graph_median(torch, lambda: ih.ih_build_moments2(img, w.bins, w.bits, out=(mxx, myy), layout="hwb"), 5)
    out = torch.empty((n, P), dtype=torch.float32, device=dev)
    samp = w.windows[:sample]
    t0 = time.perf_counter()
    bf = {k: oracle.kernel_bruteforce(w.img, w.bins, w.bits, samp, k, 0.5) for k in ("manhattan", "quadratic",
                                                                                   "gaussian")}
    cpu_s = time.perf_counter() - t0
    methods = [("swih", "manhattan", 0, lambda: ih.ih_query_weighted(c, mx, my, w.C, rects, out=out, layout="hwb")),
               ("swih", "quadratic", 0, lambda: ih.ih_query_quadratic(c, mx, my, mxx, myy, w.C, rects, out=out,
                                                                      layout="hwb"))]
    for kern in ("manhattan", "quadratic", "gaussian"):
        for L in (1, 2, 3, 5, 8):
            methods.append(("wedding", kern, L, (lambda k=kern, l=L: ih.ih_query_wedding(c, w.C, rects, l, k, 0.5,
                                                                                      out=out, layout="hwb"))))
    rows = []
    for name, kern, L, fn in methods:
        t = graph_median(torch, fn, 10)
        fn()
        torch.cuda.synchronize()
        got = out[:sample].cpu().numpy().astype(np.float64)
        ref = bf[kern]
        err = float(np.abs(got - ref).sum() / np.abs(ref).sum())
        rows.append({"method": name, "kernel": kern, "layers": L, "ms": round(t, 4),
                     "windows_per_s": round(n / t * 1e3, 1), "rel_l1_err": float("%.3g" % err)})
    return {"workload": "1920x1080 frame, 7 u8 channels x 16 bins, 100k windows 16-256 px (planes innermost)",
            "windows": int(n), "build_count_and_moments_ms": round(t_build, 4), "build_second_moments_ms":
            round(t_m2, 4), "methods": rows,
            "cpu_bruteforce": {"windows": sample, "kernels": 3, "seconds": round(cpu_s, 3),
                               "ms_per_window_per_kernel": round(cpu_s / sample / 3 * 1e3, 4),
                               "threads": oracle.num_threads()}}


def camshift_leg(torch, ih, synth, n_starts=4096):
    """FG/BG colour likelihood and CAMSHIFT (Alg. 1) on frame 0 of the
    1280x720 tracking video: the likelihood from the target box and the box
    grown by its own size on every side (Eq. 2.18-2.21), the moment integral
    images of its 8-bit code, and CAMSHIFT with the target-sized window from
    one start and from `n_starts` starts scattered around the target.  Each
    stage graph-replayed; the oracle's CAMSHIFT (direct window sums) timed
    on the same starts."""
    import oracle
    from synth.video import config5
    dev = torch.device("cuda:0")
    v = config5(n_frames=1)
    rgb_np = v.rgb(0)
    r, c, h, w = v.target_box(0)
    H, W = rgb_np.shape[1:]
    fg = (r, c, r + h, c + w)
    bg = (max(0, r - h), max(0, c - w), min(H, r + 2 * h), min(W, c + 2 * w))
    rgb = torch.from_numpy(rgb_np).to(dev)
    q = torch.empty((H, W), dtype=torch.uint8, device=dev)
    L = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws = torch.empty(ih.lib().ih_color_likelihood_workspace_size(), dtype=torch.uint8, device=dev)
    moms = tuple(torch.empty((H, W), dtype=torch.int32, device=dev) for _ in range(3))
    mws = torch.empty(ih.workspace_size(H, W, 1, 1, True, None, "bhw"), dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(5)
    st_np = np.stack([r + h / 2 + rng.uniform(-h, h, n_starts), c + w / 2 + rng.uniform(-w, w, n_starts)], 1)
    starts = torch.from_numpy(st_np).to(dev)
    one = starts[:1].contiguous()
    cen = torch.empty((n_starts, 2), dtype=torch.float64, device=dev)
    its = torch.empty(n_starts, dtype=torch.int32, device=dev)
    cen1, its1 = cen[:1], its[:1]

    def like():
        ih.ih_color_likelihood(rgb, fg, bg, q=q, L=L, ws=ws)

    def mom():
        ih.ih_moment_images(q, out=moms, ws=mws)

    def cam(n):
        if n == 1:
            ih.ih_camshift(moms, one, h, w, 0.5, 20, centers=cen1, iters=its1)
        else:
            ih.ih_camshift(moms, starts, h, w, 0.5, 20, centers=cen, iters=its)

    def frame():
        like()
        mom()
        cam(1)

    frame()
    cam(n_starts)
    torch.cuda.synchronize()
    ref = cen.clone()
    t_like = graph_median(torch, like, 20, per=10)
    t_mom = graph_median(torch, mom, 20, per=10)
    t_cam1 = graph_median(torch, lambda: cam(1), 20, per=10)
    t_camn = graph_median(torch, lambda: cam(n_starts), 20, per=10)
    t_frame = graph_median(torch, frame, 20, per=10)
    cam(n_starts)
    torch.cuda.synchronize()
    same = bool(torch.equal(cen, ref))
    t0 = time.perf_counter()
    oq, _ = oracle.color_likelihood(rgb_np, fg, bg)
    t_olike = time.perf_counter() - t0
    t0 = time.perf_counter()
    ocen, oit = oracle.camshift(oq, st_np, h, w, 0.5, 20)
    t_ocam = time.perf_counter() - t0
    agree = bool(np.array_equal(ocen, cen.cpu().numpy()) and np.array_equal(oit, its.cpu().numpy()))
    return {"workload": "1280x720 RGB tracking frame, 32^3-bin FG/BG likelihood, %dx%d CAMSHIFT window" % (h, w),
            "likelihood_ms": round(t_like, 4), "moment_images_ms": round(t_mom, 4),
            "camshift_1_start_ms": round(t_cam1, 4), "camshift_%d_starts_ms" % n_starts: round(t_camn, 4),
            "frame_ms": round(t_frame, 4), "frames_per_s": round(1e3 / t_frame, 1),
            "mean_steps": round(float(its.float().mean().item()), 2),
            "replays_match_eager": same, "matches_oracle": agree,
            "oracle_ms": {"likelihood": round(t_olike * 1e3, 2), "camshift_%d_starts" % n_starts:
                          round(t_ocam * 1e3, 2), "threads": oracle.num_threads()}}


def copy_calibration(torch, mib):
    """One device fill and one device-to-device copy of `mib` MiB: the copy
    kernel's FETCH_SIZE and WRITE_SIZE against its known bytes give the
    counters' scale."""
    n = mib << 20
    a = torch.empty(n // 4, dtype=torch.int32, device="cuda:0")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def graph_median(torch, fn, n=10, trials=3, per=1):
    """Median over trials of the device time per call: `per` calls captured in
    one HIP graph, replayed n times per trial (no host launch cost)."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per):
            fn()
    return float(np.median([time_calls(torch, g.replay, n) for _ in range(trials)])) / per


def config1_leg(torch, ih, synth, args):
    """640x480 u8 with 32 bins and 10,000 rectangles: the build in both layouts
    with the library's default configuration (one launch each, graph-replayed),
    the rectangle queries, and the same frame 64 times as one batch (phased,
    graph-replayed) for the per-frame cost when frames arrive together."""
    dev = torch.device("cuda:0")
    w = synth.config1()
    img = torch.from_numpy(w.img).to(dev)
    rects = torch.from_numpy(w.rects).to(dev)
    alg = w.P * w.H * w.W * 4 + w.H * w.W
    res = {"workload": "640x480 u8, 32 bins, 10,000 rectangles (sides 4-200)", "alg_bytes_per_build": alg,
           "layouts": {}}
    for layout in ("bhw", "hwb"):
        out = torch.empty(ih.shape_of(w.P, w.H, w.W, layout), dtype=torch.int32, device=dev)
        ws = torch.empty(ih.workspace_size(w.H, w.W, w.C, w.bins, False, None, layout), dtype=torch.uint8, device=dev)
        q = torch.empty((rects.shape[0], w.P), dtype=torch.int32, device=dev)
        tb = graph_median(torch, lambda: ih.ih_build(img, w.bins, w.bits, out=out, ws=ws, layout=layout), 10, per=20)
        tq = graph_median(torch, lambda: ih.ih_query_rect(out, rects, out=q, layout=layout), 10, per=20)
        res["layouts"][layout] = {"build": "one pass" if ih.build_passes(layout) == 1 else "three passes",
                                  "build_ms": round(tb, 4), "gpxbins_per_s": round(w.H * w.W * w.P / tb / 1e6, 2),
                                  "build_frac_of_peak": round(alg / tb / 1e6 / HBM_PEAK_GBS, 4),
                                  "rect_ms": round(tq, 4), "rect_queries_per_s": round(rects.shape[0] / tq * 1e3, 1)}
        del out, ws, q
    frames = [dict(img=img, bins=w.bins, value_bits=w.bits, tile=None) for _ in range(64)]
    for layout in ("hwb", "bhw"):
        batch = ih.Batch(frames, "chi2", layout=layout)
        t = graph_median(torch, lambda: batch.run("phased"), 5)
        res["layouts"][layout]["batch_of_64_ms_per_frame"] = round(t / 64, 4)
        res["layouts"][layout]["batch_of_64_frac_of_peak"] = round(64 * alg / t / 1e6 / HBM_PEAK_GBS, 4)
        del batch
    torch.cuda.empty_cache()
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_config1(w)
    return res


def batch_leg(torch, ih, synth, args, fixed=False):
    """64 uneven frames (320x240 to 2048x2048, 8-64 bins) built and searched
    (4,096 candidates each) as one batch: phased launches replayed from a HIP
    graph and the cooperative single launch (which cannot be captured),
    against the same frames one call at a time."""
    from paper_1711_01656_amd import tune
    dev = torch.device("cuda:0")
    fr_np = synth.config4()
    frames = []
    total = 0
    for f in fr_np:
        g = torch.from_numpy(f.img).to(dev)
        frames.append(dict(img=g, bins=f.bins, value_bits=f.bits, tile=None,
                           origins=torch.from_numpy(f.origins).to(dev), win=(32, 32), tmpl_win=f.tmpl_win))
        total += f.img.shape[1] * f.img.shape[2] * f.bins
    per_layout = {}
    for lay in ("hwb", "bhw", "any"):
        if fixed:
            if lay == "any":
                continue
            tiles = [(lay, ih.TileCfg(*FIXED_TILES["batch_" + lay]))] * len(frames)
            by_bins, uniform_ms = {f["bins"]: tiles[0] for f in frames}, None
        else:
            # a tile shape (and with "any" a layout) per bin count, each chosen
            # by timing the whole batch
            tiles, by_bins, _, uniform_ms = tune.tune_batch_classes(frames, "chi2", layout=lay, reps=2)
        for fr, (fl, t) in zip(frames, tiles):
            fr["layout"], fr["tile"] = fl, t
        batch = ih.Batch(frames, "chi2", layout="bhw" if lay == "any" else lay)
        batch.run("phased")
        torch.cuda.synchronize()
        ref = [b.clone() for b in batch.best]
        t_graph = graph_median(torch, lambda: batch.run("phased"), 5)
        t_coop = float(np.median([time_calls(torch, lambda: batch.run("cooperative"), 5) for _ in range(3)]))
        same = all(torch.equal(a, b) for a, b in zip(ref, batch.best))
        per_layout["per_class_layout" if lay == "any" else lay] = {
                           "tiles_by_bins": {str(k): "%s %r" % v for k, v in sorted(by_bins.items())},
                           "uniform_tile_ms": None if uniform_ms is None else round(uniform_ms, 3),
                           "graph_phased_ms": round(t_graph, 3),
                           "cooperative_ms": round(t_coop, 3),
                           "gpxbins_per_s_graph": round(total / t_graph / 1e6, 2),
                           "ih_write_gbs_graph": round(total * 4 / t_graph / 1e6, 1),
                           "frac_of_peak_graph": round(total * 4 / t_graph / 1e6 / HBM_PEAK_GBS, 4),
                           "modes_agree": same}
        del batch, ref
        torch.cuda.empty_cache()
    seq = []
    for fr in frames:
        fr["tile"] = (ih.TileCfg(*FIXED_TILES["batch_bhw"]) if fixed
                      else tune.tune(fr["img"], fr["bins"], fr["value_bits"], layout="bhw", reps=2)[0])
        C, H, W = fr["img"].shape
        P = C * fr["bins"]
        o = torch.empty((P, H, W), dtype=torch.int32, device=dev)
        s_ws = torch.empty(ih.workspace_size(H, W, C, fr["bins"], False, fr["tile"], "bhw"), dtype=torch.uint8,
                           device=dev)
        d = torch.empty((1, 21, P), dtype=torch.int32, device=dev)
        di = torch.empty(fr["origins"].shape[0], dtype=torch.float32, device=dev)
        bb = torch.empty(1, dtype=torch.int32, device=dev)
        tww = torch.tensor([list(fr["tmpl_win"])], dtype=torch.int32, device=dev)
        seq.append((fr, o, s_ws, d, di, bb, tww))

    def one_by_one():
        for fr, o, s_ws, d, di, bb, tww in seq:
            ih.ih_build(fr["img"], fr["bins"], fr["value_bits"], cfg=fr["tile"], out=o, ws=s_ws, layout="bhw")
            ih.ih_pyramid_desc(o, tww, 3, out=d, layout="bhw")
            ih.ih_match_candidates(o, d, 32, 32, fr["origins"], 3, "chi2", dist=di, best=bb, layout="bhw")

    t_seq = graph_median(torch, one_by_one, 3)
    del seq
    torch.cuda.empty_cache()
    res = {"frames": len(frames), "ih_bytes": total * 4, "candidates_per_frame": 4096, "layouts": per_layout,
           "one_call_per_frame_bhw_ms": round(t_seq, 3)}
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_config4(fr_np)
    return res


def config_legs(torch, ih, synth, args):
    """Every workload other than the headline step, each with its CPU oracle
    baseline where the oracle covers it."""
    res = {"640x480_u8_32bins": config1_leg(torch, ih, synth, args)}
    torch.cuda.empty_cache()
    res["1920x1080x112_moments"] = config2_leg(torch, ih, synth, args)
    torch.cuda.empty_cache()
    res["batch_64_uneven_frames"] = batch_leg(torch, ih, synth, args, args.fixed_tiles)
    torch.cuda.empty_cache()
    if not args.no_rows:
        res["phog_1920x1080_16bins"] = phog_leg(torch, ih, synth)
        res["median_768x576_256bins"] = median_leg(torch, ih, synth)
        res["swih_kernels_1920x1080x112"] = kernels_leg(torch, ih, synth)
        res["camshift_1280x720"] = camshift_leg(torch, ih, synth)
    return res


def search_cost_vs_targets(torch, trk, lp, tr, net, frame, box0, counts=(1, 4, 16, 64, 256)):
    """Device time of one frame's search step for N targets at once (the
    integral histogram already built): exhaustive = the pyramid distance of
    N x 4,225 candidate windows; learned = network on N crops, top 64 per
    target, pyramid distance of N x 64 candidates.  Targets sit on a grid
    around the benchmark target so every window lies inside the frame."""
    dev = frame.device
    tr.set_template(frame, box0)
    h, w = tr.win
    out = {}
    big = lp.ProposalNet(net.get_params(), max_batch=max(counts))
    big.pack()
    for n in counts:
        g = int(np.ceil(np.sqrt(n)))
        ys = np.linspace(40, frame.shape[1] - h - 40, g).astype(int)
        xs = np.linspace(40, frame.shape[2] - w - 40, g).astype(int)
        base = np.array([(y, x) for y in ys for x in xs][:n], np.int32)
        base_d = torch.from_numpy(base).to(dev)
        centers = torch.from_numpy(base + np.array([h // 2, w // 2], np.int32)).to(dev)
        ex_orig = lp.lp_origins(base_d, lp.RADIUS)
        ex_dist = torch.empty(n * lp.N_OFFSETS, dtype=torch.float32, device=dev)
        best = torch.empty(1, dtype=torch.int32, device=dev)
        idx = torch.empty((n, 64), dtype=torch.int32, device=dev)
        k_orig = torch.empty((n * 64, 2), dtype=torch.int32, device=dev)
        k_dist = torch.empty(n * 64, dtype=torch.float32, device=dev)

        def exhaustive():
            tr.score(ex_orig, ex_dist, best)

        def learned():
            x = big.crop(frame, centers)
            logits = big.forward(x)
            lp.lp_topk(logits.view(n, -1), 64, idx)
            lp.lp_origins(base_d, lp.RADIUS, idx=idx, out=k_orig)
            tr.score(k_orig, k_dist, best)

        out[str(n)] = {"exhaustive": round(time_calls(torch, exhaustive, 20), 4),
                       "learned": round(time_calls(torch, learned, 20), 4)}
    return out


def cpu_tracker(frames_np, box0, ex_origins, min_seconds=6.0, threads=0):
    """The oracle's exhaustive search (frame histogram by the Alg. 5
    recurrence, 65x65 candidates scored by direct counting, fixed frame-0
    template) on frames of the video, each from the GPU exhaustive track's
    previous origin, until min_seconds have passed; frames per second."""
    import oracle
    oracle.set_threads(threads)
    h, w = int(box0[2]), int(box0[3])
    tmpl = oracle.pyramid_desc_direct(frames_np[0], 16, 8, [list(box0)], 3)[0]
    d = np.arange(-32, 33)
    n, t = 0, 0.0
    agree = 0
    t0 = time.perf_counter()
    for f in range(1, len(frames_np)):
        if n and time.perf_counter() - t0 >= min_seconds:
            break
        prev = ex_origins[f - 1]
        origins = np.stack(np.meshgrid(prev[0] + d, prev[1] + d, indexing="ij"), -1).reshape(-1, 2).astype(np.int32)
        a = time.perf_counter()
        hist = oracle.ih(frames_np[f], 16, 8)
        dist = oracle.match_direct(frames_np[f], 16, 8, tmpl, h, w, 3, origins, "chi2")[0]
        t += time.perf_counter() - a
        best = int(np.argmin(np.where(np.isfinite(dist), dist, np.inf)))
        agree += int(tuple(origins[best]) == tuple(ex_origins[f]))
        n += 1
        del hist
    cores = oracle.num_threads()
    oracle.set_threads(0)
    return {"value": round(n / t, 2), "unit": "frames/s (exhaustive)", "cores": cores, "kind": "oracle",
            "sample": "%d frames of the 1280x720 video: histogram of the frame + 4,225-candidate search each; "
                      "the oracle's pick equals the GPU exhaustive track on %d of them" % (n, agree),
            "host": _host()}


# the learned search's settings: with the bounded gate they change only how
# many candidates are scored exactly (the track is the exhaustive one for any
# value); the margin-only variant's agreement depends on them
TRACKER_TAU, TRACKER_ROUNDS, TRACKER_Q = 0.1, 0, 2
MARGIN_ONLY_ROUNDS = 2


def tracker_leg(torch, args):
    """Learned vs exhaustive tracking on the 1280x720, 300-frame video."""
    from paper_1711_01656_amd import proposal as lp
    from paper_1711_01656_amd import tracker as trk
    from synth.video import config5, render, training_videos

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    # training data: independent 640x360 sequences labelled by the exhaustive search
    th, tw, tf = 360, 640, 16
    ttr = trk.PyramidTracker(th, tw, region=True)
    stack, parts = [], []
    for i, v in enumerate(training_videos(args.train_videos, tf, th, tw)):
        f = torch.from_numpy(render(v, threads=16)).to(dev)
        box = v.target_box(0)
        parts.append(trk.samples_from_track(trk.track(f, box, ttr), box[2:], frame0=i * tf))
        stack.append(f)
    stack = torch.cat(stack)
    samples = trk.concat(parts)
    t_data = time.perf_counter() - t0
    batch, lr, jitter = 64, 0.01, 20
    net = lp.ProposalNet(lp.init_params(1), max_batch=batch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = trk.train(net, stack, samples, steps=args.train_steps, batch=batch, lr=lr, jitter=jitter, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del stack, ttr
    print("tracker: data %.1fs (%d samples), training %.1fs" % (t_data, len(samples.frame), t_train),
          file=sys.stderr, flush=True)

    video = config5()
    frames_np = render(video, threads=16)
    frames = torch.from_numpy(frames_np).to(dev)
    box0 = video.target_box(0)
    tr_f = trk.PyramidTracker(video.H, video.W)                  # the frame's histogram (the thesis's tracker)
    tr_r = trk.PyramidTracker(video.H, video.W, region=True)     # the search region's histogram
    prior = trk.distance_prior().to(dev)
    tau, rounds, q = TRACKER_TAU, TRACKER_ROUNDS, TRACKER_Q

    def timed(tr, learned=None, graph=True):
        """Free-running track on the device (one captured step replayed per
        frame); frames per second of wall time, template set-up excluded."""
        trk.track_device(frames[:8], box0, tr, learned, graph=graph)          # warm-up
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = trk.track_device(frames, box0, tr, learned, graph=graph)
        torch.cuda.synchronize()
        return res, (len(frames) - 1) / (time.perf_counter() - a)

    ex, fps_ex = timed(tr_f)
    ex_r, fps_ex_r = timed(tr_r)
    # primary: the bounded learned search (exact by construction); beside it the
    # margin rule alone (the proposal's result accepted as it is)
    learned = trk.LearnedTracker(tr_r, net, k=64, tau=tau, refine_rounds=rounds, refine_q=q, bound=True)
    free, fps_l = timed(tr_r, learned)
    base = trk.LearnedTracker(tr_r, None, k=64, tau=tau, prior_logits=prior, refine_rounds=rounds, refine_q=q,
                              bound=True)
    free_b, fps_b = timed(tr_r, base)
    margin = trk.LearnedTracker(tr_r, net, k=64, tau=tau, refine_rounds=MARGIN_ONLY_ROUNDS, refine_q=q)
    free_m, fps_m = timed(tr_r, margin)
    margin_b = trk.LearnedTracker(tr_r, None, k=64, tau=tau, prior_logits=prior, refine_rounds=MARGIN_ONLY_ROUNDS,
                                  refine_q=q)
    unref = trk.LearnedTracker(tr_r, net, k=64, tau=tau)
    # per-frame agreement: every search starts from the exhaustive trajectory
    forced = trk.track(frames, box0, tr_r, learned, teacher=ex)
    forced_b = trk.track(frames, box0, tr_r, base, teacher=ex)
    forced_m = trk.track(frames, box0, tr_r, margin, teacher=ex)
    forced_mb = trk.track(frames, box0, tr_r, margin_b, teacher=ex)
    forced_u = trk.track(frames, box0, tr_r, unref, teacher=ex)
    held = trk.samples_from_track(ex, box0[2:])

    def agree(a, b, px=0):
        return float(np.mean(np.all(np.abs(a.origins[1:] - b.origins[1:]) <= px, axis=1)))

    def scorings(t):
        """Candidates scored exactly per frame: the k proposals, the refinement
        neighbourhoods and the exhaustive list's listed offsets."""
        return round(float(np.mean(64 + rounds * (2 * q + 1) ** 2 + t.scored[1:])), 1)

    sweep = {}
    for r, tau_s in ((0, tau), (1, tau), (2, tau), (4, tau), (0, 0.5), (0, math.inf)):
        lt_r = trk.LearnedTracker(tr_r, net, k=64, tau=tau_s, refine_rounds=r, refine_q=q, bound=True)
        _, fps_r = timed(tr_r, lt_r)
        f_r = trk.track(frames, box0, tr_r, lt_r, teacher=ex)
        sweep["rounds %d tau %s" % (r, tau_s)] = {
            "fps": round(fps_r, 1), "agreement_per_frame": agree(f_r, ex),
            "exact_scorings_per_frame": round(float(np.mean(64 + r * (2 * q + 1) ** 2 + f_r.scored[1:])), 1),
            "fallback_rate": float(f_r.fallback[1:].mean())}
    x = net.crop(frames[1], torch.tensor([[box0[0] + box0[2] // 2, box0[1] + box0[3] // 2]], dtype=torch.int32,
                                         device=dev))
    fwd_ms = time_calls(torch, lambda: net.forward(x), 50)
    scaling = search_cost_vs_targets(torch, trk, lp, tr_f, net, frames[1], box0)
    res = {
        "workload": "1280x720 synthetic video, 300 frames, 7 channels x 16 bins; 65x65 offsets; top-64 learned "
                    "proposals%s; bounded exhaustive search (2-level pyramid lower bound) when the margin rule "
                    "accepts, full exhaustive search otherwise"
                    % (" + %d rounds of %dx%d local refinement" % (rounds, 2 * q + 1, 2 * q + 1) if rounds else ""),
        "fps_exhaustive": round(fps_ex, 1),
        "fps_exhaustive_region_ih": round(fps_ex_r, 1),
        "fps_learned": round(fps_l, 1),
        "fps_no_network": round(fps_b, 1),
        "fps_learned_margin_only": round(fps_m, 1),
        "fps_learned_over_exhaustive": round(fps_l / fps_ex, 3),
        "fps_learned_over_exhaustive_region_ih": round(fps_l / fps_ex_r, 3),
        "region_ih_track_equals_frame_ih_track": bool(np.array_equal(ex.origins, ex_r.origins)
                                                      and np.array_equal(ex.dists, ex_r.dists)),
        "tau": tau, "refine_rounds": rounds, "refine_window": 2 * q + 1,
        "margin_only_refine_rounds": MARGIN_ONLY_ROUNDS,
        "agreement_per_frame": agree(forced, ex),
        "agreement_per_frame_no_network": agree(forced_b, ex),
        "agreement_per_frame_margin_only": agree(forced_m, ex),
        "agreement_per_frame_margin_only_no_network": agree(forced_mb, ex),
        "agreement_per_frame_margin_only_without_refinement": agree(forced_u, ex),
        "fallback_rate": float(forced.fallback[1:].mean()),
        "fallback_rate_no_network": float(forced_b.fallback[1:].mean()),
        "fallback_rate_margin_only_without_refinement": float(forced_u.fallback[1:].mean()),
        "exact_scorings_per_frame": {"exhaustive": lp.N_OFFSETS, "learned": scorings(forced),
                                     "no_network": scorings(forced_b)},
        "bounded_sweep": sweep,
        "recall_top64": round(trk.recall(net, frames, held), 4),
        "recall_top64_no_network": round(trk.recall(prior, frames, held), 4),
        "free_running_equals_exhaustive": bool(np.array_equal(free.origins, ex.origins)),
        "free_running_within_1px_margin_only": agree(free_m, ex, 1),
        "free_running_fallback_rate": float(free.fallback[1:].mean()),
        "network_forward_ms": round(fwd_ms, 4),
        "search_ms_vs_targets": scaling,
        "training": {"samples": int(len(samples.frame)), "steps": args.train_steps, "batch": batch,
                     "lr": lr, "jitter": jitter,
                     "seconds": round(t_train, 2), "ms_per_step": round(t_train / args.train_steps * 1e3, 3),
                     "loss_first": round(float(np.mean(losses[:20])), 4),
                     "loss_last": round(float(np.mean(losses[-100:])), 4)},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_tracker(frames_np, box0, ex.origins)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X and has no "
              "multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    import paper_1711_01656_amd as ih

    if args.tracker_only:
        print(json.dumps(tracker_leg(torch, args)), flush=True)
        return
    if args.workloads_only:
        res = config_legs(torch, ih, synth, args)
        if args.copy_calib:
            copy_calibration(torch, args.copy_calib)
        print(json.dumps(res), flush=True)
        return
    if args.camshift_only:
        print(json.dumps(camshift_leg(torch, ih, synth)), flush=True)
        return
    if args.kernels_only:
        print(json.dumps(kernels_leg(torch, ih, synth)), flush=True)
        return
    if args.median_only:
        res = median_leg(torch, ih, synth)
        if args.copy_calib:
            copy_calibration(torch, args.copy_calib)
        print(json.dumps(res), flush=True)
        return
    if args.phog_only:
        res = phog_leg(torch, ih, synth)
        if args.copy_calib:
            copy_calibration(torch, args.copy_calib)
        print(json.dumps(res), flush=True)
        return

    dev = torch.device("cuda:0")
    w = synth.config3()
    H, W, P = w.H, w.W, w.P
    img = torch.from_numpy(w.img).to(dev)
    rects = torch.from_numpy(w.rects).to(dev)
    origins = torch.from_numpy(w.origins).to(dev)
    tmpl_win = torch.tensor([list(w.tmpl_win)], dtype=torch.int32, device=dev)
    alg = P * H * W * 4 + H * W * 2          # int32 histogram written, u16 image read
    wl = "8192x8192 u16 64 bins"
    cfgs = {"hwb": None, "bhw": None}
    if args.tile:
        cfgs[args.layout] = ih.TileCfg(*(int(v) for v in args.tile.split(",")))
    layouts = [args.layout] + ([] if args.no_other else [lo for lo in ("hwb", "bhw") if lo != args.layout])
    per = {}
    for lay in layouts:
        step = Step3(ih, torch, w, img, rects, origins, tmpl_win, lay, cfgs[lay])
        n = args.steps if lay == args.layout else max(3, min(args.steps, 10))
        per[lay] = measure_step(torch, ih, step, n, args.warmup, args.trials if lay == args.layout else 3, alg, wl)
        per[lay]["gpxbins_per_s"] = round(H * W * P / per[lay]["ms_per_step"] / 1e6, 3)
        per[lay]["rect_queries_per_s"] = round(rects.shape[0] / per[lay]["stages_ms"]["rect"] * 1e3, 1)
        print("%s: step %.4f ms, build %.4f ms (%.3f of peak)" % (lay, per[lay]["ms_per_step"],
                                                                 per[lay]["stages_ms"]["build"],
                                                                 per[lay]["build_roofline"]["frac"]),
              file=sys.stderr, flush=True)
        del step
        torch.cuda.empty_cache()
    del img, rects, origins

    # measured stream-write ceiling: a 2 GiB device fill, best of 5
    fill = torch.empty(1 << 29, dtype=torch.int32, device=dev)
    fill_ms = min(time_calls(torch, lambda: fill.fill_(1), 3) for _ in range(5))
    write_peak = fill.numel() * 4 / (fill_ms * 1e-3) / 1e9
    del fill
    if args.copy_calib:
        copy_calibration(torch, args.copy_calib)

    head = per[args.layout]
    ms = head["ms_per_step"]
    dk = head["dominant_kernel"]
    res = {
        "metric": METRIC,
        "value": round(H * W * P / (ms * 1e-3) / 1e9, 3),
        "unit": "Gpx·bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "8192x8192 u16 aerial-style frame, 64 bins (17.2 GB int32 integral histogram); 1M "
                        "rectangle queries (sides 4-200); 3-level pyramid chi2 search of a 32x32 template over "
                        "129x129 candidate origins",
            "H": H, "W": W, "channels": 1, "bins": w.bins, "planes": P, "rect_queries": int(w.rects.shape[0]),
            "candidates": int(w.origins.shape[0]), "layout": args.layout, "build": head["build"],
            "cfg": head["cfg"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": head["build_roofline"]["kernel"],
            "achieved": head["build_roofline"]["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": head["build_roofline"]["frac"],
            "traffic": head["build_roofline"]["traffic"],
            "alg_bytes_per_launch": alg,
            "dominant_kernel": {"kernel": dk["kernel"], "achieved": dk["achieved"], "frac": dk["frac"],
                                "ms": dk["ms"], "traffic": dk["traffic"]},
            "measured_write_peak": round(write_peak, 1),
            "frac_of_measured_write_peak": round(head["build_roofline"]["achieved"] / write_peak, 4),
        },
        "layouts": per,
    }
    if not args.no_configs:
        print("other workloads ...", file=sys.stderr, flush=True)
        res["workloads"] = config_legs(torch, ih, synth, args)
    if not args.no_tracker:
        print("tracker ...", file=sys.stderr, flush=True)
        res["tracker"] = tracker_leg(torch, args)
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_config3(w)
        res["cpu_baseline_1thread"] = cpu_config3(w, min_seconds=8.0, threads=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
