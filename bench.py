"""Benchmark of the integral-histogram hot path on one MI355X.

One step = one pass of the whole path over one synthetic 1920x1080 frame with
7 uint8 feature channels x 16 bins (112 planes):
  1. ih_build with coordinate moments (binning, row/column scans, carries,
     write-out of three 112 x 1080 x 1920 tensors);
  2. 100,000 Manhattan-weighted local histograms (SWIH), windows 16-256 px;
  3. 100,000 plain four-corner region histograms over the same windows;
  4. 3-level pyramid chi-square search of a 32x32 template over a 129 x 129
     grid of candidate origins.
Inputs are resident in HBM before timing.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "integral-hist Gpx·bins/s (% HBM peak); queries/s; tracker fps learned vs exhaustive"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--tile", type=str, default="", help="tile_h,cols_per_lane,planes_per_wave")
    return ap.parse_args()


def cpu_baseline(w, windows_sample=1000):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    t0 = time.perf_counter()
    ih = oracle.ih(w.img, w.bins, w.bits)
    mx, my = oracle.moments(w.img, w.bins, w.bits)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.weighted_swih(ih, mx, my, w.C, w.windows[:windows_sample])
    t_q = time.perf_counter() - t0
    del ih, mx, my
    n_q = len(w.windows)
    t_step = t_build + t_q * (n_q / windows_sample)
    return {
        "value": round(w.H * w.W * w.P / t_step / 1e9, 4),
        "unit": "Gpx·bins/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": ("count + moment integral histograms of the full 1920x1080x112 frame (%.2f s) and "
                   "%d of the %d weighted queries (%.3f s, scaled x%d); rect queries and matching "
                   "not included" % (t_build, windows_sample, n_q, t_q, n_q // windows_sample)),
        "host": platform.processor() or platform.machine(),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X and has no "
              "multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    import paper_1711_01656_amd as ih

    dev = torch.device("cuda:0")
    w = synth.config2()
    rng_win = np.random.default_rng(205)
    img = torch.from_numpy(w.img).to(dev)
    wins = torch.from_numpy(w.windows).to(dev)
    C, H, W, P, bins = w.C, w.H, w.W, w.P, w.bins
    cfg = None
    if args.tile:
        th, cpl, pg = (int(v) for v in args.tile.split(","))
        cfg = ih.TileCfg(th, cpl, pg)
    # template: a 32x32 window of the frame; candidates: 129 x 129 origins around it
    tr = int(rng_win.integers(64, H - 32 - 64))
    tc = int(rng_win.integers(64, W - 32 - 64))
    origins = torch.from_numpy(synth.grid_origins(tr - 64, tc - 64, 129, 129)).to(dev)
    tmpl_win = torch.tensor([[tr, tc, 32, 32]], dtype=torch.int32, device=dev)

    out = torch.empty((P, H, W), dtype=torch.int32, device=dev)
    mx = torch.empty_like(out)
    my = torch.empty_like(out)
    ws = torch.empty(ih.workspace_size(H, W, C, bins, True, cfg), dtype=torch.uint8, device=dev)
    wq = torch.empty((len(w.windows), P), dtype=torch.float32, device=dev)
    rq = torch.empty((len(w.windows), P), dtype=torch.int32, device=dev)
    desc = torch.empty((1, 21, P), dtype=torch.int32, device=dev)
    dist = torch.empty(origins.shape[0], dtype=torch.float32, device=dev)
    best = torch.empty(1, dtype=torch.int32, device=dev)

    def step():
        ih.ih_build(img, bins, moments=True, cfg=cfg, out=out, mom_out=(mx, my), ws=ws)
        ih.ih_query_weighted(out, mx, my, C, wins, out=wq)
        ih.ih_query_rect(out, wins, out=rq)
        ih.ih_pyramid_desc(out, tmpl_win, 3, out=desc)
        ih.ih_match_candidates(out, desc, 32, 32, origins, 3, "chi2", dist=dist, best=best)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    # timed region; the final write-out kernel of each build is bracketed by
    # events on the same stream
    ev_k = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(args.steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for k in range(args.steps):
        ih.ih_profile_events(*ev_k[k])
        step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ih.ih_profile_events(None, None)
    ms = t0.elapsed_time(t1) / args.steps
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_k]))
    print("timed %d steps in %.3f s" % (args.steps, wall), file=sys.stderr, flush=True)

    # separate per-stage timing (not part of the headline figure)
    def time_it(fn, n=5):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    t_build = time_it(lambda: ih.ih_build(img, bins, moments=True, cfg=cfg, out=out, mom_out=(mx, my), ws=ws))
    t_wq = time_it(lambda: ih.ih_query_weighted(out, mx, my, C, wins, out=wq))
    t_rq = time_it(lambda: ih.ih_query_rect(out, wins, out=rq))
    t_match = time_it(lambda: ih.ih_match_candidates(out, desc, 32, 32, origins, 3, "chi2", dist=dist, best=best))

    if args.copy_calib:
        n = args.copy_calib << 20
        a = torch.empty(n // 4, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()

    alg_bytes = 3 * P * H * W * 4 + C * H * W   # three int32 tensors written, u8 image read
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    gpx = H * W * P / (ms * 1e-3) / 1e9
    res = {
        "metric": METRIC,
        "value": round(gpx, 3),
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
            "workload": "1920x1080 frame, 7 u8 channels x 16 bins (112 planes), count + 2 moment IHs; "
                        "100k weighted + 100k plain window queries (16-256 px); 129x129 pyramid chi2 search",
            "H": H, "W": W, "channels": C, "bins_per_channel": bins, "planes": P,
            "weighted_queries": len(w.windows), "rect_queries": len(w.windows),
            "candidates": int(origins.shape[0]), "tile": str(cfg) if cfg else "heuristic",
        },
        "stages_ms": {"build": round(t_build, 4), "final_kernel": round(k_ms, 4),
                      "weighted_queries": round(t_wq, 4), "rect_queries": round(t_rq, 4),
                      "match": round(t_match, 4)},
        "build_gpxbins_per_s": round(H * W * P / (t_build * 1e-3) / 1e9, 3),
        "weighted_queries_per_s": round(len(w.windows) / (t_wq * 1e-3), 1),
        "rect_queries_per_s": round(len(w.windows) / (t_rq * 1e-3), 1),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_final (integral-histogram write-out, with moments)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "alg_bytes_per_launch": alg_bytes,
        },
    }
    if not args.no_cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
