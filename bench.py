"""Throughput benchmark: particles/s labelled by periodic Friends-of-Friends on
one MI355X, FP32-filter path against the plain all-FP64 path, exact labels.

Workload (default): ``clustered256`` -- N = 256^3 FP32 positions in a periodic
unit box, 60 % in Plummer halos (counts ~ M^-1.9 on [20, 1e5]), 40 % uniform,
l_x = 0.2 x mean separation. One step = fof_build_cells + fof_link +
fof_finalize over the whole input, positions already in HBM, labels and sizes
left in HBM. The batched form (256 boxes of log-uniform size, one HIP graph)
and the plain FP64 path are timed beside it and reported in the same line.

Prints one JSON line. ``--gpus`` above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s FoF labelled on 1 MI355X: FP32-filter+batched vs plain FP64, exact"
FP32_VALU_PEAK_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, no packed FP32
HBM_PEAK_GBS = 8000.0
FLOP_PER_PAIR_TEST = 8            # 3 sub, 3 mul, 2 add (FMA counted as mul + add)
KERNEL_SOURCE = os.path.join(ROOT, "paper_2003_11468_amd", "csrc", "fof_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered256")
    ap.add_argument("--cell-factor", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    return ap.parse_args()


class Timer:
    """HIP events on the stream the kernels are launched on."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def event(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e


def time_pipeline(torch, fof, f, pos, w, steps, warmup, label, size):
    """Runs warmup + steps full passes; returns total ms and per-phase ms lists."""
    t = Timer(torch, f.stream)
    f.reserve(w.offsets, w.box, w.lx)
    for _ in range(warmup):
        fof.fof_build_cells(f.ctx, pos, w.offsets, w.box, w.lx)
        fof.fof_link(f.ctx)
        fof.fof_finalize(f.ctx, label, size)
    torch.cuda.synchronize()
    phases = []
    start = t.event()
    for _ in range(steps):
        e0 = t.event()
        fof.fof_build_cells(f.ctx, pos, w.offsets, w.box, w.lx)
        e1 = t.event()
        fof.fof_link(f.ctx)
        e2 = t.event()
        fof.fof_finalize(f.ctx, label, size)
        e3 = t.event()
        phases.append((e0, e1, e2, e3))
    end = t.event()
    torch.cuda.synchronize()
    total = start.elapsed_time(end)
    build = [a.elapsed_time(b) for a, b, _, _ in phases]
    link = [b.elapsed_time(c) for _, b, c, _ in phases]
    fin = [c.elapsed_time(d) for _, _, c, d in phases]
    return total, build, link, fin


def source_sha() -> str:
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_sha") != source_sha():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(w):
    """The oracle (single thread, as it stands) on a bounded sample: the
    sub-cube [0, 1/2)^3 of the same input, scaled by 2 into a unit box with
    l_x scaled by 2 (same density and clustering, 1/8 of the particles)."""
    import numpy as np

    import oracle

    keep = np.all(w.pos < 0.5, axis=1)
    sub = np.ascontiguousarray(w.pos[keep] * np.float32(2.0))
    lx = float(w.lx[0]) * 2.0
    t0 = time.perf_counter()
    ref = oracle.fof(sub, lx)
    dt = time.perf_counter() - t0
    return sub, lx, ref, {"value": len(sub) / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
                          "sample": f"sub-cube [0,1/2)^3 of {w.name} ({len(sub)} particles) scaled x2 into a unit box, "
                                    f"l_x x2; single-threaded C oracle, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2003_11468_amd as fof
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    log(f"generating {args.workload}")
    w = synth.make(args.workload)
    pos = torch.from_numpy(w.pos).to(dev)
    n = w.n

    # --- FP32 filter (the measured form) -----------------------------------
    f = fof.FoF("fp32_filter", cell_factor=args.cell_factor)
    label, size = f.outputs(n)
    log("timing fp32_filter")
    total, build, link, fin = time_pipeline(torch, fof, f, pos, w, args.steps, args.warmup, label, size)
    ms = total / args.steps
    groups = int(f.n_groups(w.n_boxes).sum())
    lab32 = label.cpu().numpy()
    size32 = size.cpu().numpy()
    f.close()

    # pair-test count of the same configuration (stats build of the link pass)
    fs = fof.FoF("fp32_filter", cell_factor=args.cell_factor, stats=True)
    fs.run(pos, w.offsets, w.box, w.lx)
    st = fs.stats()
    fs.close()

    # --- plain FP64 on the same workload -----------------------------------
    plain = None
    exact = None
    if not args.no_plain:
        log("timing fp64")
        f64 = fof.FoF("fp64", cell_factor=args.cell_factor)
        l64, s64 = f64.outputs(n)
        t64, _, link64, _ = time_pipeline(torch, fof, f64, pos, w, max(3, args.steps // 2), 1, l64, s64)
        ms64 = t64 / max(3, args.steps // 2)
        exact = bool(np.array_equal(l64.cpu().numpy(), lab32) and np.array_equal(s64.cpu().numpy(), size32))
        plain = {"value": n / (ms64 * 1e-3), "unit": "particles/s", "ms_per_step": ms64,
                 "link_ms": statistics.median(link64), "fp32_speedup": ms64 / ms}
        f64.close()

    # --- roofline of the dominant kernel -----------------------------------
    phase = {"build": statistics.median(build), "link": statistics.median(link), "finalize": statistics.median(fin)}
    link_ms = phase["link"]
    tests = st["pair_tests"]
    achieved = tests * FLOP_PER_PAIR_TEST / (link_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": measured_traffic("k_link"),
                "kernel": "k_link", "pair_tests": tests, "pair_tests_per_s": tests / (link_ms * 1e-3),
                "kernel_ms": link_ms}

    # --- batched form --------------------------------------------------------
    batched = None
    if not args.no_batched:
        log("generating batched256")
        wb = synth.make("batched256")
        pb = torch.from_numpy(wb.pos).to(dev)
        fb = fof.FoF("fp32_filter")
        lb, sb = fb.outputs(wb.n)
        fb.capture(pb, wb.offsets, wb.box, wb.lx, lb, sb)
        tm = Timer(torch, fb.stream)
        for _ in range(args.warmup):
            fb.replay()
        torch.cuda.synchronize()
        nb_steps = max(3, args.steps // 2)
        e0 = tm.event()
        for _ in range(nb_steps):
            fb.replay()
        e1 = tm.event()
        torch.cuda.synchronize()
        msb = e0.elapsed_time(e1) / nb_steps
        lab_b = lb.cpu().numpy()
        fb.close()
        batched = {"workload": "batched256", "n_boxes": wb.n_boxes, "n_particles": wb.n,
                   "fp32_graph": {"value": wb.n / (msb * 1e-3), "ms_per_step": msb}}
        if not args.no_plain:
            # plain path: FP64 predicate, one launch sequence per box, no graph
            fp = fof.FoF("fp64")
            lp, sp = fp.outputs(wb.n)
            sizes = np.diff(wb.offsets)
            fp.reserve(np.array([0, int(sizes.max())]), 1.0, float(wb.lx.min()))
            views = [(pb[wb.offsets[k]:wb.offsets[k + 1]], lp[wb.offsets[k]:wb.offsets[k + 1]],
                      sp[wb.offsets[k]:wb.offsets[k + 1]]) for k in range(wb.n_boxes)]

            def per_box():
                for k, (pk, lk, sk) in enumerate(views):
                    off = [0, int(sizes[k])]
                    fof.fof_build_cells(fp.ctx, pk, off, wb.box[k], wb.lx[k])
                    fof.fof_link(fp.ctx)
                    fof.fof_finalize(fp.ctx, lk, sk)

            per_box()
            torch.cuda.synchronize()
            e0 = tm.event()
            for _ in range(nb_steps):
                per_box()
            e1 = tm.event()
            torch.cuda.synchronize()
            msp = e0.elapsed_time(e1) / nb_steps
            same = bool(np.array_equal(lp.cpu().numpy(), lab_b))
            batched["plain_fp64_per_box"] = {"value": wb.n / (msp * 1e-3), "ms_per_step": msp}
            batched["speedup"] = msp / msb
            batched["exact_vs_plain"] = same
            fp.close()

    # --- CPU baseline and exactness on the sample ---------------------------
    cpu = None
    sample_exact = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        sub, lx_sub, ref, cpu = cpu_baseline(w)
        lab_s, size_s, ng_s = fof.label(torch.from_numpy(sub).to(dev), lx_sub)
        sample_exact = bool(np.array_equal(lab_s.cpu().numpy(), ref[0]) and
                            np.array_equal(size_s.cpu().numpy(), ref[1]) and ng_s == ref[2])

    out = {
        "metric": METRIC,
        "value": n / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_particles": n, "box": 1.0, "lx": float(w.lx[0]),
                   "b": w.meta.get("b"), "halo_frac": w.meta.get("halo_frac"), "predicate": "fp32_filter",
                   "n_cells": st["n_cells"], "parallelism": "single GPU"},
        "phases_ms": phase,
        "n_groups": groups,
        "stats": {k: st[k] for k in ("pair_tests", "links", "band_hits", "cas_retries")},
        "guard_band_hit_fraction": {"per_test": st["band_hits"] / max(1, st["pair_tests"]),
                                    "per_link": st["band_hits"] / max(1, st["links"])},
        "roofline": roofline,
        "plain_fp64": plain,
        "exact_fp32_vs_fp64": exact,
        "batched": batched,
        "cpu_baseline": cpu,
        "exact_vs_oracle_on_sample": sample_exact,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
