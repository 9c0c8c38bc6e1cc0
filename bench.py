"""Throughput benchmark: particles/s labelled by periodic Friends-of-Friends on
one MI355X, the FP32-filter + batched form against the plain all-FP64 path,
exact labels.

Headline workload: ``batched256`` -- 256 independent periodic boxes of
log-uniform size in [1e3, 1e6] particles (34.3M in all), each with 60 % of its
particles in Plummer halos (counts ~ M^-1.9 on [20, 1e5]) and 40 % uniform,
l_x = 0.2 x that box's mean separation. One step = fof_build_cells + fof_link
+ fof_finalize over all boxes, captured once in a HIP graph and replayed,
positions already in HBM, labels and sizes left in HBM. Cell size, dense-cell
threshold and the work-schedule options are autotuned beforehand (untimed).

Beside it, in the same JSON line: the all-FP64 path in the same graph form
(the filter's own gain), the plain all-FP64 path box by box without a graph,
per-kernel device times from HIP events on the launch stream (eager steps of
the same configuration: the graph replays the same launches), the roofline of
the dominant kernel, the oracle on a bounded sample of the boxes over the
host threads, and side lines for clustered256 (16.8M), clustered512 (134M,
guard-band hit fraction, FP32 == FP64), percolate1024 and lattice1024 (1.07B,
union-find contention).

Prints one JSON line. ``--gpus`` above 1 is refused: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s FoF labelled on 1 MI355X: FP32-filter+batched vs plain FP64, exact"
# Peaks (vendor figures): FP32 vector 157.3 TFLOP/s (256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed)
# x 2.4 GHz); without packed math, which this build does not emit, half of that; HBM3E 8 TB/s.
FP32_VALU_PEAK_TFLOPS = 157.3
FP32_UNPACKED_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
FLOP_PER_PAIR_TEST = 8            # 3 sub, 3 mul, 2 add (an FMA counts as mul + add)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2003_11468_amd", "csrc", f)
                  for f in ("fof_kernels.hip", "fof_link.hip", "fof_device.h", "fof_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")   # {workload: per-kernel counter bytes}


def algorithmic_bytes(kernel: str, n: int, cells: int, nonroot: int, edges: int):
    """Bytes each HBM-bound pass must move at minimum (reads + writes)."""
    segments = -(-cells // 16384)
    table = {
        "k_clear": 4 * segments,
        "k_bucket_hist": 12 * n,                  # xyz in (bucket histogram stays in LDS)
        "k_bucket_scatter": n * (12 + 16 + 4),    # xyz in; staged xyz + index, staging slot out
        "k_seg_hist": 16 * n,                     # staged particle in (segment histogram stays in LDS)
        "k_seg_scan": 8 * segments,
        "k_seg_scatter": n * (16 + 16 + 4),       # staged particle in; segment-ordered particle + slot out
        # segment-ordered particle + slot in; sorted xyz, perm, parent, size, slot map out; the starts
        # of the occupied cells (at most one per particle) and the occupancy words (8 B per 32 cells) out
        "k_cell_sort": n * (16 + 4 + 16 + 8 + 4 + 4 + 4) + 4 * min(n, cells) + cells // 4,
        "k_union_edges": 8 * edges,
        "k_flatten": 4 * n + nonroot * (4 + 4 + 8),  # parent in; root out, perm in, two atomics per non-root
        "k_resolve": n * (4 + 8 + 4 + 8),         # parent, perm, staging slot in; label+size per staging slot out
        "k_gather": n * (4 + 8 + 8),              # staging slot, label+size in; label, size out
    }
    return table.get(kernel)


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def event(torch, stream):
    e = torch.cuda.Event(enable_timing=True)
    e.record(stream)
    return e


def code_only(text: str) -> str:
    """Source text without its comments and with runs of white space folded,
    so that an edit to comments alone keeps the hash of the kernels."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(code_only(open(f).read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from committed rocprofv3
    counters, if they were taken on the current kernel sources (else None)."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    w = d.get(workload, {})
    if w.get("source_sha") != source_sha():
        return None
    k = w.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _kernel_key(name: str) -> str:
    """`void fof::(anonymous namespace)::k_link_sparse<false, false>(fof::Plan)` -> `k_link_sparse<false, false>`."""
    head = name.split("(fof::")[0].split("(int const*")[0]
    head = head.rsplit("::", 1)[-1] if "::" in head.split("<")[0] else head
    return head.strip()


def ingest_counters(d: str, workload: str) -> str:
    """Per-kernel HBM traffic from a rocprofv3 FETCH_SIZE run and a WRITE_SIZE
    run (KiB per dispatch), each scaled by what the counter reads for a copy
    of known size in the same run; average durations from the kernel-trace
    run. Writes TRAFFIC_FILE and returns a markdown summary."""
    import csv
    import collections

    def rows(sub, fname):
        return list(csv.DictReader(open(os.path.join(d, sub, fname))))

    vals = {}
    for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        per = collections.defaultdict(list)
        for r in rows(sub, "run_counter_collection.csv"):
            if r["Counter_Name"] == ctr:
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        vals[ctr] = per
    copies = vals["FETCH_SIZE"].get("__amd_rocclr_copyBuffer", [])
    fills = [v for k, vs in vals["WRITE_SIZE"].items() if "FillFunctor" in k for v in vs]
    if not copies or not fills:
        raise SystemExit("no calibration copy/fill in the counter runs (use --copy-calibration)")
    cal_kib = max(fills)                       # the fill writes exactly the calibration buffer
    fetch_factor = cal_kib / max(copies)       # the copy reads it once
    write_factor = cal_kib / max(fills)
    stats = {}
    for r in rows("trace", "run_kernel_stats.csv"):
        stats[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]))
    kernels = {}
    lines = ["| kernel | calls | avg us | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB (scaled) | GB/s |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for name, (calls, avg_ns) in sorted(stats.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
        f = vals["FETCH_SIZE"].get(name)
        w = vals["WRITE_SIZE"].get(name)
        if not f or not w or "fof::" not in name:
            continue
        fk, wk = statistics.mean(f), statistics.mean(w)
        b = (fk * fetch_factor + wk * write_factor) * 1024.0
        key = _kernel_key(name)
        lines.append(f"| `{key}` | {calls} | {avg_ns / 1e3:.1f} | {fk:.0f} | {wk:.0f} | {b / 1e6:.1f} | "
                     f"{b / avg_ns:.0f} |")
        base = key.split("<")[0]
        # the variant launched most often (the timed one) names the kernel
        if base not in kernels or calls > kernels[base]["calls"]:
            kernels[base] = {"calls": calls, "avg_ns": avg_ns, "bytes_per_launch": b, "variant": key}
    out = {"source_sha": source_sha(), "fetch_factor": fetch_factor, "write_factor": write_factor,
           "calibration_kib": cal_kib, "kernels": kernels}
    try:
        table = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        table = {}
    table[workload] = out
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    head = [f"Calibration: a {cal_kib / 1024:.0f} MiB fill reads WRITE_SIZE {max(fills):.0f} KiB "
            f"(factor {write_factor:.3f}); a copy of it reads FETCH_SIZE {max(copies):.0f} KiB "
            f"(factor {fetch_factor:.3f}).", ""]
    return "\n".join(head + lines) + "\n"


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched256", help="the headline workload")
    ap.add_argument("--eager", action="store_true", help="time the headline eagerly instead of as a graph")
    ap.add_argument("--cell-factor", type=float, default=None, help="skip tuning, use this cell size")
    ap.add_argument("--dense-min", type=int, default=None, help="skip tuning, use this dense threshold")
    ap.add_argument("--schedule", type=int, default=0, help="with --cell-factor and --dense-min: fof_options.schedule")
    ap.add_argument("--link-order", default="index", choices=("index", "random"),
                    help="with --cell-factor and --dense-min: hooking order")
    ap.add_argument("--compression", default="halving", choices=("halving", "depth2"),
                    help="with --cell-factor and --dense-min: path compression of the finds")
    ap.add_argument("--segment-log2", type=int, default=0, help="with --cell-factor and --dense-min: cell sort segments")
    ap.add_argument("--no-side", action="store_true", help="only the headline workload")
    ap.add_argument("--no-large", action="store_true", help="no 134M and 1.07B side workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-domains", action="store_true")
    ap.add_argument("--no-relink", action="store_true")
    ap.add_argument("--domains", type=int, default=8, help="slabs of the domain-decomposed measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (a known-size kernel whose "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE calibrates the counters)")
    ap.add_argument("--ingest-counters", metavar="DIR", default=None,
                    help="no GPU work: read rocprofv3 CSV output under DIR/{trace,fetch,write} (kernel trace, "
                         "FETCH_SIZE and WRITE_SIZE runs of the same command, with --copy-calibration), add "
                         "the workload's entry to profiles/traffic.json and print a markdown summary")
    ap.add_argument("--counter-workload", default="batched256", help="the workload the counters were taken on")
    ap.add_argument("--summarize-sq", metavar="DIR", nargs="+", default=None,
                    help="no GPU work: per-kernel table of the SQ counters in the rocprofv3 counter CSVs under "
                         "the given directories (instructions per wave, VALU busy share, wait share)")
    return ap.parse_args()


# fof.FoF keyword arguments a tuned configuration may carry
FOF_KEYS = ("cell_factor", "dense_min", "schedule", "link_order", "compression", "segment_log2")


def fof_kwargs(cfg: dict) -> dict:
    return {k: cfg[k] for k in FOF_KEYS if k in cfg}


def summarize_sq(dirs) -> str:
    """Markdown table of SQ counters per kernel (mean over dispatches) from
    rocprofv3 --pmc runs: VALU, SALU, LDS and vector-memory instructions per
    wave, VALU instructions per dispatch, and the share of wave cycles spent
    waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES)."""
    import csv
    import collections

    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if "fof::" in r["Kernel_Name"]:
                vals[_kernel_key(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["| kernel | waves | VALU/wave | SALU/wave | LDS/wave | VMEM rd/wave | VALU total | wait share |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]

    def mean(c, k):
        v = vals[k].get(c)
        return statistics.mean(v) if v else None

    for k in sorted(vals, key=lambda k: -(mean("SQ_WAVE_CYCLES", k) or 0)):
        waves = mean("SQ_WAVES", k)
        if not waves:
            continue
        cell = []
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD"):
            m = mean(c, k)
            cell.append("-" if m is None else f"{m / waves:.0f}")
        wa, wc = mean("SQ_WAIT_ANY", k), mean("SQ_WAVE_CYCLES", k)
        wait = "-" if wa is None or not wc else f"{wa / wc:.2f}"
        tv = mean("SQ_INSTS_VALU", k)
        lines.append(f"| `{k}` | {waves:.0f} | " + " | ".join(cell) + f" | {0 if tv is None else tv:.3g} | {wait} |")
    return "\n".join(lines) + "\n"


def choose(tune, pos, w, predicate, args, **kw):
    """The autotuner's configuration for this input (untimed), or the one
    given on the command line."""
    if args.cell_factor is not None and args.dense_min is not None:
        return {"cell_factor": args.cell_factor, "dense_min": args.dense_min, "schedule": args.schedule,
                "link_order": args.link_order, "compression": args.compression, "segment_log2": args.segment_log2,
                "tuned": False}
    t0 = time.perf_counter()
    r = tune.autotune(pos, w.offsets, w.box, w.lx, predicate, cache_path=None, repeats=2, **kw)
    out = {k: r[k] for k in r if k in FOF_KEYS}
    out.update(tuned=True, tuning_s=round(time.perf_counter() - t0, 2), candidates=len(r["tried"]))
    return out


def timed(torch, stream, step, steps, warmup, kernel_times=None):
    """Mean ms of `steps` calls of step() between two HIP events on `stream`,
    after `warmup` untimed calls; per-kernel times of that region when
    kernel_times (the context's reader) is given; then the median and standard
    deviation of single steps from as many calls again, each between events
    (outside the timed region)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if kernel_times:
        kernel_times()   # drop the warm-up record
    start = event(torch, stream)
    for _ in range(steps):
        step()
    end = event(torch, stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / max(1, steps)
    kern = None
    if kernel_times:
        kern = {k: (t / c, c) for k, (t, c) in kernel_times().items() if c}
    marks = [event(torch, stream)]
    for _ in range(steps):
        step()
        marks.append(event(torch, stream))
    torch.cuda.synchronize()
    if kernel_times:
        kernel_times()
    per = [a.elapsed_time(b) for a, b in zip(marks[:-1], marks[1:])]
    spread = {"ms_per_step_median": statistics.median(per) if per else None,
              "ms_per_step_std": statistics.stdev(per) if len(per) > 1 else 0.0}
    return ms, kern, spread


def eager_step(fof, f, pos, w, label, size):
    def step():
        fof.fof_build_cells(f.ctx, pos, w.offsets, w.box, w.lx)
        fof.fof_link(f.ctx)
        fof.fof_finalize(f.ctx, label, size)
    return step


def stats_of(fof, pos, w, predicate, cfg):
    fs = fof.FoF(predicate, stats=True, **fof_kwargs(cfg))
    try:
        label, size, _ = fs.run(pos, w.offsets, w.box, w.lx)
        st = fs.stats()
        st["largest_group"] = int(size.max().item()) if w.n else 0
        return st
    finally:
        fs.close()


def kernel_table(kern, w, st, groups):
    """Per-kernel mean device time; achieved GB/s for the HBM-bound passes."""
    out = {}
    for k, (avg_ms, count) in kern.items():
        b = algorithmic_bytes(k, w.n, st["n_cells"], w.n - groups, st["queued_links"])
        out[k] = {"ms": round(avg_ms, 4)}
        if b is not None:
            out[k]["GB/s"] = round(b / (avg_ms * 1e-3) / 1e9, 1)
            out[k]["hbm_frac"] = round(b / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
    return out


def roofline_of(kern, w, st, groups, workload):
    """Roofline of the kernel with the largest device time: pair-test kernels
    against the FP32 vector peak (8 flop per pair test), the others against
    HBM with their algorithmic bytes."""
    dom = max(kern.items(), key=lambda kv: kv[1][0])[0]
    dom_ms = kern[dom][0]
    if dom in ("k_link_sparse", "k_link_dense"):
        tests = st["sparse_pair_tests"] if dom == "k_link_sparse" else st["pair_tests"] - st["sparse_pair_tests"]
        achieved = tests * FLOP_PER_PAIR_TEST / (dom_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": measured_traffic(dom, workload),
                "kernel": dom, "kernel_ms": dom_ms, "pair_tests_per_launch": tests,
                "flop_per_pair_test": FLOP_PER_PAIR_TEST, "pair_tests_per_s": tests / (dom_ms * 1e-3),
                "frac_of_unpacked_fp32": achieved / FP32_UNPACKED_PEAK_TFLOPS}
    b = algorithmic_bytes(dom, w.n, st["n_cells"], w.n - groups, st["queued_links"])
    achieved = b / (dom_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, workload), "kernel": dom, "kernel_ms": dom_ms, "bytes_per_launch": b}


def contention(st, n):
    return {k: st[k] for k in ("pair_tests", "links", "band_hits", "cas_retries", "queued_links", "dense_items",
                               "find_depth_max", "largest_group")} | {
        "find_depth_mean": st["find_depth_sum"] / max(1, n),
        "guard_band_hit_fraction": {"per_test": st["band_hits"] / max(1, st["pair_tests"]),
                                    "per_link": st["band_hits"] / max(1, st["links"])}}


def host_info():
    model = "?"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "threads_available": len(os.sched_getaffinity(0))}


def host_threads():
    return max(1, min(16, len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16"))))


def same(a, b):
    return bool(all(np.array_equal(x, y) for x, y in zip(a, b)))


def cpu_baseline_boxes(w, lab, siz, ng):
    """The oracle (as it stands) on a bounded sample of the batch, every
    fourth box, one box per host thread; and whether the GPU's labels, sizes
    and group counts on those boxes equal the oracle's."""
    import oracle

    sizes = np.diff(w.offsets)
    sel = np.arange(0, w.n_boxes, 4)
    pos = np.concatenate([w.pos[w.offsets[k]:w.offsets[k + 1]] for k in sel])
    off = np.concatenate([[0], np.cumsum(sizes[sel])]).astype(np.int64)
    threads = host_threads()
    t0 = time.perf_counter()
    ref = oracle.fof_boxes(pos, off, np.asarray(w.box)[sel], np.asarray(w.lx)[sel], threads=threads)
    dt = time.perf_counter() - t0
    got = (np.concatenate([lab[w.offsets[k]:w.offsets[k + 1]] for k in sel]),
           np.concatenate([siz[w.offsets[k]:w.offsets[k + 1]] for k in sel]), np.asarray(ng)[sel])
    return {"value": int(off[-1]) / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"every fourth box of {w.name} ({len(sel)} boxes, {int(off[-1])} particles), one box per "
                      f"thread on {threads} host threads (sequential oracle per box), {dt:.1f} s"}, same(got, ref)


# ------------------------------------------------------------- workloads --

def headline(args, torch, fof, tune, synth, dev):
    log(f"generating {args.workload}")
    w = synth.make(args.workload)
    pos = torch.from_numpy(w.pos).to(dev)
    n = w.n
    log("tuning fp32_filter")
    cfg = choose(tune, pos, w, "fp32_filter", args)
    graph = not args.eager

    def run_form(predicate, c):
        f = fof.FoF(predicate, **fof_kwargs(c))
        label, size = f.outputs(n)
        if graph:
            f.capture(pos, w.offsets, w.box, w.lx, label, size)
            step = f.replay
        else:
            f.reserve(w.offsets, w.box, w.lx)
            step = eager_step(fof, f, pos, w, label, size)
        ms, _, spread = timed(torch, f.stream, step, args.steps, args.warmup)
        ng = f.n_groups(w.n_boxes)
        res = (label.cpu().numpy(), size.cpu().numpy(), ng)
        f.close()
        return ms, spread, res

    form = "hip_graph" if graph else "eager"
    log(f"timing fp32_filter ({form}) {cfg}")
    ms, spread, res32 = run_form("fp32_filter", cfg)
    groups = int(np.sum(res32[2]))

    # per-kernel device times: eager steps of the same configuration, HIP
    # events around every launch on the context's stream
    log("per-kernel times (eager, same configuration)")
    fe = fof.FoF("fp32_filter", timings=True, **fof_kwargs(cfg))
    le, se = fe.outputs(n)
    fe.reserve(w.offsets, w.box, w.lx)
    ms_eager, kern, _ = timed(torch, fe.stream, eager_step(fof, fe, pos, w, le, se), max(3, args.steps // 2), 1,
                              fe.kernel_times)
    fe.close()
    st = stats_of(fof, pos, w, "fp32_filter", cfg)

    out = {
        "metric": METRIC, "value": n / (ms * 1e-3), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, **spread, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n_boxes": w.n_boxes, "n_particles": n, "box": 1.0, "b": w.meta.get("b"),
                   "halo_frac": w.meta.get("halo_frac"), "predicate": "fp32_filter", "form": form,
                   **{k: v for k, v in cfg.items() if k in FOF_KEYS}, "tuned": cfg.get("tuned"),
                   "n_cells": st["n_cells"], "parallelism": "single GPU"},
        "n_groups": groups,
        "kernels": kernel_table(kern, w, st, groups),
        "kernels_from": f"eager steps of the same configuration ({ms_eager:.3f} ms per step; the graph replays "
                        "the same launches)",
        "stats": contention(st, n),
        "roofline": roofline_of(kern, w, st, groups, w.name),
        "tuning": {k: v for k, v in cfg.items() if k not in FOF_KEYS},
    }
    exact = {}
    if not args.no_plain:
        log("tuning fp64")
        cfg64 = choose(tune, pos, w, "fp64", args)
        log(f"timing fp64 ({form}) {cfg64}")
        ms64, _, res64 = run_form("fp64", cfg64)
        exact["fp32_filter_vs_fp64"] = same(res32, res64)
        out["fp64_same_form"] = {"value": n / (ms64 * 1e-3), "ms_per_step": ms64, "form": form,
                                 **{k: v for k, v in cfg64.items() if k in FOF_KEYS},
                                 "fp32_filter_speedup": ms64 / ms}
        if w.n_boxes > 1:
            # the plain path: FP64 predicate, one launch sequence per box, no graph
            log("timing fp64 box by box, no graph")
            fp = fof.FoF("fp64", **fof_kwargs(cfg64))
            lp, sp = fp.outputs(n)
            sizes = np.diff(w.offsets)
            need = max(fof.fof_workspace_bytes(fp.ctx, [0, int(sizes[k])], w.box[k], w.lx[k])
                       for k in range(w.n_boxes))
            fp.ws = torch.empty(need, dtype=torch.uint8, device=dev)
            fof.fof_set_workspace(fp.ctx, fp.ws)
            views = [(pos[w.offsets[k]:w.offsets[k + 1]], lp[w.offsets[k]:w.offsets[k + 1]],
                      sp[w.offsets[k]:w.offsets[k + 1]]) for k in range(w.n_boxes)]
            ng_plain = np.zeros(w.n_boxes, dtype=np.int64)

            def per_box():
                for k, (pk, lk, sk) in enumerate(views):
                    fof.fof_build_cells(fp.ctx, pk, [0, int(sizes[k])], w.box[k], w.lx[k])
                    fof.fof_link(fp.ctx)
                    fof.fof_finalize(fp.ctx, lk, sk)

            msp, _, _ = timed(torch, fp.stream, per_box, max(3, args.steps // 4), 1)
            for k, (pk, lk, sk) in enumerate(views):   # group counts, outside the timed region
                fof.fof_build_cells(fp.ctx, pk, [0, int(sizes[k])], w.box[k], w.lx[k])
                fof.fof_link(fp.ctx)
                ng_plain[k] = fof.fof_finalize(fp.ctx, lk, sk, 1)[0]
            exact["fp32_filter_vs_plain_per_box"] = same(res32, (lp.cpu().numpy(), sp.cpu().numpy(), ng_plain))
            out["plain_fp64_per_box"] = {"value": n / (msp * 1e-3), "ms_per_step": msp, "form": "eager, box by box",
                                         "speedup_of_headline": msp / ms}
            fp.close()
    del pos
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline and w.n_boxes > 1:
        log("cpu baseline: oracle on every fourth box over the host threads")
        out["cpu_baseline"], exact["vs_oracle_on_sample"] = cpu_baseline_boxes(w, *res32)
    out["exact"] = exact
    return out


def side_clustered256(args, torch, fof, tune, synth, dev):
    """clustered256: the single-box form, both predicates, the roofline of its
    dominant kernel, the oracle on the whole input (single thread), the group
    catalogue, the domain-decomposed merge and a relink."""
    w = synth.make("clustered256")
    pos = torch.from_numpy(w.pos).to(dev)
    n = w.n
    log("clustered256: tuning and timing both predicates")
    res, line = {}, {"n_particles": n}
    for predicate in ("fp32_filter", "fp64"):
        cfg = choose(tune, pos, w, predicate, args)
        f = fof.FoF(predicate, timings=True, **fof_kwargs(cfg))
        label, size = f.outputs(n)
        f.reserve(w.offsets, w.box, w.lx)
        ms, kern, spread = timed(torch, f.stream, eager_step(fof, f, pos, w, label, size), args.steps, args.warmup,
                                 f.kernel_times)
        ng = f.n_groups(1)
        if predicate == "fp32_filter":
            line["catalogue"] = {"min_size": 21, "groups": fof.fof_catalogue(f.ctx, label, size, 21)}
        res[predicate] = (label.cpu().numpy(), size.cpu().numpy(), ng)
        f.close()
        st = stats_of(fof, pos, w, predicate, cfg)
        groups = int(ng[0])
        line[predicate] = {"value": n / (ms * 1e-3), "ms_per_step": ms, **spread,
                           **{k: v for k, v in cfg.items() if k in FOF_KEYS},
                           "kernels": kernel_table(kern, w, st, groups),
                           "roofline": roofline_of(kern, w, st, groups, "clustered256")}
        if predicate == "fp32_filter":
            line["stats"] = contention(st, n)
            cfg32 = cfg
    line["fp32_filter_speedup"] = line["fp64"]["ms_per_step"] / line["fp32_filter"]["ms_per_step"]
    line["exact_fp32_filter_vs_fp64"] = same(res["fp32_filter"], res["fp64"])
    if not args.no_domains:
        log("clustered256: domain-decomposed merge")
        fd = fof.FoF("fp32_filter", domains=args.domains, **fof_kwargs(cfg32))
        ld, sd = fd.outputs(n)
        fd.reserve(w.offsets, w.box, w.lx)
        msd, _, _ = timed(torch, fd.stream, eager_step(fof, fd, pos, w, ld, sd), max(3, args.steps // 2), 1)
        fd.close()
        fds = fof.FoF("fp32_filter", stats=True, domains=args.domains, **fof_kwargs(cfg32))
        fds.run(pos, w.offsets, w.box, w.lx)
        std = fds.stats()
        fds.close()
        line["domain_decomposed"] = {"domains": args.domains, "value": n / (msd * 1e-3), "ms_per_step": msd,
                                     "boundary_links": std["boundary_links"],
                                     "boundary_groups": std["boundary_groups"],
                                     "exact_vs_single_domain": same(res["fp32_filter"][:2],
                                                                    (ld.cpu().numpy(), sd.cpu().numpy()))}
    if not args.no_relink:
        log("clustered256: relink at b = 0.16")
        fr = fof.FoF("fp32_filter", **fof_kwargs(cfg32))
        lr, sr = fr.outputs(n)
        fr.run(pos, w.offsets, w.box, w.lx)
        lx_r = [float(v) * 0.8 for v in w.lx]

        def relink():
            fof.fof_relink(fr.ctx, lx_r, 1)
            fof.fof_link(fr.ctx)
            fof.fof_finalize(fr.ctx, lr, sr)

        msr, _, _ = timed(torch, fr.stream, relink, max(3, args.steps // 2), 1)
        line["relink"] = {"b": 0.16, "ms_per_step": msr, "value": n / (msr * 1e-3),
                          "n_groups": int(fr.n_groups(1).sum())}
        fr.close()
    del pos
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        import oracle

        log("clustered256: the oracle on the whole input, one thread")
        t0 = time.perf_counter()
        ref = oracle.fof(w.pos, float(w.lx[0]))
        dt = time.perf_counter() - t0
        line["cpu_oracle_single_thread"] = {"value": n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
                                            "sample": f"the whole of clustered256 ({n} particles), {dt:.1f} s"}
        line["exact_vs_oracle"] = same(res["fp32_filter"][:2], ref[:2]) and int(res["fp32_filter"][2][0]) == ref[2]
    return line


def side_large(args, torch, fof, tune, synth, dev, name, both, steps):
    """A large input, few steps: time per step, statistics (guard band,
    contention), and with both=True whether the FP32 filter and the all-FP64
    path give the same labels."""
    log(f"{name}: generating")
    w = synth.make(name)
    pos = torch.from_numpy(w.pos).to(dev)
    n = w.n
    line = {"n_particles": n}
    res = {}
    for predicate in (("fp32_filter", "fp64") if both else ("fp32_filter",)):
        # a reduced search at this size: three cell sizes, two thresholds, and
        # whether to skip the giant group
        cfg = choose(tune, pos, w, predicate, args, cell_factors=(0.0, 1.5, 2.0), dense_mins=(16, 32),
                     axes={"schedule": (0, fof.schedule_bits(giant_skip=True))})
        log(f"{name}: {predicate} {cfg}")
        f = fof.FoF(predicate, **fof_kwargs(cfg))
        label, size = f.outputs(n)
        f.reserve(w.offsets, w.box, w.lx)
        ms, _, _ = timed(torch, f.stream, eager_step(fof, f, pos, w, label, size), steps, 1)
        ng = f.n_groups(1)
        res[predicate] = (label.cpu().numpy(), size.cpu().numpy(), ng) if both else None
        f.close()
        del label, size
        torch.cuda.empty_cache()
        line[predicate] = {"value": n / (ms * 1e-3), "ms_per_step": ms, "n_groups": int(ng[0]),
                           **{k: v for k, v in cfg.items() if k in FOF_KEYS}}
        if predicate == "fp32_filter":
            line["stats"] = contention(stats_of(fof, pos, w, predicate, cfg), n)
            torch.cuda.empty_cache()
    if both:
        line["exact_fp32_filter_vs_fp64"] = same(res["fp32_filter"], res["fp64"])
    del pos
    torch.cuda.empty_cache()
    return line


def main():
    args = parse()
    if args.ingest_counters:
        print(ingest_counters(args.ingest_counters, args.counter_workload), end="")
        return
    if args.summarize_sq:
        print(summarize_sq(args.summarize_sq), end="")
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2003_11468_amd as fof
    import synth
    from paper_2003_11468_amd import tune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = headline(args, torch, fof, tune, synth, dev)
    out["host"] = host_info()
    if not args.no_side:
        side = {"clustered256": side_clustered256(args, torch, fof, tune, synth, dev)}
        if not args.no_large:
            side["clustered512"] = side_large(args, torch, fof, tune, synth, dev, "clustered512", True, 5)
            side["percolate1024"] = side_large(args, torch, fof, tune, synth, dev, "percolate1024", False, 3)
            side["lattice1024"] = side_large(args, torch, fof, tune, synth, dev, "lattice1024", False, 3)
        out["side"] = side
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
