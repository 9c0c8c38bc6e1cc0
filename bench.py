"""Throughput benchmark: particles/s labelled by periodic Friends-of-Friends on
one MI355X, FP32-filter path against the plain all-FP64 path, exact labels.

Workload (default): ``clustered256`` -- N = 256^3 FP32 positions in a periodic
unit box, 60 % in Plummer halos (counts ~ M^-1.9 on [20, 1e5]), 40 % uniform,
l_x = 0.2 x mean separation. One step = fof_build_cells + fof_link +
fof_finalize over the whole input, positions already in HBM, labels and sizes
left in HBM. Cell size and dense-cell threshold are autotuned beforehand
(untimed) for each path. The batched form (256 boxes of log-uniform size in
one HIP graph) and the plain FP64 path are timed beside it and reported in
the same JSON line, with per-kernel device times from HIP events recorded on
the launch stream inside the timed region.

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

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s FoF labelled on 1 MI355X: FP32-filter+batched vs plain FP64, exact"
# Peaks: FP32 vector without packed math = 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz;
# HBM3E 8 TB/s (vendor figures).
FP32_VALU_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
FLOP_PER_PAIR_TEST = 8            # 3 sub, 3 mul, 2 add (an FMA counts as mul + add)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2003_11468_amd", "csrc", f)
                  for f in ("fof_kernels.hip", "fof_link.hip", "fof_device.h", "fof_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


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


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered256")
    ap.add_argument("--cell-factor", type=float, default=None, help="skip tuning, use this cell size")
    ap.add_argument("--dense-min", type=int, default=None, help="skip tuning, use this dense threshold")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-domains", action="store_true")
    ap.add_argument("--no-relink", action="store_true")
    ap.add_argument("--domains", type=int, default=8, help="slabs of the domain-decomposed measurement")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (a known-size kernel whose "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE calibrates the counters)")
    ap.add_argument("--ingest-counters", metavar="DIR", default=None,
                    help="no GPU work: read rocprofv3 CSV output under DIR/{trace,fetch,write} (kernel trace, "
                         "FETCH_SIZE and WRITE_SIZE runs of the same command, with --copy-calibration), write "
                         "profiles/traffic.json and print a markdown summary")
    return ap.parse_args()


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


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel sources (else None)."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_sha") != source_sha():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _kernel_key(name: str) -> str:
    """`void fof::(anonymous namespace)::k_link_sparse<false, false>(fof::Plan)` -> `k_link_sparse<false, false>`."""
    head = name.split("(fof::")[0].split("(int const*")[0]
    head = head.rsplit("::", 1)[-1] if "::" in head.split("<")[0] else head
    return head.strip()


def ingest_counters(d: str) -> str:
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
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    head = [f"Calibration: a {cal_kib / 1024:.0f} MiB fill reads WRITE_SIZE {max(fills):.0f} KiB "
            f"(factor {write_factor:.3f}); a copy of it reads FETCH_SIZE {max(copies):.0f} KiB "
            f"(factor {fetch_factor:.3f}).", ""]
    return "\n".join(head + lines) + "\n"


def choose(torch, tune, pos, w, predicate, args):
    if args.cell_factor is not None and args.dense_min is not None:
        return {"cell_factor": args.cell_factor, "dense_min": args.dense_min, "tuned": False}
    t0 = time.perf_counter()
    r = tune.autotune(pos, w.offsets, w.box, w.lx, predicate, cache_path=None, repeats=2)
    return {"cell_factor": r["cell_factor"], "dense_min": r["dense_min"], "tuned": True,
            "tuning_s": round(time.perf_counter() - t0, 2), "tried": r["tried"]}


def timed_steps(torch, fof, f, pos, w, steps, warmup, label, size):
    f.reserve(w.offsets, w.box, w.lx)
    for _ in range(warmup):
        fof.fof_build_cells(f.ctx, pos, w.offsets, w.box, w.lx)
        fof.fof_link(f.ctx)
        fof.fof_finalize(f.ctx, label, size)
    torch.cuda.synchronize()
    f.kernel_times()   # drop the warm-up record
    start = event(torch, f.stream)
    for _ in range(steps):
        fof.fof_build_cells(f.ctx, pos, w.offsets, w.box, w.lx)
        fof.fof_link(f.ctx)
        fof.fof_finalize(f.ctx, label, size)
    end = event(torch, f.stream)
    torch.cuda.synchronize()
    kt = f.kernel_times()
    # the spread of single steps, from as many steps again with an event
    # after each (kept out of the timed region above)
    marks = [event(torch, f.stream)]
    for _ in range(steps):
        fof.fof_build_cells(f.ctx, pos, w.offsets, w.box, w.lx)
        fof.fof_link(f.ctx)
        fof.fof_finalize(f.ctx, label, size)
        marks.append(event(torch, f.stream))
    torch.cuda.synchronize()
    f.kernel_times()
    per_step = [a.elapsed_time(b) for a, b in zip(marks[:-1], marks[1:])]
    return (start.elapsed_time(end) / max(1, steps), {k: (ms / max(1, c), c) for k, (ms, c) in kt.items() if c},
            per_step)


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
                          "sample": f"sub-cube [0,1/2)^3 of {w.name} ({len(sub)} particles) scaled x2 into a unit "
                                    f"box, l_x x2; single-threaded C oracle, {dt:.1f} s"}


def cpu_baseline_batched(wb, label, size, max_box: int = 50000):
    """The oracle on a bounded sample of the batch: every box of at most
    `max_box` particles (the larger boxes alone would keep one thread busy for
    tens of seconds), boxes spread over the host's threads (one box per thread,
    as many threads as the process may use, at most 16); also whether the
    GPU's labels and sizes on those boxes equal the oracle's."""
    import numpy as np

    import oracle

    sizes = np.diff(wb.offsets)
    sel = np.nonzero(sizes <= max_box)[0]
    pos = np.concatenate([wb.pos[wb.offsets[k]:wb.offsets[k + 1]] for k in sel])
    off = np.concatenate([[0], np.cumsum(sizes[sel])]).astype(np.int64)
    lab = np.concatenate([label[wb.offsets[k]:wb.offsets[k + 1]] for k in sel])
    siz = np.concatenate([size[wb.offsets[k]:wb.offsets[k + 1]] for k in sel])
    threads = max(1, min(16, len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16"))))
    t0 = time.perf_counter()
    ref = oracle.fof_boxes(pos, off, np.asarray(wb.box)[sel], np.asarray(wb.lx)[sel], threads=threads)
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(lab, ref[0]) and np.array_equal(siz, ref[1]))
    return {"value": int(off[-1]) / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"the {len(sel)} boxes of batched256 with at most {max_box} particles ({int(off[-1])} "
                      f"particles), one box per thread on {threads} host threads, {dt:.1f} s"}, exact


def main():
    args = parse()
    if args.ingest_counters:
        print(ingest_counters(args.ingest_counters), end="")
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
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
    log(f"generating {args.workload}")
    w = synth.make(args.workload)
    pos = torch.from_numpy(w.pos).to(dev)
    n = w.n

    # --- FP32 filter (the measured form) -----------------------------------
    log("tuning fp32_filter")
    cfg = choose(torch, tune, pos, w, "fp32_filter", args)
    f = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"], timings=True)
    label, size = f.outputs(n)
    log(f"timing fp32_filter cell_factor={cfg['cell_factor']} dense_min={cfg['dense_min']}")
    ms, kern, per_step = timed_steps(torch, fof, f, pos, w, args.steps, args.warmup, label, size)
    groups = int(f.n_groups(w.n_boxes).sum())
    # group catalogue of the last step (groups of more than 20 members, the paper's cut), not in the step
    cat = {"min_size": 21}
    e0, e1 = event(torch, f.stream), None
    cat["groups"] = fof.fof_catalogue(f.ctx, label, size, 21)
    e1 = event(torch, f.stream)
    torch.cuda.synchronize()
    cat["count_ms"] = round(e0.elapsed_time(e1), 4)
    lab32 = label.cpu().numpy()
    size32 = size.cpu().numpy()
    f.close()

    # counters of the same configuration (a separate stats run, not timed)
    fs = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"], stats=True)
    fs.run(pos, w.offsets, w.box, w.lx)
    st = fs.stats()
    fs.close()

    # --- relink: a shorter linking length (b = 0.16 instead of 0.2) over the
    #     cells of the same build, without rebuilding them ---------------------
    relink = None
    if not args.no_relink:
        log("timing relink at b = 0.16")
        fr = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"])
        lr, sr = fr.outputs(n)
        fr.run(pos, w.offsets, w.box, w.lx)
        lx_r = [float(v) * 0.8 for v in w.lx]
        fr.relink(lx_r, w.n_boxes, lr, sr)   # warm-up
        torch.cuda.synchronize()
        reps = max(3, args.steps // 2)
        e0 = event(torch, fr.stream)
        for _ in range(reps):
            fof.fof_relink(fr.ctx, lx_r, w.n_boxes)
            fof.fof_link(fr.ctx)
            fof.fof_finalize(fr.ctx, lr, sr)
        e1 = event(torch, fr.stream)
        torch.cuda.synchronize()
        msr = e0.elapsed_time(e1) / reps
        relink = {"b": 0.16, "ms_per_step": msr, "value": n / (msr * 1e-3),
                  "n_groups": int(fr.n_groups(w.n_boxes).sum())}
        fr.close()

    # --- domain-decomposed merge (slabs along x, global merge of the links
    #     across them) on the same workload and configuration ----------------
    domain = None
    if not args.no_domains:
        log("timing domain-decomposed merge")
        fd = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"], timings=True,
                     domains=args.domains)
        ld, sd = fd.outputs(n)
        msd, _, _ = timed_steps(torch, fof, fd, pos, w, max(3, args.steps // 2), 1, ld, sd)
        fd.close()
        fds = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"], stats=True,
                      domains=args.domains)
        fds.run(pos, w.offsets, w.box, w.lx)
        std = fds.stats()
        fds.close()
        domain = {"domains": args.domains, "value": n / (msd * 1e-3), "ms_per_step": msd,
                  "boundary_links": std["boundary_links"], "boundary_groups": std["boundary_groups"],
                  "exact_vs_single_domain": bool(np.array_equal(ld.cpu().numpy(), lab32)
                                                 and np.array_equal(sd.cpu().numpy(), size32))}

    # --- plain FP64 on the same workload -----------------------------------
    plain = None
    exact = None
    if not args.no_plain:
        log("tuning fp64")
        cfg64 = choose(torch, tune, pos, w, "fp64", args)
        f64 = fof.FoF("fp64", cell_factor=cfg64["cell_factor"], dense_min=cfg64["dense_min"], timings=True)
        l64, s64 = f64.outputs(n)
        log("timing fp64")
        ms64, kern64, _ = timed_steps(torch, fof, f64, pos, w, max(3, args.steps // 2), 1, l64, s64)
        exact = bool(np.array_equal(l64.cpu().numpy(), lab32) and np.array_equal(s64.cpu().numpy(), size32))
        plain = {"value": n / (ms64 * 1e-3), "unit": "particles/s", "ms_per_step": ms64,
                 "cell_factor": cfg64["cell_factor"], "dense_min": cfg64["dense_min"],
                 "fp32_filter_speedup": ms64 / ms,
                 "kernels_ms": {k: round(v[0], 4) for k, v in kern64.items()}}
        f64.close()

    # --- roofline of the dominant kernel and HBM rates of the passes -------
    nonroot = n - groups
    passes = {}
    for k, (avg_ms, count) in kern.items():
        b = algorithmic_bytes(k, n, st["n_cells"], nonroot, st["queued_links"])
        passes[k] = {"ms": round(avg_ms, 4)}
        if b is not None:
            passes[k]["GB/s"] = round(b / (avg_ms * 1e-3) / 1e9, 1)
            passes[k]["hbm_frac"] = round(b / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
    dom = max(kern.items(), key=lambda kv: kv[1][0])[0]
    dom_ms = kern[dom][0]
    if dom in ("k_link_sparse", "k_link_dense"):
        tests = st["sparse_pair_tests"] if dom == "k_link_sparse" else st["pair_tests"] - st["sparse_pair_tests"]
        achieved = tests * FLOP_PER_PAIR_TEST / (dom_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": measured_traffic(dom), "kernel": dom,
                    "kernel_ms": dom_ms, "pair_tests_per_launch": tests,
                    "flop_per_pair_test": FLOP_PER_PAIR_TEST}
    else:
        b = algorithmic_bytes(dom, n, st["n_cells"], nonroot, st["queued_links"])
        achieved = b / (dom_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom), "kernel": dom,
                    "kernel_ms": dom_ms, "bytes_per_launch": b}

    # --- batched form --------------------------------------------------------
    batched = None
    if not args.no_batched:
        log("generating batched256")
        wb = synth.make("batched256")
        pb = torch.from_numpy(wb.pos).to(dev)
        log("tuning batched fp32_filter")
        cfgb = choose(torch, tune, pb, wb, "fp32_filter", args)
        fb = fof.FoF("fp32_filter", cell_factor=cfgb["cell_factor"], dense_min=cfgb["dense_min"])
        lb, sb = fb.outputs(wb.n)
        fb.capture(pb, wb.offsets, wb.box, wb.lx, lb, sb)
        for _ in range(args.warmup):
            fb.replay()
        torch.cuda.synchronize()
        nb_steps = max(3, args.steps // 2)
        e0 = event(torch, fb.stream)
        for _ in range(nb_steps):
            fb.replay()
        e1 = event(torch, fb.stream)
        torch.cuda.synchronize()
        msb = e0.elapsed_time(e1) / nb_steps
        lab_b = lb.cpu().numpy()
        size_b = sb.cpu().numpy()
        fb.close()
        batched = {"workload": "batched256", "n_boxes": wb.n_boxes, "n_particles": wb.n,
                   "fp32_graph": {"value": wb.n / (msb * 1e-3), "ms_per_step": msb,
                                  "cell_factor": cfgb["cell_factor"], "dense_min": cfgb["dense_min"]}}
        if not args.no_cpu_baseline:
            log("cpu baseline on batched256 (oracle, one box per host thread)")
            batched["cpu_baseline_parallel"], exact = cpu_baseline_batched(wb, lab_b, size_b)
            batched["exact_vs_oracle_on_sample"] = exact
        if not args.no_plain:
            # plain path: FP64 predicate, one launch sequence per box, no graph
            log("timing batched fp64 per box")
            cfgp = choose(torch, tune, pb, wb, "fp64", args)
            fp = fof.FoF("fp64", cell_factor=cfgp["cell_factor"], dense_min=cfgp["dense_min"])
            lp, sp = fp.outputs(wb.n)
            sizes = np.diff(wb.offsets)
            need = max(fof.fof_workspace_bytes(fp.ctx, [0, int(sizes[k])], wb.box[k], wb.lx[k])
                       for k in range(wb.n_boxes))
            fp.ws = torch.empty(need, dtype=torch.uint8, device=dev)
            fof.fof_set_workspace(fp.ctx, fp.ws)
            views = [(pb[wb.offsets[k]:wb.offsets[k + 1]], lp[wb.offsets[k]:wb.offsets[k + 1]],
                      sp[wb.offsets[k]:wb.offsets[k + 1]]) for k in range(wb.n_boxes)]

            def per_box():
                for k, (pk, lk, sk) in enumerate(views):
                    fof.fof_build_cells(fp.ctx, pk, [0, int(sizes[k])], wb.box[k], wb.lx[k])
                    fof.fof_link(fp.ctx)
                    fof.fof_finalize(fp.ctx, lk, sk)

            per_box()
            torch.cuda.synchronize()
            e0 = event(torch, fp.stream)
            for _ in range(nb_steps):
                per_box()
            e1 = event(torch, fp.stream)
            torch.cuda.synchronize()
            msp = e0.elapsed_time(e1) / nb_steps
            same = bool(np.array_equal(lp.cpu().numpy(), lab_b))
            batched["plain_fp64_per_box"] = {"value": wb.n / (msp * 1e-3), "ms_per_step": msp,
                                             "cell_factor": cfgp["cell_factor"], "dense_min": cfgp["dense_min"]}
            batched["speedup_vs_plain"] = msp / msb
            batched["exact_vs_plain"] = same
            fp.close()

    # --- CPU baseline and exactness on the sample ---------------------------
    cpu = None
    sample_exact = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        sub, lx_sub, ref, cpu = cpu_baseline(w)
        lab_s, size_s, ng_s = fof.label(torch.from_numpy(sub).to(dev), lx_sub, cell_factor=cfg["cell_factor"],
                                        dense_min=cfg["dense_min"])
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
        "ms_per_step_median": statistics.median(per_step) if per_step else None,
        "ms_per_step_std": statistics.stdev(per_step) if len(per_step) > 1 else 0.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_particles": n, "box": 1.0, "lx": float(w.lx[0]),
                   "b": w.meta.get("b"), "halo_frac": w.meta.get("halo_frac"), "predicate": "fp32_filter",
                   "cell_factor": cfg["cell_factor"], "dense_min": cfg["dense_min"], "n_cells": st["n_cells"],
                   "parallelism": "single GPU"},
        "n_groups": groups,
        "catalogue": cat,
        "kernels": passes,
        "stats": dict({k: st[k] for k in ("pair_tests", "sparse_pair_tests", "links", "band_hits", "cas_retries",
                                          "queued_links", "dense_items", "find_depth_max")},
                      find_depth_mean=st["find_depth_sum"] / max(1, n), largest_group=int(size32.max(initial=0))),
        "guard_band_hit_fraction": {"per_test": st["band_hits"] / max(1, st["pair_tests"]),
                                    "per_link": st["band_hits"] / max(1, st["links"])},
        "roofline": roofline,
        "plain_fp64": plain,
        "exact_fp32_vs_fp64": exact,
        "batched": batched,
        "domain_decomposed": domain,
        "relink": relink,
        "cpu_baseline": cpu,
        "exact_vs_oracle_on_sample": sample_exact,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
