"""Benchmark of the CompaSO group-finding pass on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload plain256]
                [--no-cpu-baseline] [--cpu-seconds S] [--no-batched] [--no-serving]

A step is one hf_find call (binning, kernel density, L0 FoF, CompaSO L1 and the
output cut) over the whole box, with positions already resident in HBM.  Prints
one JSON line with whole-job throughput in particles/s, the roofline of the
dominant kernel (its average duration measured with HIP events on the stream it
runs on, over the timed steps) and the FP64 CPU oracle timed on a bounded
sample of the same generator.

The same box also times hf_halo_stats (level 2 inside every L1 halo and the
position statistics).  Two more workloads are reported in the same line:
  batched  96 periodic sub-boxes of side log-uniform in 24..160 in one
           hf_find_batch call, against one hf_find call per box;
  serving  a Poisson stream of requests (boxes of 1e4..1e7 particles, log-uniform,
           halo fraction 0.3..0.7) through hf_server, host arrays in and out,
           against the same requests run one at a time on hf_find.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "halo-finding particles/sec at 1 MI355X (batched+served vs plain); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FLOPS_PER_PAIR = 11          # 3 sub + 3 fma (6 flops) + max + add

WORKLOADS = {
    "plain256": "256^3 = 16,777,216 FP32 particles, periodic box 256, half uniform background, "
                "half NFW haloes (c=8, R200) of 35..20000 particles (dn/dN ~ N^-1.9), 20% of "
                "haloes in pairs at 0.5-1.5 R200; b=0.4, l=0.25, Delta_L0=60, Delta_L1=200, N>=35",
    "plain64": "64^3 = 262,144 FP32 particles, periodic box 64, same generator without pairs",
    "large512": "512^3 = 134,217,728 FP32 particles, periodic box 512, 70% in NFW haloes (c=8) of "
                "35..200000 particles, 30% of haloes in pairs and 15% in triples at 0.3-1.2 R200",
}


def _stage_models(n, stats, pairs):
    """Algorithmic work per launch of each stage (bound, work, peak, unit)."""
    ncell = stats["n_cells"]
    return {
        # density: useful pairs x 11 flops, FP32 vector ALU
        "density": ("alu", pairs * FLOPS_PER_PAIR / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"),
        # binning: read xyz 12 + sort key written and read once 16 + three
        # sorted float4 records (positions, cell-local, density operand) 48 +
        # sub-cell index 2 = 78 B per particle, plus the cell offset 4 B per
        # cell of the grid
        "bin": ("hbm", (78.0 * n + 4.0 * ncell) / 1e9, HBM_PEAK_GBS, "GB/s"),
        # FoF: read float4 x2 + density for every particle (36 B), parent r/w 8 B
        "fof": ("hbm", 44.0 * n / 1e9, HBM_PEAK_GBS, "GB/s"),
    }


STAGE_KERNELS = {
    "density": ("k_density_dense", "k_density_sparse"),
    "bin": ("k_bin_key", "k_radix_count", "k_radix_scatter", "k_bin_place", "k_cell_offsets",
            "k_bin_flags", "k_bin_lists", "k_sub_table"),
    "fof": ("k_fof_phase_a", "k_fof_dense", "k_fof_sparse_flags", "k_fof_sparse_list", "k_fof_sparse",
            "k_fof_roots", "k_fof_keys"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def source_hash() -> str:
    """Hash of the HIP sources and headers: measured traffic is valid only for them."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2110_11408_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "hf.h"), "rb").read())
    return h.hexdigest()[:16]


def pmc_summary(fetch_csv: str, write_csv: str, copy_mib: int) -> dict:
    """Per-call HBM bytes of each stage from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch) of `bench.py --steps 1 --warmup 0 --copy-probe MIB`,
    each scaled so that the probe's plain copy reads and writes copy_mib MiB."""
    import csv

    def load(path):
        rows = list(csv.DictReader(open(path)))
        probe = [float(r["Counter_Value"]) for r in rows
                 if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) > 4096]
        scale = (copy_mib * 1024.0) / max(probe) if probe else 1.0
        per = {}
        for r in rows:
            m = re.search(r"(k_[A-Za-z0-9_]+)(?:<[^>]*>)?\(", r["Kernel_Name"])
            name = m.group(1) if m else r["Kernel_Name"]
            per.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0 * scale)
        return per, scale

    fetch, fscale = load(fetch_csv)
    write, wscale = load(write_csv)
    out = {"source_hash": source_hash(), "fetch_scale": fscale, "write_scale": wscale,
           "copy_probe_mib": copy_mib, "stages": {}}
    for stage, kernels in STAGE_KERNELS.items():
        # per call of the stage: the first kernel runs once per call (the
        # binning also runs for the pair count, so it is seen twice)
        calls = max(len(fetch.get(kernels[0], [])), 1)
        rb = sum(sum(fetch.get(k, [])) for k in kernels) / calls
        wb = sum(sum(write.get(k, [])) for k in kernels) / calls
        out["stages"][stage] = {"read_bytes": rb, "write_bytes": wb, "bytes": rb + wb,
                                "calls_seen": calls, "kernels": list(kernels)}
    return out


def measured_traffic(stage: str):
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash() or stage not in t.get("stages", {}):
        return None
    return t["stages"][stage]["bytes"]


def cpu_baseline(target_s: float):
    import numpy as np  # noqa: F401
    import oracle
    from paper_2110_11408_amd import synth
    oracle.build(force=False)
    threads = oracle.num_threads()
    done = 0
    t0 = time.perf_counter()
    k = 0
    while True:
        pos, L, _ = synth.named_box("plain64", k)
        t = time.perf_counter()
        oracle.find(pos, box=L)
        done += len(pos)
        k += 1
        if time.perf_counter() - t0 > target_s or k >= 64:
            break
    wall = time.perf_counter() - t0
    return {"value": done / wall, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"full FP64 oracle pass (density, L0 FoF, literal CompaSO, cut) on {k} "
                      f"64^3 boxes of the same generator ({done} particles, {wall:.1f} s); "
                      "the 256^3 box itself takes minutes on the host"}


def _batched(ctx, np, torch, _lib, synth, reps=3, lanes=8):
    """Batched workload: 96 boxes in one hf_find_batch call vs one hf_find per box."""
    boxes = synth.batch_boxes()
    pos = torch.from_numpy(np.concatenate([b[0] for b in boxes])).cuda()
    sizes = np.array([len(b[0]) for b in boxes], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    params = [_lib.default_params(box=b[1]) for b in boxes]
    caps = np.maximum(sizes // 64, 64)
    ctx.find_batch(pos, offs, params, halos_caps=caps, n_lanes=lanes, want_l0=False)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.find_batch(pos, offs, params, halos_caps=caps, n_lanes=lanes, want_l0=False)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    views = [pos[offs[b]:offs[b + 1]] for b in range(len(boxes))]
    for b in range(len(boxes)):
        ctx.find(views[b], params[b], halos_cap=int(caps[b]), want_l0=False)
    torch.cuda.synchronize()
    tp = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for b in range(len(boxes)):
            ctx.find(views[b], params[b], halos_cap=int(caps[b]), want_l0=False)
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
    total = int(offs[-1])
    tb, tpl = float(np.median(t)), float(np.median(tp))
    return {"workload": "96 periodic boxes, side log-uniform in 24..160 (N = side^3, "
                        f"{sizes.min()}..{sizes.max()}), half NFW haloes 35..20000",
            "n_boxes": len(boxes), "n_particles": total, "lanes": lanes,
            "value": total / tb, "unit": "particles/s", "ms": tb * 1e3,
            "plain_value": total / tpl, "plain_ms": tpl * 1e3, "speedup": tpl / tb,
            "reps": reps}


def _halo_stats(ctx, pos_d, p, out, np, torch, reps=3):
    """hf_halo_stats on the benchmark box: level 2 inside every L1 halo and the
    Table 1 position statistics (fresh binning included)."""
    nh = out["n_halos"]
    ctx.halo_stats(pos_d, out["density"], out["halo_id"], p, nh)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        res = ctx.halo_stats(pos_d, out["density"], out["halo_id"], p, nh)
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    st = ctx.stats()
    ms = float(np.median(t)) * 1e3
    return {"ms": ms, "value": len(pos_d) / (ms / 1e3), "unit": "particles/s", "n_halos": nh,
            "n_l2": int(np.sum(res["n_l2"])), "reps": reps,
            "stages_ms": {k[3:]: st[k] for k in ("ms_bin", "ms_segment", "ms_candidates", "ms_accept",
                                                  "ms_assign", "ms_output", "ms_total")}}


def _fifo_latency(arrivals, service):
    """Latencies of a one-at-a-time FIFO server with the given service times."""
    done, lat = 0.0, []
    for a, s in zip(arrivals, service):
        start = max(a, done)
        done = start + s
        lat.append(done - a)
    return lat


def _serving(ctx, np, torch, _lib, synth, count=32, slots=4, budget_gb=64):
    """Serving workload: Poisson arrivals at a rate that keeps the plain
    one-at-a-time path fully busy; latency from submission to host results."""
    from paper_2110_11408_amd.api import Server
    reqs = synth.request_stream(count, rate_hz=1.0)
    boxes = []
    for r in reqs:
        pos, L, _ = synth.make_box(synth.BoxRecipe(n=r["n"], side=r["side"], halo_frac=r["halo_frac"]),
                                   r["seed"])
        boxes.append((Server.pinned_positions(pos), L))
    sizes = np.array([len(b[0]) for b in boxes], np.int64)
    params = [_lib.default_params(box=b[1]) for b in boxes]
    total = int(sizes.sum())
    # plain path: host positions -> device, hf_find, results -> host, one at a time
    def plain_one(b):
        pos_h, _ = boxes[b]
        d = pos_h.to("cuda", non_blocking=True)
        out = ctx.find(d, params[b], want_density=False, want_l0=False)
        out["halo_id"].cpu()
        out["halos"].cpu()
    plain_one(int(np.argmax(sizes)))
    torch.cuda.synchronize()
    service = []
    for b in range(count):
        t0 = time.perf_counter()
        plain_one(b)
        service.append(time.perf_counter() - t0)
    mean_s = float(np.mean(service))
    rate = 1.0 / mean_s            # the plain path's capacity in requests/s
    gaps = np.diff(np.r_[0.0, [r["t"] for r in reqs]])  # exponential, mean 1 s
    arrivals = np.cumsum(gaps / rate)
    plain_lat = _fifo_latency(arrivals, service)
    srv = Server(0, slots=slots, budget_bytes=int(budget_gb) << 30)
    try:
        # warm every slot once
        for t in [srv.submit(boxes[b][0], params[b]) for b in np.argsort(sizes)[-slots:]]:
            srv.wait(t)
        # saturated: everything queued at once
        t0 = srv.now()
        tickets = [srv.submit(boxes[b][0], params[b]) for b in range(count)]
        res = [srv.wait(t) for t in tickets]
        sat = total / (max(r["t_done"] for r in res) - t0)
        # open loop at the Poisson arrival times
        base = time.perf_counter()
        tickets = []
        for b in range(count):
            while time.perf_counter() - base < arrivals[b]:
                time.sleep(min(0.0005, max(0.0, arrivals[b] - (time.perf_counter() - base))))
            tickets.append(srv.submit(boxes[b][0], params[b]))
        res = [srv.wait(t) for t in tickets]
        lat = [r["t_done"] - r["t_submit"] for r in res]
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        held = srv.held_bytes()
    finally:
        srv.close()
    ms = lambda x: float(x) * 1e3  # noqa: E731
    return {"workload": f"{count} requests, N log-uniform in 1e4..1e7 ({sizes.min()}..{sizes.max()}), "
                        "halo fraction 0.3..0.7, side N^(1/3); host arrays in and out",
            "requests": count, "n_particles": total, "slots": slots, "budget_gb": budget_gb,
            "value": sat, "unit": "particles/s", "plain_value": total / float(np.sum(service)),
            "rate_hz": rate, "open_loop_value": total / span,
            "p50_ms": ms(np.percentile(lat, 50)), "p99_ms": ms(np.percentile(lat, 99)),
            "plain_p50_ms": ms(np.percentile(plain_lat, 50)),
            "plain_p99_ms": ms(np.percentile(plain_lat, 99)),
            "plain_latency_model": "FIFO one at a time with the measured plain service times "
                                   "at the same arrival times",
            "held_gb": held / 2 ** 30}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (a traffic "
                         "reference for hardware counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter files "
                         "and exit (no GPU needed)")
    args = ap.parse_args()
    if args.pmc_summary:
        t = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.copy_probe or 1024)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library runs "
              "each box on a single device", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_11408_amd import _lib, synth
    from paper_2110_11408_amd.api import Context

    dev = torch.device("cuda:0")
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pos, L, _ = synth.named_box(args.workload)
    n = len(pos)
    pos_d = torch.from_numpy(pos).to(dev)
    p = _lib.default_params(box=L)
    ctx = Context(0)
    pairs = ctx.count_pairs(pos_d, p)
    cap = max(1024, n // 64)
    for _ in range(args.warmup):
        ctx.find(pos_d, p, halos_cap=cap)
    torch.cuda.synchronize()
    keys = ("ms_bin", "ms_density", "ms_fof", "ms_segment", "ms_candidates", "ms_accept",
            "ms_assign", "ms_output", "ms_total")
    acc = {k: 0.0 for k in keys}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.find(pos_d, p, halos_cap=cap)
        st = ctx.stats()
        for k in keys:
            acc[k] += st[k]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    stages = {k[3:]: acc[k] / args.steps for k in keys}
    models = _stage_models(n, st, pairs)
    lines = {}
    for k, (bound, work, peak, unit) in models.items():
        achieved = work / (stages[k] / 1e3)
        lines[k] = {"bound": bound, "kernel": k, "ms": stages[k], "achieved": achieved, "peak": peak,
                    "unit": unit, "frac": achieved / peak, "traffic": measured_traffic(k)}
    dom = max(lines, key=lambda k: stages[k])
    roof = lines[dom]
    res = {
        "metric": METRIC, "value": n / (ms_step / 1e3), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "n_particles": n, "box": L, "path": "plain (hf_find, one box per call)"},
        "roofline": roof,
        "stage_rooflines": lines,
        "stages_ms": stages,
        "counts": {"pairs_within_b": pairs, "n_cells": st["n_cells"], "n_members": st["n_members"],
                   "n_groups": st["n_groups"], "n_candidates": st["n_candidates"],
                   "n_found": st["n_found"], "n_halos": out["n_halos"],
                   "n_dense_cells": st["n_dense_cells"], "n_dense_chunks": st["n_dense_chunks"],
                   "n_sparse": st["n_sparse"], "n_hard": st["n_hard"]},
    }
    res["halo_stats"] = _halo_stats(ctx, pos_d, p, out, np, torch)
    if not args.no_batched:
        res["batched"] = _batched(ctx, np, torch, _lib, synth)
    if not args.no_serving:
        res["serving"] = _serving(ctx, np, torch, _lib, synth)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
