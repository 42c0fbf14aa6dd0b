"""Benchmark of the CompaSO group-finding pass on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched96]
                [--no-cpu-baseline] [--cpu-seconds S] [--no-plain256] [--no-serving]
                [--large] [--only-steps] [--lanes L] [--tune-groups G] [--tune-table F]

Headline workload (``batched96``): 96 independent periodic sub-boxes of side
log-uniform in 24..160 (about 60M particles), found in one ``hf_find_batch``
call per step, positions already resident in HBM.  Before the warmup (untimed),
``hf_tune_batch`` picks the fused group count for the batch, which the timed
calls take.  Whole-job particles/s over the K timed steps is ``value``;
``plain_value`` is the same boxes found one ``hf_find`` call at a time.  The
line also carries:
  roofline      the dominant stage over the batch's boxes, timed with HIP events
                on the stream each box runs on (boxes one at a time, so that no
                other box shares the device during a stage);
  serving       Poisson streams of requests (boxes of 1e4..1e7 particles) at
                three rates through ``hf_server``, host arrays in and out,
                against the same requests run one at a time on ``hf_find`` at
                the same arrival times: p50/p99 latency and particles/s of both;
  plain256      the 256^3 box (16.8M particles) as a single ``hf_find`` call,
                with its stage rooflines and ``hf_halo_stats``;
  plain64       the 64^3 box (262k particles) as a single ``hf_find`` call;
  large512      (``--large``) the 512^3 box (134M particles);
  cpu_baseline  the FP64 oracle on a bounded sample of the headline workload's
                boxes, per stage, on all host threads and on one.
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
    "batched96": "96 independent periodic boxes in one call, side log-uniform in 24..160 (N = side^3, "
                 "14k..3.5M particles, 59.7M in all), each half uniform background and half NFW haloes "
                 "(c=8, R200) of 35..20000 particles (dn/dN ~ N^-1.9); b=0.4, l=0.25, Delta_L0=60, "
                 "Delta_L1=200, N>=35",
    "plain256": "256^3 = 16,777,216 FP32 particles, periodic box 256, half uniform background, "
                "half NFW haloes (c=8, R200) of 35..20000 particles (dn/dN ~ N^-1.9), 20% of "
                "haloes in pairs at 0.5-1.5 R200; b=0.4, l=0.25, Delta_L0=60, Delta_L1=200, N>=35",
    "plain64": "64^3 = 262,144 FP32 particles, periodic box 64, same generator without pairs",
    "large512": "512^3 = 134,217,728 FP32 particles, periodic box 512, 70% in NFW haloes (c=8) of "
                "35..200000 particles, 30% of haloes in pairs and 15% in triples at 0.3-1.2 R200",
}

STAGE_KEYS = ("ms_bin", "ms_density", "ms_fof", "ms_segment", "ms_candidates", "ms_accept",
              "ms_assign", "ms_output", "ms_total")
STAGE_KERNELS = {
    "density": ("k_density_dense", "k_density_sparse"),
    "bin": ("k_bin_key", "k_radix_count", "k_radix_scatter", "k_bin_place", "k_cell_offsets",
            "k_bin_flags", "k_bin_lists", "k_sub_table"),
    "fof": ("k_fof_phase_a", "k_fof_dense", "k_fof_sparse_flags", "k_fof_sparse_list", "k_fof_sparse",
            "k_fof_roots", "k_fof_keys"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ rooflines

def stage_work(n, ncell, pairs):
    """Algorithmic work of each stage for n particles on a grid of ncell cells
    with `pairs` ordered pairs within b: (bound, work, peak, unit)."""
    return {
        # density: useful pairs x 11 flops on the FP32 ALU
        "density": ("alu", pairs * FLOPS_PER_PAIR / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"),
        # binning: read xyz 12 + sort key written and read once 16 + three
        # sorted float4 records (positions, cell-local, density operand) 48 +
        # sub-cell index 2 = 78 B per particle, plus the cell offset 4 B per
        # cell of the grid
        "bin": ("hbm", (78.0 * n + 4.0 * ncell) / 1e9, HBM_PEAK_GBS, "GB/s"),
        # FoF: read float4 x2 + density for every particle (36 B), parent r/w 8 B
        "fof": ("hbm", 44.0 * n / 1e9, HBM_PEAK_GBS, "GB/s"),
    }


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


def pmc_summary(fetch_csv: str, write_csv: str, copy_mib: int, workload: str, steps: int) -> dict:
    """Per-step HBM bytes of each stage from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch) of `bench.py --workload W --steps S --warmup 0
    --only-steps --copy-probe MIB`, each scaled so that the probe's plain copy
    reads and writes copy_mib MiB.  Every dispatch of a stage's kernels in that
    run belongs to one of the S steps."""
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
           "copy_probe_mib": copy_mib, "steps": steps, "stages": {}}
    for stage, kernels in STAGE_KERNELS.items():
        rb = sum(sum(fetch.get(k, [])) for k in kernels) / steps
        wb = sum(sum(write.get(k, [])) for k in kernels) / steps
        out["stages"][stage] = {"read_bytes": rb, "write_bytes": wb, "bytes": rb + wb,
                                "kernels": list(kernels)}
    return out


def measured_traffic(workload: str, stage: str):
    """HBM bytes per step of a stage, from profiles/traffic.json, when they were
    measured on this workload with the current sources; else None."""
    try:
        t = json.load(open(TRAFFIC_FILE)).get(workload)
    except (OSError, ValueError):
        return None
    if not t or t.get("source_hash") != source_hash() or stage not in t.get("stages", {}):
        return None
    return t["stages"][stage]["bytes"]


def rooflines(workload, n, ncell, pairs, stages_ms):
    lines = {}
    for k, (bound, work, peak, unit) in stage_work(n, ncell, pairs).items():
        achieved = work / (stages_ms[k] / 1e3)
        lines[k] = {"bound": bound, "kernel": k, "ms": stages_ms[k], "achieved": achieved, "peak": peak,
                    "unit": unit, "frac": achieved / peak, "traffic": measured_traffic(workload, k)}
    dom = max(lines, key=lambda k: stages_ms[k])
    return lines[dom], lines


# ------------------------------------------------------------------ CPU baseline

def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(boxes, target_s: float):
    """The FP64 oracle as it stands (density, L0 FoF, literal CompaSO and the
    cut), per stage, on a seeded sample of the workload's boxes: all host threads
    for about target_s seconds, then one thread for about a quarter of that."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    order = np.random.default_rng(7).permutation(len(boxes))

    def run(budget_s):
        t0 = time.perf_counter()
        st = {"density": 0.0, "fof": 0.0, "compaso": 0.0}
        done = used = 0
        for b in order:
            pos, L = boxes[b][0], boxes[b][1]
            t = time.perf_counter()
            d = oracle.density(pos, box=L)
            t1 = time.perf_counter()
            l0, _ = oracle.fof(pos, d, box=L)
            t2 = time.perf_counter()
            oracle.compaso(pos, d, l0, box=L)
            t3 = time.perf_counter()
            st["density"] += t1 - t
            st["fof"] += t2 - t1
            st["compaso"] += t3 - t2
            done += len(pos)
            used += 1
            if time.perf_counter() - t0 > budget_s:
                break
        wall = time.perf_counter() - t0
        return done, used, wall, st

    threads = oracle.num_threads()
    done, used, wall, st = run(target_s)
    oracle.set_threads(1)
    try:
        done1, used1, wall1, st1 = run(target_s / 4)
    finally:
        oracle.set_threads(threads)
    return {"value": done / wall, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"full FP64 oracle pass (density, L0 FoF, literal CompaSO, cut) on {used} of the "
                      f"workload's boxes in a seeded order ({done} particles, {wall:.1f} s)",
            "stages_s": st, "value_1thread": done1 / wall1,
            "sample_1thread": f"{used1} boxes ({done1} particles, {wall1:.1f} s) on one thread",
            "stages_s_1thread": st1, "nproc": os.cpu_count(), "cpu_model": cpu_model()}


# ------------------------------------------------------------------ workloads

def _boxes_on_device(boxes, torch, np):
    pos = torch.from_numpy(np.concatenate([b[0] for b in boxes])).cuda()
    sizes = np.array([len(b[0]) for b in boxes], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return pos, sizes, offs


def batched(ctx, boxes, args, np, torch, _lib):
    """The headline: K timed hf_find_batch steps over the boxes; the same boxes
    one hf_find call at a time; the stage rooflines over the boxes."""
    pos, sizes, offs = _boxes_on_device(boxes, torch, np)
    params = [_lib.default_params(box=b[1]) for b in boxes]
    caps = np.maximum(sizes // 64, 64)
    lanes = args.lanes
    tuned = None
    if lanes <= 0 and args.tune_groups > 0:
        # untimed: hf_tune_batch picks the fused group count for this batch shape,
        # which the timed calls (n_lanes = 0) then take from the context
        g, ms, _ = ctx.tune_batch(pos, offs, params, max_groups=args.tune_groups, reps=1,
                                  table_path=args.tune_table or None)
        tuned = {"groups": g, "ms": ms, "max_groups": args.tune_groups}
    for _ in range(args.warmup):
        ctx.find_batch(pos, offs, params, halos_caps=caps, n_lanes=lanes, want_l0=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.find_batch(pos, offs, params, halos_caps=caps, n_lanes=lanes, want_l0=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total = int(offs[-1])
    res = {"value": total * args.steps / wall, "ms_per_step": wall * 1e3 / args.steps,
           "n_halos": int(np.sum(out["n_halos"])),
           "groups": ctx.batch_groups(len(boxes), total, n_lanes=lanes), "tuning": tuned}
    if args.only_steps:
        return res
    # one hf_find per box, in the same order, as the plain comparison
    views = [pos[offs[b]:offs[b + 1]] for b in range(len(boxes))]
    for b in range(len(boxes)):
        ctx.find(views[b], params[b], halos_cap=int(caps[b]), want_l0=False)
    torch.cuda.synchronize()
    tp = []
    for _ in range(3):
        t0 = time.perf_counter()
        for b in range(len(boxes)):
            ctx.find(views[b], params[b], halos_cap=int(caps[b]), want_l0=False)
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
    tpl = float(np.median(tp))
    res.update({"plain_value": total / tpl, "plain_ms": tpl * 1e3,
                "speedup_vs_plain": tpl / (wall / args.steps)})
    # stage times of every box with no other box on the device (one lane), and
    # the work of every box
    ctx.find_batch(pos, offs, params, halos_caps=caps, n_lanes=1, want_l0=False)
    torch.cuda.synchronize()
    st = ctx.stats()
    pairs = sum(ctx.count_pairs(views[b], params[b]) for b in range(len(boxes)))
    stages = {k[3:]: st[k] for k in STAGE_KEYS}
    roof, lines = rooflines("batched96", total, st["n_cells"], pairs, stages)
    res.update({"roofline": roof, "stage_rooflines": lines, "stages_ms_one_lane": stages,
                "counts": {"pairs_within_b": pairs, "n_cells": st["n_cells"],
                           "n_members": st["n_members"], "n_groups": st["n_groups"],
                           "n_candidates": st["n_candidates"], "n_halos": st["n_halos"]}})
    return res


def single_box(ctx, name, steps, warmup, np, torch, _lib, synth, halo_stats=False, count=True):
    """One box found by one hf_find call per step, with its stage rooflines
    (count=False: no pair count and no rooflines, so that a counter run sees
    only the steps' dispatches)."""
    pos, L, _ = synth.named_box(name)
    n = len(pos)
    pos_d = torch.from_numpy(pos).cuda()
    p = _lib.default_params(box=L)
    pairs = ctx.count_pairs(pos_d, p) if count else 0
    cap = max(1024, n // 64)
    for _ in range(warmup):
        ctx.find(pos_d, p, halos_cap=cap)
    torch.cuda.synchronize()
    acc = {k: 0.0 for k in STAGE_KEYS}
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.find(pos_d, p, halos_cap=cap)
        st = ctx.stats()
        for k in STAGE_KEYS:
            acc[k] += st[k]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = {k[3:]: acc[k] / steps for k in STAGE_KEYS}
    roof, lines = rooflines(name, n, st["n_cells"], pairs, stages) if count else (None, None)
    res = {"workload": name, "description": WORKLOADS[name], "n_particles": n,
           "value": n * steps / wall, "unit": "particles/s", "ms_per_step": wall * 1e3 / steps,
           "steps": steps, "roofline": roof, "stage_rooflines": lines, "stages_ms": stages,
           "counts": {"pairs_within_b": pairs, "n_cells": st["n_cells"], "n_members": st["n_members"],
                      "n_groups": st["n_groups"], "n_candidates": st["n_candidates"],
                      "n_found": st["n_found"], "n_halos": out["n_halos"],
                      "n_dense_cells": st["n_dense_cells"], "n_dense_chunks": st["n_dense_chunks"],
                      "n_sparse": st["n_sparse"], "n_hard": st["n_hard"]}}
    if halo_stats:
        nh = out["n_halos"]
        ctx.halo_stats(pos_d, out["density"], out["halo_id"], p, nh)
        torch.cuda.synchronize()
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            r = ctx.halo_stats(pos_d, out["density"], out["halo_id"], p, nh)
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        ms = float(np.median(t)) * 1e3
        res["halo_stats"] = {"ms": ms, "value": n / (ms / 1e3), "unit": "particles/s", "n_halos": nh,
                             "n_l2": int(np.sum(r["n_l2"]))}
        res["variants"] = variants(ctx, pos_d, p, cap, out, np, torch)
    del pos_d
    torch.cuda.empty_cache()
    return res


def variants(ctx, pos_d, p, cap, ref, np, torch):
    """The same box with the threshold radius searched by radial bins
    (Sec. 2.3.4) and with the members collected into group order (Sec. 2.3.5,
    hf_find_grouped): per-call ms (median of 3) and the acceptance stage ms,
    with a check that the labels equal the reference call's."""
    def timed(call):
        call()
        torch.cuda.synchronize()
        t, acc = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            o = call()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
            acc.append(ctx.stats()["ms_accept"])
        return o, float(np.median(t)) * 1e3, float(np.median(acc))
    base, ms0, acc0 = timed(lambda: ctx.find(pos_d, p, halos_cap=cap))
    ctx.set_radius_search("bins")
    try:
        rb, ms1, acc1 = timed(lambda: ctx.find(pos_d, p, halos_cap=cap))
    finally:
        ctx.set_radius_search("histogram")
    gr, ms2, _ = timed(lambda: ctx.find_grouped(pos_d, p, halos_cap=cap))
    same = bool(torch.equal(rb["halo_id"], ref["halo_id"]) and torch.equal(gr["halo_id"], ref["halo_id"]))
    return {"find_ms": ms0, "accept_ms": acc0, "radius_bins_ms": ms1, "radius_bins_accept_ms": acc1,
            "grouped_ms": ms2, "grouped_extra_ms": ms2 - ms0, "labels_identical": same}


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x) * 1e3, q))


def serving(ctx, np, torch, _lib, synth, count=200, pool=24, slots=4, budget_gb=64,
            loads=(0.5, 0.9, 1.3)):
    """Poisson request streams at several rates (fractions of the plain path's
    capacity).  Requests are drawn (seeded) from a pool of distinct boxes of
    1e4..1e7 particles (log-uniform, halo fraction 0.3..0.7).  The served path
    is hf_server; the plain path runs the same requests one at a time on hf_find
    (host positions in, halo ids and table out) at the same arrival times.
    Latency is from arrival to results in host memory, both measured."""
    from paper_2110_11408_amd.api import Server
    reqs = synth.request_stream(pool, rate_hz=1.0)
    boxes = []
    for r in reqs:
        pos, L, _ = synth.make_box(synth.BoxRecipe(n=r["n"], side=r["side"], halo_frac=r["halo_frac"]),
                                   r["seed"])
        boxes.append((Server.pinned_positions(pos), L))
    sizes = np.array([len(b[0]) for b in boxes], np.int64)
    params = [_lib.default_params(box=b[1]) for b in boxes]
    halo_host = {b: torch.empty(int(sizes[b]), dtype=torch.int32).pin_memory() for b in range(pool)}

    def plain_one(b):
        pos_h, _ = boxes[b]
        d = pos_h.to("cuda", non_blocking=True)
        out = ctx.find(d, params[b], want_density=False, want_l0=False)
        halo_host[b].copy_(out["halo_id"], non_blocking=True)
        out["halos"].cpu()

    for b in range(pool):
        plain_one(b)
    torch.cuda.synchronize()
    service = []
    for b in range(pool):
        t0 = time.perf_counter()
        plain_one(b)
        service.append(time.perf_counter() - t0)
    mean_n = float(sizes.mean())
    capacity = 1.0 / float(np.mean(service))   # requests/s of the plain path on the pool
    rng = np.random.default_rng(77)
    which = rng.integers(0, pool, count)
    gaps = rng.exponential(1.0, count)
    srv = Server(0, slots=slots, budget_bytes=int(budget_gb) << 30)
    out = {"workload": f"{count} requests per rate drawn from {pool} distinct boxes of "
                       f"{sizes.min()}..{sizes.max()} particles (N log-uniform in 1e4..1e7, halo fraction "
                       "0.3..0.7, side N^(1/3)); host arrays in and out",
           "requests_per_rate": count, "slots": slots, "budget_gb": budget_gb,
           "plain_capacity_hz": capacity, "rates": []}
    try:
        for b in np.argsort(sizes)[-slots:]:
            srv.wait(srv.submit(boxes[b][0], params[b]))
        for load in loads:
            rate = load * capacity
            arrivals = np.cumsum(gaps / rate)
            total = int(sizes[which].sum())
            # served
            base = time.perf_counter()
            tickets = []
            for k in range(count):
                while time.perf_counter() - base < arrivals[k]:
                    time.sleep(min(0.0005, max(0.0, arrivals[k] - (time.perf_counter() - base))))
                tickets.append(srv.submit(boxes[which[k]][0], params[which[k]]))
            res = [srv.wait(t) for t in tickets]
            lat = [r["t_done"] - r["t_submit"] for r in res]
            span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
            # plain, one at a time at the same arrival times
            base = time.perf_counter()
            plat = []
            last = 0.0
            for k in range(count):
                now = time.perf_counter() - base
                if now < arrivals[k]:
                    time.sleep(arrivals[k] - now)
                plain_one(int(which[k]))
                torch.cuda.synchronize()
                last = time.perf_counter() - base
                plat.append(last - arrivals[k])
            out["rates"].append({
                "load": load, "rate_hz": rate, "n_particles": total,
                "served_value": total / span, "served_p50_ms": _pct(lat, 50), "served_p99_ms": _pct(lat, 99),
                "plain_value": total / last, "plain_p50_ms": _pct(plat, 50), "plain_p99_ms": _pct(plat, 99)})
            _say(f"[bench] serving load {load}: served p50/p99 {_pct(lat, 50):.2f}/{_pct(lat, 99):.2f} ms, "
                 f"plain {_pct(plat, 50):.2f}/{_pct(plat, 99):.2f} ms")
        out["held_gb"] = srv.held_bytes() / 2 ** 30
        # saturated: every request of the stream queued at once
        t0 = srv.now()
        tickets = [srv.submit(boxes[which[k]][0], params[which[k]]) for k in range(count)]
        res = [srv.wait(t) for t in tickets]
        out["saturated_value"] = int(sizes[which].sum()) / (max(r["t_done"] for r in res) - t0)
    finally:
        srv.close()
    out["mean_request_particles"] = mean_n
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched96", choices=sorted(WORKLOADS))
    ap.add_argument("--lanes", type=int, default=0, help="pipelines of hf_find_batch (0: the library's)")
    ap.add_argument("--tune-groups", type=int, default=4,
                    help="hf_tune_batch over 1..G fused groups before timing (0: no tuning)")
    ap.add_argument("--tune-table", default="", help="tuning table file hf_tune_batch rewrites")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-plain256", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--large", action="store_true", help="also time the 512^3 box")
    ap.add_argument("--only-steps", action="store_true",
                    help="run the warmup and timed steps of the workload and nothing else (for counters)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (a traffic "
                         "reference for hardware counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="record the per-step stage traffic of --workload in profiles/traffic.json from "
                         "two rocprofv3 --pmc counter files of an --only-steps run and exit (no GPU needed)")
    args = ap.parse_args()
    if args.pmc_summary:
        try:
            allt = json.load(open(TRAFFIC_FILE))
        except (OSError, ValueError):
            allt = {}
        allt = {k: v for k, v in allt.items() if k in WORKLOADS}
        allt[args.workload] = pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.copy_probe or 1024,
                                          args.workload, args.steps + args.warmup)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(allt, f, indent=1)
        print(json.dumps(allt[args.workload]))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: every box and request "
              "runs on a single device (the multi-GPU sharding is a design, not a build)", file=sys.stderr)
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
    ctx = Context(0)
    res = {"metric": METRIC, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic"}
    if args.workload == "batched96":
        _say("[bench] generating the 96 boxes")
        boxes = synth.batch_boxes()
        _say("[bench] batched steps")
        b = batched(ctx, boxes, args, np, torch, _lib)
        res.update({"value": b.pop("value"), "ms_per_step": b.pop("ms_per_step"),
                    "config": {"workload": "batched96", "description": WORKLOADS["batched96"],
                               "n_boxes": len(boxes), "n_particles": int(sum(len(x[0]) for x in boxes)),
                               "path": "hf_find_batch (all boxes in one call)"}})
        if "roofline" in b:
            res["roofline"] = b.pop("roofline")
        res["batched"] = b
    else:
        s = single_box(ctx, args.workload, args.steps, args.warmup, np, torch, _lib, synth,
                       halo_stats=not args.only_steps, count=not args.only_steps)
        res.update({"value": s.pop("value"), "ms_per_step": s.pop("ms_per_step"), "roofline": s.pop("roofline"),
                    "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                               "n_particles": s["n_particles"], "path": "hf_find (one box per call)"}})
        res["plain"] = s
        boxes = None
    if args.only_steps:
        print(json.dumps(res), flush=True)
        return
    if args.workload == "batched96" and not args.no_plain256:
        _say("[bench] plain256")
        res["plain256"] = single_box(ctx, "plain256", 5, 2, np, torch, _lib, synth, halo_stats=True)
        _say("[bench] plain64")
        res["plain64"] = single_box(ctx, "plain64", 20, 3, np, torch, _lib, synth)
    if args.large:
        _say("[bench] large512")
        res["large512"] = single_box(ctx, "large512", 3, 1, np, torch, _lib, synth)
    if not args.no_serving:
        _say("[bench] serving")
        res["serving"] = serving(ctx, np, torch, _lib, synth)
    if not args.no_cpu_baseline:
        _say("[bench] cpu baseline")
        if boxes is None:
            pos, L, _ = synth.named_box("plain64")
            boxes = [(pos, L)]
        res["cpu_baseline"] = cpu_baseline(boxes, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
