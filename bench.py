#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 Block-Parallel IDA* path.

One step = one full ``bpida_solve_device`` call (``bpida_solve_mixed_device``
for the mixed-width workload) over the workload's batch
(ingest, root split, every f-limit of every instance with its search launch
and reduction, outputs), with the start states already resident in HBM.

Prints one JSON line: nodes expanded per second over the timed steps (the
node total is the sum over instances and f-limits of the expanded-node
counts, final limit run to completion), instances per second, the search
kernel's position against the VALU integer-issue roofline, and the CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "nodes expanded/sec and instances/sec (15-puzzle, Manhattan), batched vs plain"

# MI355X integer VALU issue: 256 CUs x 4 SIMDs, each issuing up to two wave64
# VALU instructions per 4 clocks (dual issue of the simple two-operand class),
# x 64 lanes x 2.4 GHz = 128 32-bit lane-operations per CU per clock (the
# same 128 lanes per CU-clock as the fp32 vector peak, 157.3 TFLOP/s with an
# FMA counted as two flops).  PEAK_INT_SINGLE_GOPS is the rate when nothing
# pairs (one wave64 instruction per CU per clock).
PEAK_INT_GOPS = 256 * 128 * 2.4
PEAK_INT_SINGLE_GOPS = 256 * 64 * 2.4
# Algorithmic integer operations per expanded node (derivation in the design
# notes): per generated move 15 (applicability 2, successor 7, f 4,
# compare 1, push-or-min 1) x 4 moves, plus 4 per node (pop, goal test,
# count, parent bookkeeping).
OPS_PER_NODE = 64

WORKLOADS = {
    "c2_md30_38": ("100 15-puzzle states from seeded 300-move non-backtracking walks, Manhattan "
                   "30..38, all-optimal-solutions final limit", 4),
    "c1_walk40": ("64 15-puzzle states from seeded 40-move non-backtracking walks", 4),
    "c3_uneven": ("4096 15-puzzle states from seeded non-backtracking walks of length U{20..300}, "
                  "Manhattan <= 38, all-optimal-solutions final limit", 4),
    "c4_mixed": ("2048 3x3 (walks U{20..300}) + 2048 4x4 (walks U{20..300}, Manhattan <= 38) + "
                 "256 5x5 (60-move walks) states in one launch, all-optimal-solutions final limit", 0),
}
# the mixed workload's stored oracle results, one file per width (launch order)
MIXED_PARTS = (("c4_mixed_w3", 3), ("c4_mixed_w4", 4), ("c4_mixed_w5", 5))
MODES = {"plain": 0, "batched": 1}


# The device sources the search kernels are built from (host-side driver
# code does not change what a kernel launch moves or executes).
DEVICE_SOURCES = ("bpida_batch.hip", "bpida_board.h", "bpida_internal.h", "bpida_kernels.hip",
                  "bpida_lb.hip", "bpida_round.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_02843_amd", "csrc")
    for fn in DEVICE_SOURCES:
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


def make_parts(name):
    """[(golden file name, states [n, w*w], width)] in launch order."""
    from paper_1705_02843_amd import instances
    if name == "c4_mixed":
        d = instances.c4_mixed()
        return [(g, d[w][0], w) for g, w in MIXED_PARTS]
    return [(name, getattr(instances, name)()[0], WORKLOADS[name][1])]


def golden_total(parts):
    tot = 0
    for g, _, _ in parts:
        path = os.path.join(ROOT, "tests", "golden", g + ".json")
        if not os.path.exists(path):
            return None
        with open(path) as f:
            tot += int(json.load(f)["total_nodes"])
    return tot


def progress(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU as lscpu names it (model name, family/model/stepping)."""
    import subprocess
    fields = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if not fields.get("Model name"):
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        fields["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    name = fields.get("Model name", "unknown")
    extra = ", ".join("%s %s" % (k.lower(), fields[k]) for k in ("CPU family", "Model", "Stepping")
                      if fields.get(k))
    return "%s (%s)" % (name, extra) if extra else name


def host_threads() -> tuple:
    """(threads the oracle may use, the CPUs this process may run on, nproc).
    The oracle takes every CPU of the process's affinity set, at most 16: a
    one-GPU share of the host."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return min(16, aff), aff, os.cpu_count() or 1


def cpu_baseline(parts, budget_nodes, nthreads, single_nodes=2.5e8):
    """The oracle, untouched, on a bounded sample: from each part (width) of
    the workload, instances taken in order, skipping any whose stored node
    total alone exceeds a thread's share, until the part's sample holds about
    its share of ``budget_nodes`` (in proportion to its node total)."""
    from oracle import oracle
    per_part = []
    for g, _, _ in parts:
        with open(os.path.join(ROOT, "tests", "golden", g + ".json")) as f:
            per_part.append([sum(r["nodes"]) for r in json.load(f)["instances"]])
    grand = sum(sum(p) for p in per_part)
    nodes = secs = count = 0
    # one thread on the smallest instances (the paper's one-core comparison)
    g0, states0, w0 = max(zip(parts, per_part), key=lambda x: sum(x[1]))[0]
    per0 = max(per_part, key=sum)
    order = np.argsort(per0, kind="stable")
    pick0, tot0 = [], 0
    for i in order[len(order) // 4:]:
        pick0.append(int(i))
        tot0 += per0[i]
        if tot0 >= single_nodes:
            break
    t0 = time.perf_counter()
    r1 = oracle.solve(states0[sorted(pick0)], w0, nthreads=1)
    single = r1.total_nodes / (time.perf_counter() - t0)
    assert r1.rc == 0
    for (g, states, w), per in zip(parts, per_part):
        budget = budget_nodes * sum(per) / grand
        share = max(budget / max(1, nthreads) * 2, min(per))
        pick, tot = [], 0
        for i, n in enumerate(per):
            if n > share:
                continue
            pick.append(i)
            tot += n
            if tot >= budget:
                break
        t0 = time.perf_counter()
        r = oracle.solve(states[pick], w, nthreads=nthreads)
        secs += time.perf_counter() - t0
        assert r.rc == 0
        nodes += r.total_nodes
        count += len(pick)
    return {"value": round(nodes / secs, 1), "unit": "nodes/s", "cores": nthreads,
            "kind": "oracle",
            "sample": "%d of the workload's instances (%d nodes, %.1f s wall, %d threads)" % (
                count, nodes, secs, nthreads),
            "single_thread_value": round(single, 1),
            "single_thread_sample": "%d instances from the second quartile up by size (%d nodes)" % (
                len(pick0), r1.total_nodes),
            "cpu_model": cpu_model()}


def first_solution_leg(bpida, part, states, width, d_states, d_len, d_nodes, stream, with_cpu,
                       sample_nodes=6e8):
    """The final limit stopping at its first goal (Alg. 1 as printed; the
    semantics of the paper's single-core comparison): the GPU on the whole
    batch, and the GPU and the oracle on one host thread on the same bounded
    sample.  Context, not the metric."""
    import torch
    bpida.set_option("first_solution", 1)
    try:
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            rc = bpida.solve_device(d_states, d_len, d_nodes, width=width, stream=stream)
            ts.append(time.perf_counter() - t0)
            if rc != bpida.OK:
                raise bpida.BpidaError(rc, "first-solution solve")
        torch.cuda.synchronize()
        n = states.shape[0]
        res = {"gpu_ms_per_step": round(float(np.median(ts)) * 1e3, 3),
               "gpu_instances_per_s": round(n / float(np.median(ts)), 2),
               "nodes_per_step": int(d_nodes.cpu().numpy().view(np.uint64).sum(dtype=np.uint64))}
        if not with_cpu:
            return res
        with open(os.path.join(ROOT, "tests", "golden", part[0] + ".json")) as f:
            per = [sum(r["nodes"]) for r in json.load(f)["instances"]]
        pick, tot = [], 0
        for i, c in enumerate(per):
            if c > sample_nodes / 4:
                continue
            pick.append(i)
            tot += c
            if tot >= sample_nodes:
                break
        sub = np.ascontiguousarray(states[pick])
        gs = []
        for _ in range(3):
            t0 = time.perf_counter()
            rc, _, _ = bpida.solve_raw(sub, width)
            gs.append(time.perf_counter() - t0)
            if rc != bpida.OK:
                raise bpida.BpidaError(rc, "first-solution sample")
    finally:
        bpida.set_option("first_solution", 0)
    from oracle import oracle
    t0 = time.perf_counter()
    r = oracle.solve(sub, width, nthreads=1, first_solution=True)
    cpu = time.perf_counter() - t0
    assert r.rc == 0
    res.update({"sample": "%d instances (oracle: %d nodes)" % (len(pick), r.total_nodes),
                "sample_gpu_ms": round(float(np.median(gs)) * 1e3, 3),
                "sample_oracle_one_thread_ms": round(cpu * 1e3, 1),
                "speedup_vs_one_core": round(cpu / float(np.median(gs)), 1)})
    return res


def valu_issue_probe():
    """The integer VALU issue rates measured on this device, per instruction
    class: independent chains in every lane of 16384 waves
    (libvalu_probe.so, built with the library): the class most of the search
    round consists of (three-operand, 64-bit, multiply, mbcnt, compare and
    select instructions, timed with v_bfe_u32) issues one wave64 instruction
    per SIMD per 4 clocks, the simple two-operand class (timed with
    v_add_u32) up to two.  ``gops`` is the faster one.  None if the probe is
    not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_1705_02843_amd", "libvalu_probe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.bpida_valu_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.bpida_valu_probe.restype = ctypes.c_int
    res = {}
    for kind, tag in ((1, "bfe_class"), (0, "add_class")):
        rate, ms = ctypes.c_double(0), ctypes.c_double(0)
        if lib.bpida_valu_probe(kind, 4096, 20000, ctypes.byref(rate), ctypes.byref(ms)) != 0:
            return None
        res[tag] = {"wave64_valu_per_s": round(rate.value, 1),
                    "per_cu_clock_at_2_4_ghz": round(rate.value / (256 * 2.4e9), 3),
                    "gops": round(rate.value * 64 / 1e9, 1)}
    res["gops"] = res["add_class"]["gops"]
    res["note"] = ("independent chains, 4096 workgroups of 4 waves; gops: the faster (dual-issued) "
                   "add class; most of the round's instructions are of the single-issue bfe class")
    return res


def load_traffic(src_hash, mode, workload):
    """The committed rocprofv3 counter record of the timed search kernel (HBM
    bytes per launch, VALU busy, active lanes), if it was taken on the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (
        "batch4" if mode == "batched" else "search4", workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != src_hash:
        return None
    return t


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3_uneven", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget-nodes", type=float, default=4e9)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="batched", choices=sorted(MODES),
                    help="path timed for `value` (batched: one persistent launch with a device "
                         "work queue; plain: one launch per instance and f-limit)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other mode beside it")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="timed steps of the other mode (median reported; one warm-up step first)")
    ap.add_argument("--untuned", action="store_true",
                    help="ignore the autotuner's table (paper_1705_02843_amd/tuning/) and use the "
                         "library defaults")
    ap.add_argument("--no-static-lb", action="store_true",
                    help="plain mode without BPIDA*'s static load balancing (Sec. 5)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the timed steps (no comparison, host-buffer, first-solution or CPU "
                         "legs): for profiling runs")
    ap.add_argument("--no-first-solution", action="store_true",
                    help="skip the first-solution leg (final limit stops at its first goal)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg (continuous batching on a Poisson request stream)")
    ap.add_argument("--serve-n", type=int, default=4000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.kernel_only:
        args.no_compare = args.no_first_solution = args.no_cpu_baseline = args.no_serving = True

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(instances shard across GPUs with no exchange; see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1705_02843_amd import bpida

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    desc, width = WORKLOADS[args.workload]
    parts = make_parts(args.workload)
    widths = None
    if width == 0:  # mixed widths: bytes back to back, widths on the host
        widths = np.concatenate([np.full(p[1].shape[0], p[2], np.int32) for p in parts])
        states = np.concatenate([p[1].reshape(-1) for p in parts])
        n = widths.shape[0]
        if args.mode != "batched":
            raise SystemExit("bench.py: the mixed-width workload runs in batched mode only")
    else:
        states = parts[0][1]
        n = states.shape[0]
    tuned = None
    if not args.untuned:
        from paper_1705_02843_amd import autotune
        tuned = autotune.lookup(n, width)
        if tuned and args.mode == "batched":
            autotune.apply(tuned)
    d_states = torch.from_numpy(states).cuda()
    d_len = torch.empty(n, dtype=torch.int32, device="cuda")
    d_nodes = torch.empty((n, bpida.MAX_THRESHOLDS), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    if args.calibrate_copy_mib:
        nb = args.calibrate_copy_mib << 20
        x = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    bpida.set_option("static_lb", 0 if args.no_static_lb else 1)

    def run_mode(mode, steps, warmup):
        bpida.set_option("mode", MODES[mode])
        if mode == "plain":  # the plain path always runs with its own defaults
            for k in ("frontier_depth", "lds_stack_capacity", "max_workgroups"):
                bpida.set_option(k, -1 if k != "max_workgroups" else 0)

        def step():
            if widths is not None:
                rc = bpida.solve_mixed_device(d_states, widths, d_len, d_nodes, stream=stream)
            else:
                rc = bpida.solve_device(d_states, d_len, d_nodes, width=width, stream=stream)
            if rc != bpida.OK:
                raise bpida.BpidaError(rc, "bpida_solve_device")

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        progress("%s: %d warm-up step(s) done" % (mode, warmup))
        acc = {}
        per_step = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            step()  # returns once the results are in device memory
            per_step.append(time.perf_counter() - ts)
            progress("%s: step %d of %d, %.3f s" % (mode, len(per_step), steps, per_step[-1]))
            for k, v in bpida.last_stats().items():
                acc[k] = acc.get(k, 0) + v
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc["median_step_s"] = float(np.median(per_step))
        nodes_step = int(d_nodes.cpu().numpy().view(np.uint64).sum(dtype=np.uint64))
        if expect is not None and nodes_step != expect:
            raise SystemExit("%s: node total %d differs from the stored oracle total %d" % (
                mode, nodes_step, expect))
        assert (d_len.cpu().numpy() >= 0).all()
        return dt, nodes_step, acc

    expect = golden_total(parts)
    dt, nodes_per_step, acc = run_mode(args.mode, args.steps, args.warmup)
    search_nodes, search_us, launches = acc["search_nodes"], acc["search_us"], acc["launches"]
    rounds = acc["rounds"]
    total_nodes = nodes_per_step * args.steps
    value = total_nodes / dt
    avg_launch_s = (search_us / launches) * 1e-6 if launches else float("nan")
    ops_per_launch = search_nodes * OPS_PER_NODE / launches if launches else 0.0
    achieved = ops_per_launch / avg_launch_s / 1e9 if launches else 0.0
    # algorithmic HBM bytes per launch: 16 per split-tree root read per limit
    # (8 bytes of state, 8 of bookkeeping); the search itself stays on chip
    algo_bytes = (16 * acc.get("roots_read", 0) // launches) if launches else None
    src_hash = kernel_source_hash()
    counters = load_traffic(src_hash, args.mode, args.workload)
    traffic = counters.get("bytes_per_launch") if counters else None
    npl = (bpida.get_option("nodes_per_round") if args.mode == "batched"
           else bpida.get_option("plain_nodes_per_round"))
    cap = bpida.get_option("lds_stack_capacity")
    if cap < 0:
        cap = 1024 if npl == 64 else 512
    if args.mode == "batched":
        kname = "batch4_kernel<%d, %d, %d, %s>" % (cap, npl, bpida.get_option("wg_size") // 64,
                                                    "true" if bpida.get_option("first_solution") else "false")
    else:
        pn = bpida.get_option("plain_nodes_per_round")
        kname = ("search64_kernel<%d>" if pn == 64 else "search4_kernel<%d>") % cap
    wg_total = acc.get("wg_us_search", 0) + acc.get("wg_us_queue", 0) + acc.get("wg_us_idle", 0)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n_instances": n,
                   "mode": args.mode,
                   "frontier_depth": bpida.get_option("frontier_depth"),
                   "lds_stack_capacity": bpida.get_option("lds_stack_capacity"),
                   "nodes_per_round": bpida.get_option("nodes_per_round"),
                   "wg_size": bpida.get_option("wg_size"),
                   "max_workgroups": bpida.get_option("max_workgroups"),
                   "donate_every": bpida.get_option("donate_every"),
                   "donate_min": bpida.get_option("donate_min"),
                   "queue_chunk": bpida.get_option("queue_chunk"),
                   "tuned": bool(tuned) and args.mode == "batched"},
        "instances_per_s": round(n * args.steps / dt, 2),
        "ms_per_step_median": round(acc["median_step_s"] * 1e3, 3),
        "nodes_per_step": nodes_per_step,
        "roofline": {"bound": "alu", "achieved": round(achieved, 1), "peak": round(PEAK_INT_GOPS, 1),
                     "unit": "Gop/s", "frac": round(achieved / PEAK_INT_GOPS, 4),
                     "peak_single_issue": round(PEAK_INT_SINGLE_GOPS, 1),
                     "frac_single_issue": round(achieved / PEAK_INT_SINGLE_GOPS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes": algo_bytes,
                     "traffic_over_algorithmic": (round(traffic / algo_bytes, 2)
                                                  if traffic and algo_bytes else None),
                     "kernel": kname,
                     "ops_per_node": OPS_PER_NODE,
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "launches_per_step": launches // max(1, args.steps),
                     "search_nodes_per_s_in_kernel": round(search_nodes / (search_us * 1e-6), 1)
                     if search_us else None},
        "counters": ({k: counters[k] for k in ("instructions_per_round", "salu_instructions_per_round",
                                                "valu_instructions_per_node", "valu_per_cu_clock",
                                                "valu_issue_frac",
                                                "active_lanes_frac", "lds_bank_conflict_cycles",
                                                "waves_per_simd")
                      if k in counters} if counters else None),
        "search_rounds_per_step": rounds // max(1, args.steps),
        "pop_occupancy": round(search_nodes / (float(npl) * rounds), 4) if rounds else None,
        "kernel_source_hash": src_hash,
    }
    if args.mode == "batched" and wg_total:
        out["batched"] = {"grid": acc["grid"] // max(1, args.steps),
                          "busy_frac": round(acc["wg_us_search"] / wg_total, 4),
                          "queue_frac": round(acc["wg_us_queue"] / wg_total, 4),
                          "chunks_donated_per_step": acc["chunks_pushed"] // max(1, args.steps)}
    if not args.no_compare and widths is None:
        # the other mode on the same states: for batched, plain BPIDA* (one
        # launch per instance and limit) with Alg. 1's 16-node lane map and
        # with the batched kernel's 64-node round, so that the batching win
        # and the round's own win are stated apart
        legs = ([("plain16", "plain", 16), ("plain64", "plain", 64)] if args.mode == "batched"
                else [("batched", "batched", 16)])
        saved = {k: bpida.get_option(k) for k in ("frontier_depth", "lds_stack_capacity",
                                                  "max_workgroups", "plain_nodes_per_round")}
        out["compare"] = {}
        for tag, other, pnpl in legs:
            bpida.set_option("plain_nodes_per_round", pnpl)
            _, _, oacc = run_mode(other, args.compare_steps, 1)
            for k, v in saved.items():
                bpida.set_option(k, v)
            odt = oacc["median_step_s"]
            oshare = (oacc["search_nodes"] / (oacc["search_us"] * 1e-6)) if oacc["search_us"] else None
            out["compare"][tag] = {
                "mode": other, "value": round(nodes_per_step / odt, 1), "unit": "nodes/s",
                "ms_per_step_median": round(odt * 1e3, 3), "instances_per_s": round(n / odt, 2),
                "steps": args.compare_steps, "warmup": 1,
                "search_nodes_per_s_in_kernel": round(oshare, 1) if oshare else None,
                "launches_per_step": oacc["launches"] // max(1, args.compare_steps),
                "speedup_of_instances_per_s": round((n * args.steps / dt) / (n / odt), 3)}
        bpida.set_option("mode", MODES[args.mode])
    if args.mode == "batched" and not args.kernel_only:
        # the host-buffer entry (PCIe copies in and out included), beside `value`
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            if widths is not None:
                rc, _, hn = bpida.solve_mixed_raw([states[o:o + w * w] for o, w in zip(
                    np.concatenate([[0], np.cumsum(widths.astype(np.int64) ** 2)[:-1]]), widths)])
            else:
                rc, _, hn = bpida.solve_raw(states, width)
            ts.append(time.perf_counter() - t0)
            if rc != bpida.OK:
                raise bpida.BpidaError(rc, "host-buffer solve")
        if int(hn.sum(dtype=np.uint64)) != nodes_per_step:
            raise SystemExit("host-buffer solve: node total differs")
        out["host_buffers"] = {"ms_per_call_median": round(float(np.median(ts[1:])) * 1e3, 3),
                               "nodes_per_s": round(nodes_per_step / float(np.median(ts[1:])), 1),
                               "note": "bpida_solve / bpida_solve_mixed on host arrays: "
                                       "copies in and out included"}
    if args.mode == "batched" and widths is None and not args.no_first_solution:
        out["first_solution"] = first_solution_leg(bpida, parts[0], states, width, d_states, d_len,
                                                   d_nodes, stream, not args.no_cpu_baseline)
    if not args.kernel_only and not args.no_serving and widths is None and width == 4:
        # the continuous-batching server on the c5 stream (Poisson arrivals),
        # answers checked against the batched solve of the same states
        from paper_1705_02843_amd import serve_bench
        progress("serving: %d requests at %.0f per second" % (args.serve_n, args.serve_rate))
        sv = serve_bench.serve(n=args.serve_n, rate=args.serve_rate)
        if not sv["identical_to_batched_solve"]:
            raise SystemExit("served answers differ from the batched solve")
        out["serving"] = {k: sv[k] for k in ("requests", "rate_req_per_s", "p50_ms", "p90_ms",
                                             "p99_ms", "max_ms", "instances_per_s", "nodes_per_s",
                                             "elapsed_s", "identical_to_batched_solve",
                                             "max_inflight")}
    probe = None if args.kernel_only else valu_issue_probe()
    if probe:
        out["roofline"]["peak_measured"] = probe
        out["roofline"]["frac_of_measured"] = round(achieved / probe["gops"], 4)
    if not args.no_cpu_baseline:
        nthreads, aff, nproc = host_threads()
        progress("oracle on %d host threads" % nthreads)
        out["cpu_baseline"] = cpu_baseline(parts, args.cpu_budget_nodes, nthreads)
        out["cpu_baseline"]["host_cpus"] = {"affinity": aff, "nproc": nproc}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
