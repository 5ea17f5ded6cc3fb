"""Autotuner for the batched search: searches the launch options on a
workload, checks that every configuration returns identical results, and
writes the fastest configuration to a JSON table keyed by (architecture,
width, batch size class).

    python -m paper_1705_02843_amd.autotune --workload c3_uneven

Axes: nodes per round with the LDS stack capacity (16: four lanes per node,
Alg. 1's map; 64: one node per lane), the workgroup size (64, 128 or 256
threads: 1, 2 or 4 independent waves, Sec. 5's block = one wave, several
per workgroup), the root split depth D (4..10), the size of the persistent
grid (the occupancy limit, or a half, a quarter or an eighth of it), and the
donation policy (rounds between checks, smallest donating stack, entries per
donated chunk).  Batch size classes: tiny (up to 64 states), small (256),
medium (2048), large.  The
search is coordinate descent: starting from the stored or the library's
options, each axis in turn is swept with the others fixed and the fastest
value kept, for two passes over all axes.  Mixed-width workloads are keyed
"mixed" instead of by width.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning", "gfx950.json")
KEYS = ("nodes_per_round", "lds_stack_capacity", "wg_size", "frontier_depth", "max_workgroups",
        "donate_every", "donate_min", "queue_chunk")


def size_class(n: int) -> str:
    return "tiny" if n <= 64 else "small" if n <= 256 else "medium" if n <= 2048 else "large"


def axes(grid_full: int):
    """The values swept per axis; (nodes per round, stack capacity) move
    together."""
    return [
        ("round", [(16, 512), (64, 512), (64, 640), (64, 672), (64, 768), (64, 1024), (64, 2048)]),
        ("wg_size", [64, 128, 256]),
        ("frontier_depth", [4, 5, 6, 7, 8, 9, 10]),
        ("max_workgroups", [0, grid_full // 2, grid_full // 4, grid_full // 8]),
        ("donate_every", [64, 128, 256, 512]),
        ("donate_min", [-1, 16, 32, 64, 128, 256]),
        ("queue_chunk", [16, 32, 64]),
    ]


def valid(cfg: dict) -> bool:
    # several waves per workgroup need 64-node rounds and a power-of-two stack
    cap = cfg["lds_stack_capacity"]
    return cfg["wg_size"] == 64 or (cfg["nodes_per_round"] == 64 and cap & (cap - 1) == 0)


def set_axis(cfg: dict, axis: str, value) -> dict:
    out = dict(cfg)
    if axis == "round":
        out["nodes_per_round"], out["lds_stack_capacity"] = value
    else:
        out[axis] = value
    return out


def apply(options: dict) -> None:
    from . import bpida
    for k in KEYS:
        if k in options:
            bpida.set_option(k, int(options[k]))


def table_key(width: int) -> str:
    return "mixed" if width == 0 else "w%d" % width


def lookup(n: int, width: int = 4, path: str = TABLE):
    """Tuned options for a batch of n states of this width (0: mixed
    widths), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    entry = table.get(table_key(width), {}).get(size_class(n))
    return entry["best"] if entry else None


def tune(states: np.ndarray, width: int = 4, reps: int = 2, log=print, widths=None,
         start: dict | None = None, passes: int = 2) -> dict:
    """Coordinate descent over the axes on ``states`` (uint8 [n, w*w], or
    for a mixed batch the bytes back to back with ``widths`` int32 [n]),
    from ``start`` (or the library's current options)."""
    import torch

    from . import bpida
    n = states.shape[0] if widths is None else widths.shape[0]
    d_states = torch.from_numpy(np.ascontiguousarray(states)).cuda()
    d_len = torch.empty(n, dtype=torch.int32, device="cuda")
    d_nodes = torch.empty((n, bpida.MAX_THRESHOLDS), dtype=torch.int64, device="cuda")
    saved = {k: bpida.get_option(k) for k in KEYS + ("mode", "budget_ms")}
    bpida.set_option("mode", 1)
    ref = None
    results = []
    try:
        def solve():
            if widths is not None:
                return bpida.solve_mixed_device(d_states, widths, d_len, d_nodes)
            return bpida.solve_device(d_states, d_len, d_nodes, width=width)

        bpida.set_option("max_workgroups", 0)
        for _ in range(2):  # the first call sizes the workspace; the second is timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc = solve()
            if rc != bpida.OK:
                raise bpida.BpidaError(rc, "autotune reference solve")
            torch.cuda.synchronize()
            t_ref = time.perf_counter() - t0
        grid_full = bpida.last_stats()["grid"]
        # a configuration far slower than the reference is stopped by the
        # launch's own time budget (its workgroups exit; BPIDA_EINTERNAL)
        bpida.set_option("budget_ms", int(max(2000.0, 8000.0 * t_ref)))
        seen = {}

        def measure(cfg):
            nonlocal ref
            key = tuple(cfg[k] for k in KEYS)
            if key in seen:
                return seen[key]
            apply(cfg)
            best = float("inf")
            for _ in range(reps + 1):  # the first call warms up / sizes the workspace
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc = solve()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                too_slow = rc == bpida.EINTERNAL and bpida.last_stats()["error_bits"] & 8
                if rc in (bpida.ENOMEM, bpida.EINVAL) or too_slow:
                    # a small stack on a large batch overflows the work queue,
                    # or the configuration ran past the time budget: not
                    # usable on this workload
                    log("autotune %s rejected: %s" % (
                        cfg, "time budget" if too_slow else bpida.strerror(rc)))
                    seen[key] = float("inf")
                    return seen[key]
                if rc != bpida.OK:
                    raise bpida.BpidaError(rc, "autotune %r" % cfg)
                best = min(best, dt)
                if dt > 4 * t_ref + 0.05:  # far off the default: not worth repeating
                    break
            out = (d_len.cpu().numpy().copy(), d_nodes.cpu().numpy().copy())
            if ref is None:
                ref = out
            elif not (np.array_equal(ref[0], out[0]) and np.array_equal(ref[1], out[1])):
                raise RuntimeError("configuration %r changed the results" % cfg)
            results.append(dict(cfg, seconds=round(best, 5)))
            log("autotune %s %.4f s" % (cfg, best))
            seen[key] = best
            return best

        cur = {k: start[k] for k in KEYS} if start else None
        if cur is None:
            cur = {k: (saved[k] if k != "max_workgroups" else 0) for k in KEYS}
            if cur["lds_stack_capacity"] < 0:
                cur["lds_stack_capacity"] = 1024 if cur["nodes_per_round"] == 64 else 512
            if cur["frontier_depth"] < 0:
                cur["frontier_depth"] = 6
        cur_t = measure(cur)
        for _ in range(passes):
            for axis, values in axes(grid_full):
                for v in values:
                    cfg = set_axis(cur, axis, v)
                    if not valid(cfg) or cfg == cur:
                        continue
                    t = measure(cfg)
                    if t < cur_t:
                        cur, cur_t = cfg, t
    finally:
        for k, v in saved.items():
            bpida.set_option(k, v)
    results.sort(key=lambda r: r["seconds"])
    total = int(ref[1].view(np.uint64).sum(dtype=np.uint64))
    return {"best": {k: results[0][k] for k in KEYS}, "seconds": results[0]["seconds"],
            "nodes": total, "n": n, "search": "coordinate descent, %d passes" % passes,
            "results": results}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="c2_md30_38")
    ap.add_argument("--n", type=int, default=0, help="use the first n states of the workload")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--fresh", action="store_true",
                    help="start from the library's options, not the stored best")
    args = ap.parse_args()
    from . import instances
    widths = None
    width = 4
    if args.workload == "c4_mixed":
        d = instances.c4_mixed()
        widths = np.concatenate([np.full(d[w][0].shape[0], w, np.int32) for w in (3, 4, 5)])
        states = np.concatenate([d[w][0].reshape(-1) for w in (3, 4, 5)])
        width = 0
        n = widths.shape[0]
    else:
        states = getattr(instances, args.workload)()[0]
        if args.n:
            states = states[:args.n]
        n = states.shape[0]
    start = lookup(n, width, args.out) if not args.fresh else None
    if start:
        start = dict({"wg_size": 64, "queue_chunk": 64}, **start)
    res = tune(states, width, args.reps if n <= 2048 else 1, widths=widths, start=start,
               passes=args.passes)
    table = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            table = json.load(f)
    entry = dict(res, workload=args.workload, arch="gfx950")
    table.setdefault(table_key(width), {})[size_class(n)] = entry
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({"best": res["best"], "seconds": res["seconds"]}))


if __name__ == "__main__":
    main()
