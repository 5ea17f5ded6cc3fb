"""Serving benchmark: a Poisson stream of 15-puzzle requests into the
continuous-batching server, with per-request latency percentiles.

    python -m paper_1705_02843_amd.serve_bench [--n 4000 --rate 200]

Requests are the seeded c5 stream (exponential inter-arrival times, states
drawn as in the 4096-state uneven workload).  Each request is submitted at
its arrival time; latency = time its answer is first seen - arrival time.
Every answer is compared with a batched solve of the same states (exact
integers), so the numbers are for identical results.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def serve(n: int = 4000, rate: float = 200.0, inflight: int = 1024, ring: int = 8192,
          budget_s: float = 300.0) -> dict:
    """Replay the seeded c5 stream of ``n`` requests at ``rate`` per second
    into a running server; every answer is checked against a batched solve of
    the same states.  Returns the latency percentiles and throughput."""
    import torch

    from . import bpida, instances

    assert torch.cuda.is_available()
    arrivals, states, _ = instances.c5_poisson(n=n, rate_hz=rate)
    n = states.shape[0]

    # reference: the same states solved as one batch
    rc, ref_len, ref_nodes = bpida.solve_raw(states)
    if rc != bpida.OK:
        raise bpida.BpidaError(rc, "reference batched solve")

    saved_budget = bpida.get_option("budget_ms")
    bpida.set_option("budget_ms", int(budget_s * 1000))
    srv = bpida.Server(max_inflight=inflight, ring_capacity=ring)
    done_at = np.zeros(n)
    got_len = np.full(n, -9, np.int32)
    got_nodes = np.zeros((n, bpida.MAX_THRESHOLDS), np.uint64)
    pending = {}
    refused = 0
    k = 0
    t0 = time.perf_counter()
    try:
        while k < n or pending:
            now = time.perf_counter() - t0
            while k < n and arrivals[k] <= now:
                t = srv.submit(states[k])
                if t is None:  # ring full: retry this request after collecting
                    refused += 1
                    break
                pending[t] = k
                k += 1
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    i = pending.pop(t)
                    done_at[i] = time.perf_counter() - t0
                    got_len[i], got_nodes[i] = r[0], r[1]
            if time.perf_counter() - t0 > budget_s:
                raise RuntimeError("serving run exceeded its time budget")
    finally:
        rc = srv.stop()
        bpida.set_option("budget_ms", saved_budget)
    if rc != bpida.OK:
        raise bpida.BpidaError(rc, "bpida_server_stop")
    elapsed = done_at.max()
    same = bool((got_len == ref_len).all() and (got_nodes == ref_nodes).all())
    lat = (done_at - arrivals) * 1e3
    total_nodes = int(ref_nodes.sum(dtype=np.uint64))
    return {
        "metric": "serving latency and throughput (15-puzzle, Manhattan), continuous batching",
        "requests": n, "rate_req_per_s": rate,
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p90_ms": round(float(np.percentile(lat, 90)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "max_ms": round(float(lat.max()), 3),
        "instances_per_s": round(n / elapsed, 2),
        "nodes_per_s": round(total_nodes / elapsed, 1),
        "offered_nodes_per_s": round(total_nodes / arrivals[-1], 1),
        "elapsed_s": round(float(elapsed), 3),
        "ring_full_retries": refused,
        "identical_to_batched_solve": same,
        "max_inflight": inflight,
        "data": "synthetic (seeded c5 stream)",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=4000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--inflight", type=int, default=1024)
    ap.add_argument("--ring", type=int, default=8192)
    ap.add_argument("--budget-s", type=float, default=300.0)
    args = ap.parse_args()
    out = serve(args.n, args.rate, args.inflight, args.ring, args.budget_s)
    print(json.dumps(out), flush=True)
    if not out["identical_to_batched_solve"]:
        raise SystemExit("served answers differ from the batched solve")


if __name__ == "__main__":
    main()
