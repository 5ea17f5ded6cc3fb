"""Write the stored oracle results used by the parity tests.

Calls only the seeded instance generator and the CPU oracle (``oracle/``);
nothing here touches the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py c1_walk40 c2_md30_38

Each ``<workload>.json`` holds, per instance, the start state (hex nibbles),
the optimal length, the f-limits and the nodes expanded under each limit with
the final limit run to completion.

    python tests/golden/make_golden.py --paths c1_walk40 c2_md30_38 ...

writes ``<workload>_paths.json``: for the instances PATH_PICK selects, the
oracle's path (the moves U, L, R, D = 0..3 of the first goal its depth-first
search expands at the optimal limit: the lexicographically smallest optimal
move sequence), as a string of digits.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle  # noqa: E402
from paper_1705_02843_amd import instances  # noqa: E402

SPECS = {
    "c1_walk40": (lambda: instances.c1_walk40(), 4),
    "c2_md30_38": (lambda: instances.c2_md30_38(), 4),
    "c3_uneven_first512": (lambda: tuple(x[:512] for x in instances.c3_uneven()), 4),
    "c3_uneven": (lambda: instances.c3_uneven(), 4),
    # the mixed-width workload, one file per width (launch order 3, 4, 5)
    "c4_mixed_w3": (lambda: instances.c4_mixed()[3], 3),
    "c4_mixed_w4": (lambda: instances.c4_mixed()[4], 4),
    "c4_mixed_w5": (lambda: instances.c4_mixed()[5], 5),
}


# Instances whose paths are stored: all of a small workload, a prefix of a
# large one, or those whose stored all-solutions node total is below a bound.
PATH_PICK = {
    "c1_walk40": ("all", None),
    "c2_md30_38": ("all", None),
    "c3_uneven": ("first", 256),
    "c4_mixed_w3": ("all", None),
    "c4_mixed_w4": ("first", 256),
    "c4_mixed_w5": ("below", 3e8),
}


def write_paths(name: str, nthreads: int) -> None:
    make, width = SPECS[name]
    states, _ = make()
    how, arg = PATH_PICK[name]
    if how == "all":
        pick = list(range(states.shape[0]))
    elif how == "first":
        pick = list(range(min(arg, states.shape[0])))
    else:
        with open(os.path.join(HERE, name + ".json")) as f:
            tot = [sum(r["nodes"]) for r in json.load(f)["instances"]]
        pick = [i for i, t in enumerate(tot) if t < arg]
    sub = np.ascontiguousarray(states[pick])
    t0 = time.time()
    r = oracle.solve(sub, width, nthreads=nthreads, first_solution=True, with_path=True)
    dt = time.time() - t0
    assert r.rc == 0, r.rc
    recs = []
    for k, i in enumerate(pick):
        L = int(r.length[k])
        recs.append({"index": int(i),
                     "state": "".join("%x" % v if width <= 4 else "%02x" % v for v in states[i]),
                     "length": L,
                     "path": "".join(str(int(a)) for a in r.path[k, :L])})
    out = {"workload": name, "width": width, "n": len(recs), "pick": [how, arg],
           "oracle_seconds": round(dt, 1), "oracle_threads": nthreads, "instances": recs}
    with open(os.path.join(HERE, name + "_paths.json"), "w") as f:
        json.dump(out, f, indent=0, separators=(",", ":"))
    print(name, "paths of", len(recs), "instances", round(dt, 1), "s")


def write(name: str, nthreads: int) -> None:
    make, width = SPECS[name]
    states, walk = make()
    t0 = time.time()
    r = oracle.solve(states, width, nthreads=nthreads)
    dt = time.time() - t0
    assert r.rc == 0, r.rc
    recs = []
    for i in range(states.shape[0]):
        k = int(r.niter[i])
        recs.append({
            "state": "".join("%x" % v if width <= 4 else "%02x" % v for v in states[i]),
            "walk": int(walk[i]),
            "length": int(r.length[i]),
            "limits": [int(x) for x in r.limits[i, :k]],
            "nodes": [int(x) for x in r.nodes[i, :k]],
        })
    out = {"workload": name, "width": width, "n": int(states.shape[0]),
           "total_nodes": int(sum(sum(x["nodes"]) for x in recs)),
           "oracle_seconds": round(dt, 1), "oracle_threads": nthreads, "instances": recs}
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0, separators=(",", ":"))
    print(name, out["total_nodes"], "nodes", round(dt, 1), "s")


if __name__ == "__main__":
    args = sys.argv[1:]
    paths = bool(args) and args[0] == "--paths"
    if paths:
        args = args[1:]
    names = args or list(PATH_PICK if paths else SPECS)
    for nm in names:
        (write_paths if paths else write)(nm, os.cpu_count() or 1)
