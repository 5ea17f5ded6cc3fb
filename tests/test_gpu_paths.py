"""One optimal path per instance: Alg. 1's BPDFS returns the goal "and its
parents".  The GPU rebuilds it after the solve by exact-limit probes; it must
equal, move for move, the oracle's path (the moves to the first goal of a
U, L, R, D depth-first search at the optimal limit: the lexicographically
smallest optimal move sequence, unique), stored by
``tests/golden/make_golden.py --paths`` or computed live; it must replay from
the start to the goal in exactly out_len moves; and lengths and per-limit
counts must equal those of bpida_solve.
"""
import json
import os
import sys

import numpy as np
import pytest

import puzzle_ref as P

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1705_02843_amd import bpida
    keys = ("frontier_depth", "wg_size", "first_solution", "mode")
    saved = {k: bpida.get_option(k) for k in keys}
    yield bpida
    for k, v in saved.items():
        bpida.set_option(k, v)


def parse_state(txt, w):
    step = 1 if w <= 4 else 2
    return np.array([int(txt[k:k + step], 16) for k in range(0, len(txt), step)], np.uint8)


def load_paths(name):
    path = os.path.join(GOLDEN, name + "_paths.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    w = g["width"]
    states = np.stack([parse_state(r["state"], w) for r in g["instances"]])
    length = np.array([r["length"] for r in g["instances"]], np.int32)
    paths = [[int(c) for c in r["path"]] for r in g["instances"]]
    index = [r["index"] for r in g["instances"]]
    return w, states, length, paths, index


def load_counts(name, index):
    g = json.load(open(os.path.join(GOLDEN, name + ".json")))
    nodes = np.zeros((len(index), 64), np.uint64)
    for k, i in enumerate(index):
        rec = g["instances"][i]
        nodes[k, :len(rec["nodes"])] = rec["nodes"]
    return nodes


def check_paths(w, states, got_len, got_path, want_len, want_paths, tag):
    np.testing.assert_array_equal(got_len, want_len)
    for i in range(states.shape[0]):
        L = int(want_len[i])
        row = got_path[i]
        assert list(row[:L]) == want_paths[i], (tag, i, list(row[:L]), want_paths[i])
        assert (row[L:] == 0xFF).all(), (tag, i)
        end = P.replay(tuple(int(x) for x in states[i]), w, row[:L])
        assert end == P.goal(w), (tag, i)


@pytest.mark.parametrize("name", ["c1_walk40", "c2_md30_38", "c3_uneven", "c4_mixed_w3",
                                  "c4_mixed_w4", "c4_mixed_w5"])
def test_paths_equal_the_oracle_paths(B, name):
    d = load_paths(name)
    if d is None:
        pytest.skip("no stored paths for %s" % name)
    w, states, want_len, want_paths, index = d
    _say("case: paths of %s, %d instances, width %d" % (name, len(index), w))
    rc, ln, nodes, path = B.solve_paths_raw(states, w)
    assert rc == B.OK, B.strerror(rc)
    check_paths(w, states, ln, path, want_len, want_paths, name)
    np.testing.assert_array_equal(nodes, load_counts(name, index))


def test_paths_of_short_walks_and_bad_states(B):
    """Goal, one-move and short-walk states (the goal inside the split tree
    at depth 10), and an unsolvable and an invalid state, against the oracle
    run live."""
    from oracle import oracle
    from paper_1705_02843_amd import instances as I
    rng = np.random.Generator(np.random.PCG64(78))
    states = [np.arange(16, dtype=np.uint8)]
    states += [I.random_walk(rng, 4, k)[0] for k in range(1, 15) for _ in range(2)]
    states = np.stack(states)
    bad = states[:3].copy()
    bad[1, 1], bad[1, 2] = bad[1, 2], bad[1, 1]  # unsolvable
    bad[2, 0] = bad[2, 5]                         # invalid
    allst = np.concatenate([states, bad[1:]])
    want = oracle.solve(states, 4, nthreads=8, with_path=True)
    assert want.rc == 0
    for depth in (10, 2):
        _say("case: paths of short walks, frontier depth %d" % depth)
        B.set_option("frontier_depth", depth)
        rc, ln, nodes, path = B.solve_paths_raw(allst, 4)
        assert rc == B.EUNSOLVABLE
        n = states.shape[0]
        np.testing.assert_array_equal(ln[:n], want.length)
        np.testing.assert_array_equal(nodes[:n], want.nodes)
        np.testing.assert_array_equal(path[:n], want.path)
        assert (ln[n:] == -1).all() and (path[n:] == 0xFF).all()
        assert (path[0] == 0xFF).all()  # the goal itself: no move


def test_paths_device_entry_wide_workgroups_first_solution(B):
    """The device entry on a side stream, with 4-wave workgroups and the
    first_solution option (the last count then varies; lengths and paths
    do not)."""
    import torch
    d = load_paths("c1_walk40")
    w, states, want_len, want_paths, index = d
    B.set_option("wg_size", 256)
    B.set_option("first_solution", 1)
    n = states.shape[0]
    _say("case: device-entry paths of c1_walk40, wg_size 256, first solution")
    d_states = torch.from_numpy(states).cuda()
    d_len = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    d_nodes = torch.zeros((n, 64), dtype=torch.int64, device="cuda")
    d_path = torch.zeros((n, 256), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc = B.solve_paths_device(d_states, d_len, d_nodes, d_path, stream=s)
    s.synchronize()
    assert rc == B.OK, B.strerror(rc)
    check_paths(w, states, d_len.cpu().numpy(), d_path.cpu().numpy(), want_len, want_paths, "dev")
