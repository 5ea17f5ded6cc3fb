"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact on every output (integer search): optimal lengths and the node
count of every f-limit, final limit run to completion.  Full-size cases use
the stored oracle results in tests/golden/ (written by make_golden.py from the
oracle alone); small cases call the oracle directly.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU test on a box without a GPU"
    from paper_1705_02843_amd import bpida
    return bpida


OPTION_KEYS = ("mode", "frontier_depth", "lds_stack_capacity", "spill_capacity",
               "max_workgroups", "max_threshold", "queue_capacity", "watchdog_ms",
               "nodes_per_round", "budget_ms", "first_solution", "static_lb", "start_threshold",
               "seed_chunk", "plain_nodes_per_round", "push_spin", "wg_size", "donate_every",
               "donate_min")
# plain: one launch per instance and limit, 16-node rounds (Alg. 1's map);
# plain64: the same with 64-node rounds; batched: persistent launch, 64-node
# rounds; batched16: persistent, 16-node rounds (tracks pruned f, so every
# limit advance checks f_next = L + 2 on the device)
MODES = {"plain": {"mode": 0, "plain_nodes_per_round": 16},
         "plain64": {"mode": 0, "plain_nodes_per_round": 64},
         "batched": {"mode": 1, "nodes_per_round": 64},
         "batched16": {"mode": 1, "nodes_per_round": 16}}


def set_mode(B, mode):
    for k, v in MODES[mode].items():
        B.set_option(k, v)


@pytest.fixture
def opts(B):
    keys = OPTION_KEYS
    saved = {k: B.get_option(k) for k in keys}
    yield B
    for k, v in saved.items():
        B.set_option(k, v)


def load_golden(name):
    g = json.load(open(os.path.join(GOLDEN, name + ".json")))
    states = np.array([[int(c, 16) for c in rec["state"]] for rec in g["instances"]], np.uint8)
    n = len(g["instances"])
    length = np.array([rec["length"] for rec in g["instances"]], np.int32)
    nodes = np.zeros((n, 64), np.uint64)
    for i, rec in enumerate(g["instances"]):
        nodes[i, :len(rec["nodes"])] = rec["nodes"]
        h0 = rec["limits"][0]
        assert rec["limits"] == [h0 + 2 * j for j in range(len(rec["limits"]))]
    return states, length, nodes


def oracle_expect(states, width=4):
    from oracle import oracle
    r = oracle.solve(states, width, nthreads=8)
    return r


def assert_parity(got_len, got_nodes, want_len, want_nodes, tag=""):
    bad = np.nonzero((got_len != want_len) | (got_nodes != want_nodes).any(axis=1))[0]
    assert bad.size == 0, "%s: %d instances differ, first %d: len %d vs %d, nodes %s vs %s" % (
        tag, bad.size, bad[0], got_len[bad[0]], want_len[bad[0]],
        got_nodes[bad[0], :12].tolist(), want_nodes[bad[0], :12].tolist())


@pytest.mark.parametrize("mode", sorted(MODES))
def test_walk40_64_instances_exact(opts, mode):
    B = opts
    _say("case: c1_walk40 full, mode=%s" % mode)
    set_mode(B, mode)
    states, want_len, want_nodes = load_golden("c1_walk40")
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, nodes, want_len, want_nodes, "c1")


@pytest.mark.parametrize("mode", sorted(MODES))
def test_md30_38_100_instances_exact(opts, mode):
    B = opts
    _say("case: c2_md30_38 full (100 instances, 2.2e10 nodes), mode=%s" % mode)
    set_mode(B, mode)
    states, want_len, want_nodes = load_golden("c2_md30_38")
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, nodes, want_len, want_nodes, "c2")
    st = B.last_stats()
    _say("c2 stats: %s" % st)


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("depth", [0, 1, 2, 5, 8, 12])
def test_split_depths_agree(opts, depth, mode):
    B = opts
    _say("case: c1 first 24, frontier_depth=%d, mode=%s" % (depth, mode))
    set_mode(B, mode)
    states, want_len, want_nodes = load_golden("c1_walk40")
    states, want_len, want_nodes = states[:24], want_len[:24], want_nodes[:24]
    B.set_option("frontier_depth", depth)
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, nodes, want_len, want_nodes, "D=%d" % depth)


CAPS = [("plain", 128), ("plain", 1024), ("plain64", 512), ("plain64", 2048),
        ("batched16", 128), ("batched16", 256), ("batched16", 2048), ("batched", 512),
        ("batched", 640), ("batched", 672), ("batched", 768), ("batched", 1024), ("batched", 2048)]


@pytest.mark.parametrize("mode,cap", CAPS)
def test_lds_capacity_and_spill_agree(opts, cap, mode):
    B = opts
    _say("case: c2 6 instances, lds_stack_capacity=%d, depth 6, mode=%s" % (cap, mode))
    set_mode(B, mode)
    states, want_len, want_nodes = load_golden("c2_md30_38")
    pick = [1, 4, 17, 26, 39, 77]
    states, want_len, want_nodes = states[pick], want_len[pick], want_nodes[pick]
    B.set_option("lds_stack_capacity", cap)
    B.set_option("frontier_depth", 6)
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, nodes, want_len, want_nodes, "cap=%d" % cap)
    if cap == 128 or (mode in ("batched", "plain64") and cap == 512):
        assert B.last_stats()["spilled"] > 0  # the spill path was exercised


@pytest.mark.parametrize("cap", [640, 672, 1024])
def test_aggressive_donation_exact(opts, cap):
    """Donation at every 64-round poll from any stack of two or more entries
    (the smallest interval and threshold the options allow), on the split
    (640, 1024) and interleaved (672) width-4 stacks: every donated half
    moves through the stack's own layout and back; exact against the stored
    oracle results, with donations counted."""
    B = opts
    _say("case: c2 first 30, donate_every 64, donate_min 2, stack %d" % cap)
    set_mode(B, "batched")
    B.set_option("lds_stack_capacity", cap)
    B.set_option("donate_every", 64)
    B.set_option("donate_min", 2)
    states, want_len, want_nodes = load_golden("c2_md30_38")
    states, want_len, want_nodes = states[:30], want_len[:30], want_nodes[:30]
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, nodes, want_len, want_nodes, "cap=%d" % cap)
    assert B.last_stats()["donations_voluntary"] > 0


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("maxwg", [1, 7, 300])
def test_grid_size_does_not_change_counts(opts, maxwg, mode):
    B = opts
    _say("case: c1 first 16, max_workgroups=%d, mode=%s" % (maxwg, mode))
    set_mode(B, mode)
    states, want_len, want_nodes = load_golden("c1_walk40")
    states, want_len, want_nodes = states[:16], want_len[:16], want_nodes[:16]
    B.set_option("max_workgroups", maxwg)
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK
    assert_parity(ln, nodes, want_len, want_nodes, "maxwg=%d" % maxwg)


@pytest.mark.parametrize("mode", sorted(MODES))
def test_short_walks_goal_inside_split_tree(opts, mode):
    B = opts
    set_mode(B, mode)
    from paper_1705_02843_amd import instances as I
    _say("case: walks of 0..14 moves, depth 10 (goal inside the split tree)")
    rng = np.random.Generator(np.random.PCG64(77))
    states = np.stack([I.random_walk(rng, 4, k)[0] for k in range(15) for _ in range(3)])
    want = oracle_expect(states)
    B.set_option("frontier_depth", 10)
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK
    assert_parity(ln, nodes, want.length, want.nodes, "short")


@pytest.mark.parametrize("mode", sorted(MODES))
def test_invalid_and_unsolvable_mixed_in(opts, mode):
    B = opts
    set_mode(B, mode)
    _say("case: batch with invalid and unsolvable states, mode=%s" % mode)
    states, want_len, want_nodes = load_golden("c1_walk40")
    s = states[:5].copy()
    s[1, 1], s[1, 2] = s[1, 2], s[1, 1]     # odd permutation: unsolvable
    s[3, 0] = s[3, 5]                         # duplicate tile: invalid
    rc, ln, nodes = B.solve_raw(s)
    assert rc == B.EUNSOLVABLE  # first failure in instance order
    assert ln[1] == -1 and ln[3] == -1 and (nodes[[1, 3]] == 0).all()
    ok = [0, 2, 4]
    assert_parity(ln[ok], nodes[ok], want_len[ok], want_nodes[ok], "mixed")


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("depth", [0, 6])
def test_goal_and_one_move(opts, mode, depth):
    B = opts
    set_mode(B, mode)
    B.set_option("frontier_depth", depth)
    _say("case: goal state and one-move states, mode=%s depth=%d" % (mode, depth))
    g = np.arange(16, dtype=np.uint8)
    r1 = g.copy(); r1[0], r1[1] = 1, 0
    d1 = g.copy(); d1[0], d1[4] = 4, 0
    rc, ln, nodes = B.solve_raw(np.stack([g, r1, d1]))
    assert rc == B.OK
    assert ln.tolist() == [0, 1, 1]
    assert nodes[:, 0].tolist() == [1, 2, 2] and (nodes[:, 1:] == 0).all()


@pytest.mark.parametrize("mode", sorted(MODES))
def test_limit_cap_keeps_completed_counts(opts, mode):
    B = opts
    set_mode(B, mode)
    _say("case: max_threshold cap, mode=%s" % mode)
    states, want_len, want_nodes = load_golden("c1_walk40")
    s = states[:4]
    h0 = [int(want_len[i]) for i in range(4)]
    B.set_option("max_threshold", 24)
    rc, ln, nodes = B.solve_raw(s)
    for i in range(4):
        if want_len[i] <= 24:
            assert ln[i] == want_len[i] and (nodes[i] == want_nodes[i]).all()
        else:
            assert ln[i] == -1 and rc == B.ELIMIT
            k = int((nodes[i] != 0).sum())
            assert (nodes[i, :k] == want_nodes[i, :k]).all()
    del h0


@pytest.mark.parametrize("mode", sorted(MODES))
def test_device_entry_on_torch_stream(opts, mode):
    import torch
    B = opts
    set_mode(B, mode)
    _say("case: bpida_solve_device on a side stream, mode=%s" % mode)
    states, want_len, want_nodes = load_golden("c1_walk40")
    d_states = torch.from_numpy(states).cuda()
    d_len = torch.full((64,), -9, dtype=torch.int32, device="cuda")
    d_nodes = torch.full((64, 64), 7, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc = B.solve_device(d_states, d_len, d_nodes, stream=s)
    s.synchronize()
    assert rc == B.OK
    assert_parity(d_len.cpu().numpy(), d_nodes.cpu().numpy().view(np.uint64), want_len,
                  want_nodes, "device")


def test_empty_batch(B):
    rc, ln, nodes = B.solve_raw(np.zeros((0, 16), np.uint8))
    assert rc == B.OK and ln.size == 0


def test_batched_queue_too_small_reports_enomem(opts):
    B = opts
    set_mode(B, "batched")
    _say("case: batched, one workgroup, 64-chunk queue, 3 instances at depth 12 (~700 seed chunks)")
    B.set_option("mode", 1)
    B.set_option("frontier_depth", 12)
    B.set_option("queue_capacity", 64)
    B.set_option("max_workgroups", 1)
    B.set_option("watchdog_ms", 300)
    states, _, _ = load_golden("c1_walk40")
    rc, ln, nodes = B.solve_raw(states[:3])
    assert rc == B.ENOMEM


def test_batched_uneven_batch_exact(opts):
    """Instances of very different depths in one persistent launch."""
    B = opts
    from paper_1705_02843_amd import instances as I
    _say("case: batched, 96 walks of length U{20..120}, max Manhattan 30")
    states, _ = I.walks_uniform_len(96, 4, 20, 120, 30, 31)
    want = oracle_expect(states)
    for mode in ("batched", "batched16"):
        set_mode(B, mode)
        rc, ln, nodes = B.solve_raw(states)
        assert rc == B.OK
        assert_parity(ln, nodes, want.length, want.nodes, "uneven " + mode)
    st = B.last_stats()
    _say("stats: %s" % st)


@pytest.mark.parametrize("cap", [128, 256])
def test_batched_rejects_ring_too_small_for_64_node_rounds(opts, cap):
    """4x4 with 64-node rounds needs 512 entries: a round can add 192, so a
    smaller stack spills on almost every round and the queue runs away."""
    B = opts
    set_mode(B, "batched")
    B.set_option("lds_stack_capacity", cap)
    states, _, _ = load_golden("c1_walk40")
    rc, _, _ = B.solve_raw(states[:2])
    assert rc == B.EINVAL


def test_lost_work_fails_fast(opts):
    """A queue too small for the batch drops work: the call reports
    BPIDA_ENOMEM, and the workgroups stop instead of searching on (or
    waiting for the idle watchdog).  One workgroup seeds all 100 instances
    before it takes anything, so a 64-chunk queue overflows for sure."""
    import time
    B = opts
    set_mode(B, "batched")
    B.set_option("queue_capacity", 64)
    B.set_option("max_workgroups", 1)
    states, _, _ = load_golden("c2_md30_38")
    _say("case: c2 with a 64-chunk work queue, one workgroup")
    t = time.time()
    rc, _, _ = B.solve_raw(states)
    dt = time.time() - t
    assert rc == B.ENOMEM, B.strerror(rc)
    assert B.last_stats()["error_bits"] & (1 | 2 | 16)
    assert dt < 5.0, dt


@pytest.mark.parametrize("mode,wg,cap", [("batched", 64, -1), ("batched16", 64, -1), ("batched", 128, -1),
                                         ("batched", 256, -1), ("batched", 64, 640), ("batched", 64, 672),
                                         ("batched", 64, 768)])
def test_c3_4096_batched_exact_where_stored_and_valid_everywhere(opts, mode, wg, cap):
    """The 4096-state uneven workload in one persistent launch (the grid is
    smaller than the batch): exact against the stored oracle results, and
    every instance consistent with its walk and its heuristic, for every
    workgroup size and for the small stacks (more waves, more spills).  With
    16-node rounds every pruned child's f is tracked and each limit advance
    checks f_next = L + 2 on the device."""
    B = opts
    from paper_1705_02843_amd import instances as I
    _say("case: c3_uneven, 4096 states, %s, wg_size %d, stack %d" % (mode, wg, cap))
    states, walk = I.c3_uneven()
    set_mode(B, mode)
    B.set_option("wg_size", wg)
    B.set_option("lds_stack_capacity", cap)
    rc, ln, nodes = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    name = "c3_uneven" if os.path.exists(os.path.join(GOLDEN, "c3_uneven.json")) else \
        "c3_uneven_first512"
    gs, want_len, want_nodes = load_golden(name)
    k = gs.shape[0]
    assert (gs == states[:k]).all()
    assert_parity(ln[:k], nodes[:k], want_len, want_nodes, name)
    h0 = np.array([I.manhattan_filter_value(x, 4) for x in states])
    assert (ln >= h0).all() and (ln <= walk).all() and ((walk - ln) % 2 == 0).all()
    ncols = (nodes != 0).sum(axis=1)
    assert (ncols == (ln - h0) // 2 + 1).all()
    for i in range(len(states)):
        row = nodes[i, :ncols[i]]
        assert (np.diff(row.astype(np.int64)) > 0).all()
    _say("c3 stats: %s" % B.last_stats())


@pytest.mark.parametrize("lb", [0, 1])
def test_plain_static_load_balancing_exact(opts, lb):
    """Plain BPIDA* with and without its static load balancing (Sec. 5): the
    re-split root sets expand exactly the oracle's nodes at every limit."""
    B = opts
    _say("case: plain, static_lb=%d, c1_walk40 + first 30 of c2_md30_38" % lb)
    set_mode(B, "plain")
    B.set_option("static_lb", lb)
    for name, k in (("c1_walk40", 64), ("c2_md30_38", 30)):
        states, length, nodes = load_golden(name)
        rc, ln, got = B.solve_raw(states[:k])
        assert rc == B.OK, B.strerror(rc)
        assert_parity(ln, got, length[:k], nodes[:k], "%s lb=%d" % (name, lb))
        added = B.last_stats()["lb_roots_added"]
        if lb == 0:
            assert added == 0
        elif name == "c2_md30_38":
            assert added > 0, "no root was re-split"


def test_plain_static_lb_small_split_depth(opts):
    """Re-splitting from a shallow split (D = 2, a handful of roots) goes
    several levels deep within one instance; counts stay exact."""
    B = opts
    _say("case: plain, static_lb=1, split depth 2")
    set_mode(B, "plain")
    B.set_option("static_lb", 1)
    B.set_option("frontier_depth", 2)
    states, length, nodes = load_golden("c2_md30_38")
    rc, ln, got = B.solve_raw(states[:12])
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, got, length[:12], nodes[:12], "D=2 lb")
    assert B.last_stats()["lb_roots_added"] > 0


def test_plain64_static_load_balancing_exact(opts):
    """Plain BPIDA* with 64-node rounds and the static load balancing: the
    per-root round counts it re-splits by come from the other kernel."""
    B = opts
    _say("case: plain64, static_lb=1, first 30 of c2_md30_38")
    set_mode(B, "plain64")
    B.set_option("static_lb", 1)
    states, length, nodes = load_golden("c2_md30_38")
    rc, ln, got = B.solve_raw(states[:30])
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, got, length[:30], nodes[:30], "plain64 lb")
    assert B.last_stats()["lb_roots_added"] > 0


def test_plain64_rejects_small_stacks(opts):
    B = opts
    set_mode(B, "plain64")
    B.set_option("lds_stack_capacity", 256)
    states, _, _ = load_golden("c1_walk40")
    rc, _, _ = B.solve_raw(states[:2])
    assert rc == B.EINVAL


@pytest.mark.parametrize("mode", ["plain", "plain64", "batched"])
def test_start_threshold_at_the_optimum(opts, mode):
    """Starting at the optimal length (or one below it: rounded up to h0's
    parity) runs only the final limit: its count is the stored one, the
    skipped columns stay zero."""
    B = opts
    _say("case: start_threshold = optimum, c1_walk40, %s" % mode)
    set_mode(B, mode)
    states, length, nodes = load_golden("c1_walk40")
    try:
        for delta in (0, -1):
            for i in (3, 17, 40):
                B.set_option("start_threshold", int(length[i]) + delta)
                rc, ln, got = B.solve_raw(states[i:i + 1])
                assert rc == B.OK, B.strerror(rc)
                k = int(np.count_nonzero(nodes[i]))
                assert ln[0] == length[i]
                assert got[0, k - 1] == nodes[i, k - 1] and not got[0, :k - 1].any()
                assert not got[0, k:].any()
    finally:
        B.set_option("start_threshold", -1)


@pytest.mark.parametrize("wg", [128, 256])
def test_workgroup_size_does_not_change_results(opts, wg):
    """Two or four independent waves per workgroup, each with its own stack:
    every count equal to the stored oracle results, also with a grid of a
    few workgroups (donation between waves of one workgroup and across)."""
    B = opts
    set_mode(B, "batched")
    B.set_option("wg_size", wg)
    for name, k, maxwg in (("c1_walk40", 64, 0), ("c2_md30_38", 30, 0), ("c2_md30_38", 12, 3)):
        _say("case: batched, wg_size=%d, %s first %d, max_workgroups=%d" % (wg, name, k, maxwg))
        B.set_option("max_workgroups", maxwg)
        states, length, nodes = load_golden(name)
        rc, ln, got = B.solve_raw(states[:k])
        assert rc == B.OK, B.strerror(rc)
        assert_parity(ln, got, length[:k], nodes[:k], "%s wg=%d" % (name, wg))


def test_workgroup_size_needs_64_node_rounds(opts):
    B = opts
    set_mode(B, "batched16")
    B.set_option("wg_size", 128)
    states, _, _ = load_golden("c1_walk40")
    rc, _, _ = B.solve_raw(states[:2])
    assert rc == B.EINVAL


@pytest.mark.parametrize("sc", [8, 16])
def test_batched_small_seed_chunks_exact(opts, sc):
    """Seeding a limit in chunks of fewer than 64 roots (several queue pushes
    per 64 candidate roots) leaves every count unchanged."""
    B = opts
    _say("case: batched, seed_chunk=%d, c1_walk40 + first 20 of c2_md30_38" % sc)
    set_mode(B, "batched")
    B.set_option("seed_chunk", sc)
    for name, k in (("c1_walk40", 64), ("c2_md30_38", 20)):
        states, length, nodes = load_golden(name)
        rc, ln, got = B.solve_raw(states[:k])
        assert rc == B.OK, B.strerror(rc)
        assert_parity(ln, got, length[:k], nodes[:k], "%s seed_chunk=%d" % (name, sc))


def test_batched_100k_cheap_instances_exact(opts):
    """A batch far larger than the grid (100,000 states from walks of 0..30
    moves, split tree and queue sized from the batch): exact against the
    oracle run live on the same states."""
    B = opts
    from paper_1705_02843_amd import instances as I
    rng = np.random.Generator(np.random.PCG64(77))
    states = np.stack([I.random_walk(rng, 4, int(k))[0] for k in rng.integers(0, 31, size=100000)])
    want = oracle_expect(states)
    assert want.rc == 0
    _say("case: batched, 100000 cheap states in one launch")
    set_mode(B, "batched")
    rc, ln, got = B.solve_raw(states)
    assert rc == B.OK, B.strerror(rc)
    assert_parity(ln, got, want.length, want.nodes, "100k")
