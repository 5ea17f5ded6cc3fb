"""Batched search on 3x3 and 5x5 boards and on mixed-width batches.

Bit-exact against the CPU oracle run live on the same states (the oracle
handles every width).  5x5 states come from walks short enough for the
oracle to finish in seconds, plus the easy part of the 60-move workload.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1705_02843_amd import bpida
    keys = ("mode", "nodes_per_round", "lds_stack_capacity", "frontier_depth", "max_workgroups")
    saved = {k: bpida.get_option(k) for k in keys}
    bpida.set_option("mode", 1)
    yield bpida
    for k, v in saved.items():
        bpida.set_option(k, v)


def oracle_of(states, w):
    from oracle import oracle
    r = oracle.solve(np.stack(states), w, nthreads=8)
    assert r.rc == 0
    return r


def five_by_five_states(n_short=24):
    from paper_1705_02843_amd import instances as I
    rng = np.random.Generator(np.random.PCG64(55))
    out = [I.random_walk(rng, 5, k)[0] for k in range(2, 2 + n_short)]
    d = I.c4_mixed(n3=1, n4=1, n5=16)
    # the 60-move states whose optimum the oracle reaches within h0 + 10
    from oracle import oracle
    for s in d[5][0]:
        r = oracle.solve(s[None], 5, max_limit=oracle.manhattan(s, 5) + 10)
        if r.rc == 0:
            out.append(s)
    return out


def check(B, got_len, got_nodes, want, tag):
    bad = np.nonzero((got_len != want.length) | (got_nodes != want.nodes).any(axis=1))[0]
    assert bad.size == 0, "%s: %d differ, first %d: %s vs %s" % (
        tag, bad.size, bad[0], got_nodes[bad[0], :8], want.nodes[bad[0], :8])


@pytest.mark.parametrize("depth", [0, 4, 8])
def test_width3_exact(B, depth):
    from paper_1705_02843_amd import instances as I
    print("case: 3x3, 512 states, depth %d" % depth, flush=True)
    s3, _ = I.c4_mixed(n3=512, n4=1, n5=1)[3]
    want = oracle_of(list(s3), 3)
    B.set_option("frontier_depth", depth)
    rc, ln, nodes = B.solve_raw(s3, 3)
    assert rc == B.OK, B.strerror(rc)
    check(B, ln, nodes, want, "3x3")


@pytest.mark.parametrize("cap", [1024, 2048])
def test_width5_exact(B, cap):
    print("case: 5x5, short walks + easy 60-move states, ring %d" % cap, flush=True)
    states = five_by_five_states()
    want = oracle_of(states, 5)
    B.set_option("lds_stack_capacity", cap)
    rc, ln, nodes = B.solve_raw(np.stack(states), 5)
    assert rc == B.OK, B.strerror(rc)
    check(B, ln, nodes, want, "5x5")


def test_mixed_widths_one_launch_exact(B):
    from paper_1705_02843_amd import instances as I
    print("case: mixed 3x3 / 4x4 / 5x5 batch in one launch", flush=True)
    d = I.c4_mixed(n3=96, n4=48, n5=1)
    s3, s4 = list(d[3][0]), list(d[4][0][:48])
    s4 = [s for s in s4 if I.manhattan_filter_value(s, 4) <= 30][:24]
    s5 = five_by_five_states(12)
    w3, w4, w5 = oracle_of(s3, 3), oracle_of(s4, 4), oracle_of(s5, 5)
    rng = np.random.default_rng(4)
    items = [(s, w3, i) for i, s in enumerate(s3)] + [(s, w4, i) for i, s in enumerate(s4)] + \
        [(s, w5, i) for i, s in enumerate(s5)]
    order = rng.permutation(len(items))
    items = [items[k] for k in order]
    rc, ln, nodes = B.solve_mixed_raw([it[0] for it in items])
    assert rc == B.OK, B.strerror(rc)
    for k, (s, want, i) in enumerate(items):
        assert ln[k] == want.length[i] and (nodes[k] == want.nodes[i]).all(), k


def test_plain_mode_is_15_puzzle_only(B):
    from paper_1705_02843_amd import instances as I
    B.set_option("mode", 0)
    s3, _ = I.c4_mixed(n3=4, n4=1, n5=1)[3]
    rc, _, _ = B.solve_raw(s3, 3)
    assert rc == B.EINVAL


@pytest.mark.parametrize("cap", [256, 512])
def test_ring_too_small_for_5x5(B, cap):
    """5x5 needs 1024 entries (512 wide ones): with fewer, 64-node rounds
    spill on almost every round and the work queue runs away."""
    B.set_option("lds_stack_capacity", cap)
    s = five_by_five_states(4)[:4]
    rc, _, _ = B.solve_raw(np.stack(s), 5)
    assert rc == B.EINVAL


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def test_c4_mixed_one_launch_exact_and_same_as_alone(B):
    """The mixed-width workload (2048 3x3 + 2048 4x4 + 256 5x5) in one
    launch: every instance equal to its width's batch run alone, and exact
    against the stored oracle results of every width that has them."""
    import torch
    from paper_1705_02843_amd import instances as I
    print("case: c4 mixed workload, 4352 states, one launch", flush=True)
    d = I.c4_mixed()
    parts = [(3, d[3][0]), (4, d[4][0]), (5, d[5][0])]
    widths = np.concatenate([np.full(s.shape[0], w, np.int32) for w, s in parts])
    flat = np.concatenate([s.reshape(-1) for _, s in parts])
    n = widths.shape[0]
    d_states = torch.from_numpy(flat).cuda()
    d_len = torch.empty(n, dtype=torch.int32, device="cuda")
    d_nodes = torch.empty((n, B.MAX_THRESHOLDS), dtype=torch.int64, device="cuda")
    rc = B.solve_mixed_device(d_states, widths, d_len, d_nodes)
    assert rc == B.OK, B.strerror(rc)
    torch.cuda.synchronize()
    ln = d_len.cpu().numpy()
    nodes = d_nodes.cpu().numpy().view(np.uint64)
    off = 0
    for w, s in parts:
        k = s.shape[0]
        print("case: c4 width %d alone" % w, flush=True)
        rc, aln, anodes = B.solve_raw(s, w)
        assert rc == B.OK, B.strerror(rc)
        assert (aln == ln[off:off + k]).all() and (anodes == nodes[off:off + k]).all(), w
        g = _golden("c4_mixed_w%d" % w)
        if g is not None:
            for i, r in enumerate(g["instances"]):
                m = len(r["nodes"])
                assert ln[off + i] == r["length"], (w, i)
                assert list(nodes[off + i, :m]) == r["nodes"] and not nodes[off + i, m:].any(), (w, i)
        else:
            h0 = np.array([I.manhattan_filter_value(x, w) for x in s])
            assert (ln[off:off + k] >= h0).all() and ((ln[off:off + k] - h0) % 2 == 0).all()
        off += k


def test_c4_4x4_part_with_16_node_rounds_exact(B):
    """The 2048 4x4 states of the mixed workload with 16-node rounds, which
    track every pruned child's f (the device checks f_next = L + 2 at each
    limit advance): exact against the stored oracle results."""
    from paper_1705_02843_amd import instances as I
    g = _golden("c4_mixed_w4")
    if g is None:
        pytest.skip("no stored results for the 4x4 part")
    print("case: c4 4x4 part, 2048 states, batched 16-node rounds", flush=True)
    s = I.c4_mixed()[4][0]
    old = B.get_option("nodes_per_round")
    B.set_option("nodes_per_round", 16)
    try:
        rc, ln, nodes = B.solve_raw(s, 4)
    finally:
        B.set_option("nodes_per_round", old)
    assert rc == B.OK, B.strerror(rc)
    for i, r in enumerate(g["instances"]):
        m = len(r["nodes"])
        assert ln[i] == r["length"], i
        assert list(nodes[i, :m]) == r["nodes"] and not nodes[i, m:].any(), i


def test_c4_3x3_and_4x4_parts_on_the_interleaved_stack(B):
    """The 3x3 and 4x4 parts of the mixed workload in one launch on 672-entry
    stacks, where the 4x4 stack interleaves each entry's state and meta word
    and the 3x3 stack shares its LDS: exact against the stored oracle
    results of both widths."""
    from paper_1705_02843_amd import instances as I
    g3, g4 = _golden("c4_mixed_w3"), _golden("c4_mixed_w4")
    if g3 is None or g4 is None:
        pytest.skip("no stored results for the 3x3 and 4x4 parts")
    print("case: c4 3x3 + 4x4 parts, one launch, 672-entry stacks", flush=True)
    d = I.c4_mixed()
    s3, s4 = d[3][0], d[4][0]
    old = {k: B.get_option(k) for k in ("mode", "nodes_per_round", "lds_stack_capacity", "wg_size")}
    B.set_option("mode", 1)
    B.set_option("nodes_per_round", 64)
    B.set_option("wg_size", 64)
    B.set_option("lds_stack_capacity", 672)
    try:
        rc, ln, nodes = B.solve_mixed_raw(list(s3) + list(s4))
    finally:
        for k, v in old.items():
            B.set_option(k, v)
    assert rc == B.OK, B.strerror(rc)
    for off, g in ((0, g3), (len(s3), g4)):
        for i, r in enumerate(g["instances"]):
            m = len(r["nodes"])
            assert ln[off + i] == r["length"], (off, i)
            assert list(nodes[off + i, :m]) == r["nodes"] and not nodes[off + i, m:].any(), (off, i)


def test_mixed_batch_with_bad_states(B):
    """Invalid and unsolvable boards of every width inside one mixed batch:
    each gets its own status (-1 length, zero counts), the first failing code
    is returned, and every other instance is still exact."""
    from paper_1705_02843_amd import instances as I
    print("case: mixed batch with invalid and unsolvable boards", flush=True)
    d = I.c4_mixed(n3=8, n4=8, n5=1)
    s3 = list(d[3][0])
    s4 = [s for s in d[4][0] if I.manhattan_filter_value(s, 4) <= 30][:4]
    s5 = five_by_five_states(4)[:4]
    bad3 = np.arange(9, dtype=np.uint8)[[0, 2, 1, 3, 4, 5, 6, 7, 8]]   # two tiles swapped: wrong parity
    bad4 = np.zeros(16, np.uint8)                                      # not a permutation
    bad5 = np.arange(25, dtype=np.uint8)[[0, 2, 1] + list(range(3, 25))]  # two tiles swapped
    items = [bad3] + s3 + [bad4] + s4 + s5 + [bad5]
    rc, ln, nodes = B.solve_mixed_raw(items)
    assert rc in (B.EUNSOLVABLE, B.EINVAL)
    bad = {0, 1 + len(s3), len(items) - 1}
    for k in bad:
        assert ln[k] == -1 and not nodes[k].any(), k
    good = [k for k in range(len(items)) if k not in bad]
    ws = [int(round(len(items[k]) ** 0.5)) for k in good]
    for w in (3, 4, 5):
        ks = [k for k, ww in zip(good, ws) if ww == w]
        want = oracle_of([items[k] for k in ks], w)
        for j, k in enumerate(ks):
            assert ln[k] == want.length[j] and (nodes[k] == want.nodes[j]).all(), (w, k)


@pytest.mark.parametrize("depth", [0, 6])
def test_5x5_high_slack_smallest_ring_exact(B, depth):
    """5x5 instances whose final limit leaves a slack of 18-20 at the start
    state, on the smallest stack a 5x5 allows (512 wide entries).  High
    slack keeps nearly every legal move, so 64-node rounds can grow the stack
    by more than one spilled chunk per round: the spill continues until the
    next round fits, and the run stays exact with no error bit set."""
    g = _golden("c4_mixed_w5")
    assert g is not None
    pick = [r for r in g["instances"]
            if r["length"] - r["limits"][0] >= 18 and sum(r["nodes"]) < 3e7]
    assert len(pick) >= 8
    states = np.array([list(bytes.fromhex(r["state"])) for r in pick], np.uint8)
    assert states.shape == (len(pick), 25)
    B.set_option("lds_stack_capacity", 1024)
    B.set_option("nodes_per_round", 64)
    B.set_option("frontier_depth", depth)
    print("case: 5x5 high slack, ring 1024, D=%d, %d states" % (depth, len(pick)), flush=True)
    rc, ln, nodes = B.solve_raw(states, 5)
    assert rc == B.OK, B.strerror(rc)
    assert B.last_stats()["error_bits"] == 0
    for i, r in enumerate(pick):
        m = len(r["nodes"])
        assert ln[i] == r["length"], i
        assert list(nodes[i, :m]) == r["nodes"] and not nodes[i, m:].any(), i
