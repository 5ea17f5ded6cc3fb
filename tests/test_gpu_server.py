"""Continuous batching: requests submitted while others are being searched.

Every answer must equal the oracle's result for that state alone (exact
integers: length and every per-limit node count), whatever else was in
flight; invalid requests get their status; a full request ring reports
EAGAIN and recovers once answers are collected.
"""
import json
import os
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    g = json.load(open(os.path.join(GOLDEN, name + ".json")))
    states = np.array([[int(c, 16) for c in rec["state"]] for rec in g["instances"]], np.uint8)
    length = np.array([rec["length"] for rec in g["instances"]], np.int32)
    nodes = np.zeros((len(g["instances"]), 64), np.uint64)
    for i, rec in enumerate(g["instances"]):
        nodes[i, :len(rec["nodes"])] = rec["nodes"]
    return states, length, nodes


@pytest.fixture
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_1705_02843_amd import bpida
    saved = {k: bpida.get_option(k) for k in ("budget_ms", "frontier_depth")}
    bpida.set_option("budget_ms", 90000)
    yield bpida
    for k, v in saved.items():
        bpida.set_option(k, v)


def drain(srv, pending, got, deadline):
    while pending and time.time() < deadline:
        for t in list(pending):
            r = srv.poll(t)
            if r is not None:
                got[pending.pop(t)] = r
        time.sleep(0.0005)


def test_mixed_stream_answers_equal_alone_results(B):
    print("case: server, 64 + 24 golden states and 2 bad ones, random gaps", flush=True)
    s1, l1, n1 = load_golden("c1_walk40")
    s2, l2, n2 = load_golden("c2_md30_38")
    pick = [0, 3, 7, 12, 18, 25, 31, 44, 50, 63, 66, 70, 75, 80, 88, 91, 95, 99, 5, 9, 14, 21,
            40, 57]
    states = np.concatenate([s1, s2[pick]])
    want_len = np.concatenate([l1, l2[pick]])
    want_nodes = np.concatenate([n1, n2[pick]])
    bad_perm = s1[0].copy()
    bad_perm[1], bad_perm[2] = bad_perm[2], bad_perm[1]
    bad_dup = s1[1].copy()
    bad_dup[0] = bad_dup[3]
    rng = np.random.default_rng(0)
    order = rng.permutation(len(states))
    got, pending = {}, {}
    with B.Server(max_inflight=64, ring_capacity=256) as srv:
        t_bad1 = srv.submit(bad_perm)
        for k in order:
            t = srv.submit(states[k])
            assert t is not None
            pending[t] = int(k)
            time.sleep(float(rng.exponential(0.002)))  # arrivals overlap running work
            for tt in list(pending):
                r = srv.poll(tt)
                if r is not None:
                    got[pending.pop(tt)] = r
        t_bad2 = srv.submit(bad_dup)
        drain(srv, pending, got, time.time() + 60)
        rb1, rb2 = None, None
        deadline = time.time() + 30
        while (rb1 is None or rb2 is None) and time.time() < deadline:
            rb1 = rb1 or srv.poll(t_bad1)
            rb2 = rb2 or srv.poll(t_bad2)
            time.sleep(0.001)
        rc = srv.stop()
    assert rc == B.OK, B.strerror(rc)
    assert not pending and len(got) == len(states)
    for k in range(len(states)):
        ln, nodes, status = got[k]
        assert status == 1, (k, status)
        assert ln == want_len[k] and (nodes == want_nodes[k]).all(), k
    assert rb1[2] == B.EUNSOLVABLE and rb1[0] == -1
    assert rb2[2] == B.EINVAL and rb2[0] == -1
    print("server stats: %s" % B.last_stats(), flush=True)


def test_full_ring_reports_eagain_and_recovers(B):
    print("case: server ring of 64 requests, 100 submitted without collecting", flush=True)
    s1, l1, n1 = load_golden("c1_walk40")
    with B.Server(max_inflight=16, ring_capacity=64) as srv:
        tickets = []
        refused = 0
        for i in range(100):
            t = srv.submit(s1[i % 64])
            if t is None:
                refused += 1
            else:
                tickets.append((t, i % 64))
        assert refused > 0 and len(tickets) == 64
        res = {}
        deadline = time.time() + 60
        while len(res) < len(tickets) and time.time() < deadline:
            for t, k in tickets:
                if t not in res:
                    r = srv.poll(t)
                    if r is not None:
                        res[t] = (k, r)
            time.sleep(0.0005)
        assert len(res) == len(tickets)
        t2 = srv.submit(s1[5])
        assert t2 is not None
        r2 = None
        deadline = time.time() + 30
        while r2 is None and time.time() < deadline:
            r2 = srv.poll(t2)
        assert srv.stop() == B.OK
    for t, (k, r) in res.items():
        assert r is not None and r[2] == 1 and r[0] == l1[k] and (r[1] == n1[k]).all()
    assert r2[0] == l1[5] and (r2[1] == n1[5]).all()


def test_first_limit_past_the_output_columns_answers_elimit(B):
    """A first limit whose output column is past the 64 per request (a start
    threshold far above h0) is answered BPIDA_ELIMIT with no counts, as the
    batched solve answers it, and the server keeps serving."""
    print("case: server with start_threshold 250, 4 c1 states", flush=True)
    s1, l1, n1 = load_golden("c1_walk40")
    old = B.get_option("start_threshold")
    B.set_option("start_threshold", 250)
    try:
        with B.Server(max_inflight=16, ring_capacity=64) as srv:
            pending = {srv.submit(s1[i]): i for i in range(4)}
            assert None not in pending
            got = {}
            drain(srv, pending, got, time.time() + 60)
            assert srv.stop() == B.OK
        rc, ln, _ = B.solve_raw(s1[:4])
    finally:
        B.set_option("start_threshold", old)
    assert len(got) == 4
    for i in range(4):
        length, nodes, status = got[i]
        assert status == B.ELIMIT and length == -1 and not nodes.any(), (i, status, length)
    assert rc == B.ELIMIT and (ln == -1).all()


def test_queue_overflow_answers_enomem_never_wrong_counts(B):
    print("case: server with a 64-slot queue, a 1-poll push wait and one searching "
          "workgroup, 64 + 12 golden states", flush=True)
    s1, l1, n1 = load_golden("c1_walk40")
    s2, l2, n2 = load_golden("c2_md30_38")
    # the 12 smallest of c2 (at most 4.1e6 nodes each): one workgroup searches them
    pick = [39, 77, 26, 96, 17, 44, 30, 84, 35, 36, 70, 66]
    states = np.concatenate([s1, s2[pick]])
    want_len = np.concatenate([l1, l2[pick]])
    want_nodes = np.concatenate([n1, n2[pick]])
    saved = {k: B.get_option(k) for k in ("queue_capacity", "push_spin", "max_workgroups",
                                          "admit_backlog")}
    B.set_option("queue_capacity", 64)
    B.set_option("push_spin", 1)
    B.set_option("max_workgroups", 2)  # the admitter and one searcher
    B.set_option("admit_backlog", 0)  # no frontier budget: admit whatever the queue holds
    got, pending = {}, {}
    try:
        with B.Server(max_inflight=64, ring_capacity=256) as srv:
            for k in range(len(states)):
                t = srv.submit(states[k])
                assert t is not None
                pending[t] = k
            drain(srv, pending, got, time.time() + 60)
            rc = srv.stop()
    finally:
        for k, v in saved.items():
            B.set_option(k, v)
    assert not pending and len(got) == len(states)
    lost = 0
    for k in range(len(states)):
        ln, nodes, status = got[k]
        if status == B.ENOMEM:
            lost += 1
            assert ln == -1, k
            continue
        assert status == 1, (k, status)
        assert ln == want_len[k] and (nodes == want_nodes[k]).all(), k
    print("answers lost to the full queue: %d of %d; stop rc %d" % (lost, len(states), rc),
          flush=True)
    assert lost > 0 and rc == B.ENOMEM
    # a fresh server with the default queue answers every request exactly
    with B.Server(max_inflight=16, ring_capacity=64) as srv:
        t = srv.submit(s1[7])
        r = None
        deadline = time.time() + 30
        while r is None and time.time() < deadline:
            r = srv.poll(t)
        assert srv.stop() == B.OK
    assert r is not None and r[2] == 1 and r[0] == l1[7] and (r[1] == n1[7]).all()


def test_frontier_budget_keeps_a_small_queue_from_overflowing(B):
    """The same burst into a small queue (256 chunks) and few workgroups, with
    the admission's HBM frontier budget on (half the queue): requests wait to
    be admitted instead of overflowing it, and every answer is exact."""
    print("case: server, 256-chunk queue, 8 workgroups, frontier budget, 64 + 12 states",
          flush=True)
    s1, l1, n1 = load_golden("c1_walk40")
    s2, l2, n2 = load_golden("c2_md30_38")
    pick = [39, 77, 26, 96, 17, 44, 30, 84, 35, 36, 70, 66]
    states = np.concatenate([s1, s2[pick]])
    want_len = np.concatenate([l1, l2[pick]])
    want_nodes = np.concatenate([n1, n2[pick]])
    saved = {k: B.get_option(k) for k in ("queue_capacity", "max_workgroups", "admit_backlog")}
    B.set_option("queue_capacity", 256)
    B.set_option("max_workgroups", 8)
    B.set_option("admit_backlog", -1)
    got, pending = {}, {}
    try:
        with B.Server(max_inflight=64, ring_capacity=256) as srv:
            for k in range(len(states)):
                t = srv.submit(states[k])
                assert t is not None
                pending[t] = k
            drain(srv, pending, got, time.time() + 60)
            rc = srv.stop()
    finally:
        for k, v in saved.items():
            B.set_option(k, v)
    assert rc == B.OK, B.strerror(rc)
    assert not pending and len(got) == len(states)
    for k in range(len(states)):
        ln, nodes, status = got[k]
        assert status == 1 and ln == want_len[k] and (nodes == want_nodes[k]).all(), k


def test_poisson_stream_of_c3_states_equals_the_oracle(B):
    """512 states of the 4096-state uneven workload arriving as a Poisson
    stream at 2000 requests per second (10 times the serving workload's
    rate): every answer equals the stored oracle result for that state."""
    print("case: server, Poisson stream of 512 c3_uneven states at 2000/s", flush=True)
    states, want_len, want_nodes = load_golden("c3_uneven")
    rng = np.random.default_rng(55)
    order = rng.permutation(states.shape[0])[:512]
    gaps = rng.exponential(1.0 / 2000.0, size=order.size)
    arrivals = np.cumsum(gaps)
    got, pending = {}, {}
    with B.Server(max_inflight=256, ring_capacity=1024) as srv:
        t0 = time.time()
        k = 0
        while k < order.size:
            if time.time() - t0 >= arrivals[k]:
                t = srv.submit(states[order[k]])
                if t is None:
                    time.sleep(0.0002)
                else:
                    pending[t] = int(order[k])
                    k += 1
            for tt in list(pending):
                r = srv.poll(tt)
                if r is not None:
                    got[pending.pop(tt)] = r
        drain(srv, pending, got, time.time() + 60)
        rc = srv.stop()
    assert rc == B.OK, B.strerror(rc)
    assert not pending and len(got) == order.size
    for i, (ln, nodes, status) in got.items():
        assert status == 1 and ln == want_len[i] and (nodes == want_nodes[i]).all(), i
