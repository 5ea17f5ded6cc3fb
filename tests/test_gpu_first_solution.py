"""First-solution mode (Alg. 1 returns at its first goal) on the GPU.

Its final-iteration count depends on which workgroup reaches a goal first,
so it is not unique; what is: the optimal length and every earlier
iteration's count (stored oracle results, all-solutions mode).  The final
count must lie between the L + 1 nodes of a path to the goal and the
all-solutions count of that iteration.
"""
import numpy as np
import pytest

from test_gpu_parity import B, MODES, _say, load_golden, opts, set_mode  # noqa: F401

pytestmark = pytest.mark.gpu


def check_first_solution(got_len, got_nodes, length, nodes, tag):
    n = len(length)
    assert (got_len == length).all(), tag
    stopped_early = 0
    for i in range(n):
        k = int(np.count_nonzero(nodes[i]))
        assert (got_nodes[i, :k - 1] == nodes[i, :k - 1]).all(), (tag, i)
        assert not got_nodes[i, k:].any(), (tag, i)
        fin = int(got_nodes[i, k - 1])
        assert int(length[i]) + 1 <= fin <= int(nodes[i, k - 1]), (tag, i, fin, int(nodes[i, k - 1]))
        stopped_early += fin < int(nodes[i, k - 1])
    return stopped_early


@pytest.mark.parametrize("mode", sorted(MODES))
def test_first_solution_c1(opts, mode):
    B = opts
    _say("case: first solution, c1_walk40, %s" % mode)
    set_mode(B, mode)
    B.set_option("first_solution", 1)
    try:
        states, length, nodes = load_golden("c1_walk40")
        rc, ln, got = B.solve_raw(states)
    finally:
        B.set_option("first_solution", 0)
    assert rc == B.OK, B.strerror(rc)
    check_first_solution(ln, got, length, nodes, mode)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_first_solution_c2_stops_early(opts, mode):
    B = opts
    _say("case: first solution, c2_md30_38 (first 40 states), %s" % mode)
    set_mode(B, mode)
    states, length, nodes = load_golden("c2_md30_38")
    states, length, nodes = states[:40], length[:40], nodes[:40]
    B.set_option("first_solution", 1)
    try:
        rc, ln, got = B.solve_raw(states)
    finally:
        B.set_option("first_solution", 0)
    assert rc == B.OK, B.strerror(rc)
    early = check_first_solution(ln, got, length, nodes, mode)
    assert early >= 20, early  # most instances stop well before the end
    # and all-solutions mode afterwards is exact again
    rc, ln, got = B.solve_raw(states)
    assert rc == B.OK and (ln == length).all() and (got == nodes).all()


def test_first_solution_mixed_widths(opts):
    B = opts
    from oracle import oracle
    from paper_1705_02843_amd import instances as I
    _say("case: first solution, mixed 3x3 / 4x4 batch")
    d = I.c4_mixed(n3=64, n4=16, n5=1)
    s3, s4 = list(d[3][0]), [s for s in d[4][0] if I.manhattan_filter_value(s, 4) <= 30][:8]
    a3, a4 = oracle.solve(np.stack(s3), 3, nthreads=8), oracle.solve(np.stack(s4), 4, nthreads=8)
    B.set_option("first_solution", 1)
    try:
        rc, ln, got = B.solve_mixed_raw(s3 + s4)
    finally:
        B.set_option("first_solution", 0)
    assert rc == B.OK, B.strerror(rc)
    check_first_solution(ln[:64], got[:64], a3.length, a3.nodes, "3x3")
    check_first_solution(ln[64:], got[64:], a4.length, a4.nodes, "4x4")


def test_first_solution_plain_with_static_lb(opts):
    B = opts
    _say("case: first solution, plain with static load balancing, c2_md30_38 (first 20)")
    set_mode(B, "plain")
    B.set_option("static_lb", 1)
    states, length, nodes = load_golden("c2_md30_38")
    B.set_option("first_solution", 1)
    try:
        rc, ln, got = B.solve_raw(states[:20])
    finally:
        B.set_option("first_solution", 0)
    assert rc == B.OK, B.strerror(rc)
    check_first_solution(ln, got, length[:20], nodes[:20], "plain+lb")
