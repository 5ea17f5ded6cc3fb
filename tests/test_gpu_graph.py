"""The batched solve recorded into a HIP graph and replayed.

bpida_solve_device_async enqueues the whole batched solve without host
synchronisation.  The graph is replayed several times with eager work and
synchronisations in between; every replay must reproduce the stored oracle
results (the set-up kernels re-initialise all device state on each replay).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    g = json.load(open(os.path.join(GOLDEN, name + ".json")))
    states = np.array([[int(c, 16) for c in rec["state"]] for rec in g["instances"]], np.uint8)
    n = len(g["instances"])
    length = np.array([rec["length"] for rec in g["instances"]], np.int32)
    nodes = np.zeros((n, 64), np.uint64)
    for i, rec in enumerate(g["instances"]):
        nodes[i, :len(rec["nodes"])] = rec["nodes"]
    return states, length, nodes


def test_async_matches_golden_and_replays_in_a_graph():
    import torch
    from paper_1705_02843_amd import bpida as B

    print("case: async batched solve of c1_walk40, then a captured graph replayed 3 times",
          flush=True)
    states, want_len, want_nodes = load_golden("c1_walk40")
    n = states.shape[0]
    d_states = torch.from_numpy(states).cuda()
    d_len = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    d_nodes = torch.zeros((n, 64), dtype=torch.int64, device="cuda")
    d_status = torch.zeros(n, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rc = B.solve_device_async(d_states, d_len, d_nodes, d_status, stream=s)
    s.synchronize()
    assert rc == B.OK
    assert (d_status.cpu().numpy() == 1).all()
    np.testing.assert_array_equal(d_len.cpu().numpy(), want_len)
    np.testing.assert_array_equal(d_nodes.cpu().numpy().view(np.uint64), want_nodes)

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rc = B.solve_device_async(d_states, d_len, d_nodes, d_status,
                                  stream=torch.cuda.current_stream())
    assert rc == B.OK
    for rep in range(3):
        d_len.fill_(-9)
        d_nodes.fill_(7)
        d_status.fill_(0)
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (d_status.cpu().numpy() == 1).all(), rep
        np.testing.assert_array_equal(d_len.cpu().numpy(), want_len)
        np.testing.assert_array_equal(d_nodes.cpu().numpy().view(np.uint64), want_nodes)
        del junk


def test_async_reports_per_instance_status():
    import torch
    from paper_1705_02843_amd import bpida as B

    print("case: async solve with an unsolvable and an invalid state", flush=True)
    states, want_len, want_nodes = load_golden("c1_walk40")
    st = states[:4].copy()
    st[1, 1], st[1, 2] = st[1, 2], st[1, 1]
    st[2, 0] = st[2, 3]
    d_states = torch.from_numpy(st).cuda()
    d_len = torch.empty(4, dtype=torch.int32, device="cuda")
    d_nodes = torch.empty((4, 64), dtype=torch.int64, device="cuda")
    d_status = torch.empty(4, dtype=torch.int32, device="cuda")
    rc = B.solve_device_async(d_states, d_len, d_nodes, d_status)
    torch.cuda.synchronize()
    assert rc == B.OK
    assert d_status.cpu().tolist() == [1, B.EUNSOLVABLE, B.EINVAL, 1]
    ln = d_len.cpu().numpy()
    assert ln[0] == want_len[0] and ln[3] == want_len[3] and ln[1] == -1 and ln[2] == -1
