"""The seeded instance generator: determinism and the workload recipes."""
import json
import os

import numpy as np

import puzzle_ref as P
from paper_1705_02843_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_walks_are_deterministic_and_non_backtracking():
    a = np.random.Generator(np.random.PCG64(np.random.SeedSequence(9)))
    b = np.random.Generator(np.random.PCG64(np.random.SeedSequence(9)))
    for w in (3, 4, 5):
        s1, m1 = I.random_walk(a, w, 50)
        s2, m2 = I.random_walk(b, w, 50)
        assert (s1 == s2).all() and m1 == m2
        assert all(m1[i + 1] != 3 - m1[i] for i in range(len(m1) - 1))
        assert tuple(int(x) for x in s1) == P.random_state_at(w, m1)
        assert sorted(s1.tolist()) == list(range(w * w))


def test_workload_shapes_and_filters():
    s, l = I.c1_walk40()
    assert s.shape == (64, 16) and s.dtype == np.uint8 and (l == 40).all()
    s2, _ = I.c2_md30_38()
    assert s2.shape == (100, 16)
    md = [P.manhattan(tuple(x), 4) for x in s2]
    assert min(md) >= 30 and max(md) <= 38
    s3, l3 = I.walks_uniform_len(200, 4, 20, 300, 38, 3)
    assert (l3 >= 20).all() and (l3 <= 300).all()
    assert max(P.manhattan(tuple(x), 4) for x in s3) <= 38


def test_goldens_match_generator_bytes():
    for name, make in (("c1_walk40", I.c1_walk40), ("c2_md30_38", I.c2_md30_38)):
        path = os.path.join(GOLDEN, name + ".json")
        g = json.load(open(path))
        states, _ = make()
        assert g["n"] == states.shape[0]
        for rec, st in zip(g["instances"], states):
            assert rec["state"] == "".join("%x" % v for v in st)


def test_poisson_stream_is_sorted():
    t, s, l = I.c5_poisson(n=50)
    assert (np.diff(t) > 0).all() and s.shape == (50, 16)
