"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_1705_02843_amd import bpida
    return bpida


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(bpida_[a-z_0-9]+)\s*\(",
                                text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(B):
    names = declared_functions()
    assert "bpida_solve" in names and "bpida_solve_device" in names
    for nm in names:
        assert hasattr(B.lib, nm), nm
    assert set(B.EXPORTS) == set(names)


def test_argument_errors_before_device_work(B):
    P = ctypes.POINTER
    st = np.zeros(16, np.uint8)
    ln = np.zeros(1, np.int32)
    nd = np.zeros(64, np.uint64)
    sp = st.ctypes.data_as(P(ctypes.c_uint8))
    lp = ln.ctypes.data_as(P(ctypes.c_int32))
    npp = nd.ctypes.data_as(P(ctypes.c_uint64))
    assert B.lib.bpida_solve(None, 1, 4, lp, npp) == B.EINVAL
    assert B.lib.bpida_solve(sp, 1, 4, None, npp) == B.EINVAL
    assert B.lib.bpida_solve(sp, 1, 4, lp, None) == B.EINVAL
    assert B.lib.bpida_solve(sp, -1, 4, lp, npp) == B.EINVAL
    assert B.lib.bpida_solve(sp, 1, 7, lp, npp) == B.EINVAL
    assert B.lib.bpida_solve(sp, 0, 4, lp, npp) == B.OK  # empty batch: nothing to do
    assert B.lib.bpida_solve_device(None, 1, 4, None, None, None) == B.EINVAL
    assert B.lib.bpida_solve_device(ctypes.c_void_p(8), 0, 4, ctypes.c_void_p(8),
                                    ctypes.c_void_p(8), None) == B.OK
    wd = np.array([4], np.int32)
    wp = wd.ctypes.data_as(P(ctypes.c_int32))
    bad = np.array([6], np.int32).ctypes.data_as(P(ctypes.c_int32))
    assert B.lib.bpida_solve_mixed(sp, None, 1, lp, npp) == B.EINVAL
    assert B.lib.bpida_solve_mixed(sp, bad, 1, lp, npp) == B.EINVAL
    assert B.lib.bpida_solve_mixed(sp, wp, 0, lp, npp) == B.OK
    assert B.lib.bpida_solve_mixed_device(None, wp, 1, ctypes.c_void_p(8), ctypes.c_void_p(8),
                                          None) == B.EINVAL
    assert B.lib.bpida_solve_mixed_device(ctypes.c_void_p(8), bad, 1, ctypes.c_void_p(8),
                                          ctypes.c_void_p(8), None) == B.EINVAL
    assert B.lib.bpida_solve_mixed_device(ctypes.c_void_p(8), wp, 0, ctypes.c_void_p(8),
                                          ctypes.c_void_p(8), None) == B.OK
    pp = np.zeros(256, np.uint8).ctypes.data_as(P(ctypes.c_uint8))
    assert B.lib.bpida_solve_paths(sp, 1, 4, lp, npp, None) == B.EINVAL
    assert B.lib.bpida_solve_paths(None, 1, 4, lp, npp, pp) == B.EINVAL
    assert B.lib.bpida_solve_paths(sp, 1, 2, lp, npp, pp) == B.EINVAL
    assert B.lib.bpida_solve_paths(sp, 0, 4, lp, npp, pp) == B.OK
    v8 = ctypes.c_void_p(8)
    assert B.lib.bpida_solve_paths_device(v8, 1, 4, v8, v8, None, None) == B.EINVAL
    assert B.lib.bpida_solve_paths_device(v8, 0, 4, v8, v8, v8, None) == B.OK
    for fn in (B.lib.bpida_solve_device_async, B.lib.bpida_solve_device_noalloc):
        v = ctypes.c_void_p(8)
        assert fn(None, 1, 4, v, v, v, None) == B.EINVAL
        assert fn(v, 1, 4, v, v, None, None) == B.EINVAL
        assert fn(v, -1, 4, v, v, v, None) == B.EINVAL
        assert fn(v, 1, 6, v, v, v, None) == B.EINVAL
        assert fn(v, 0, 4, v, v, v, None) == B.OK
    assert (ln == 0).all() and (nd == 0).all()  # outputs untouched


def test_options_roundtrip_and_validation(B):
    old = B.get_option("frontier_depth")
    B.set_option("frontier_depth", 6)
    assert B.get_option("frontier_depth") == 6
    B.set_option("frontier_depth", old)
    for k, v in (("frontier_depth", 17), ("frontier_depth", -2), ("lds_stack_capacity", 300), ("mode", 2), ("nodes_per_round", 32),
                 ("queue_capacity", -1), ("watchdog_ms", 0),
                 ("spill_capacity", 65), ("max_threshold", -2), ("donate_every", 48),
                 ("donate_every", 2), ("donate_min", 0), ("donate_min", 4096), ("queue_chunk", 48), ("start_threshold", -2), ("seed_chunk", 12), ("seed_chunk", -1),
                 ("static_lb", 2), ("first_solution", 2), ("wg_size", 96), ("wg_size", 512),
                 ("plain_nodes_per_round", 32), ("push_spin", 0), ("no_such_key", 1)):
        with pytest.raises(B.BpidaError):
            B.set_option(k, v)
    assert B.get_option("no_such_key") == -(2 ** 63)
    assert B.get_option("donate_every") == 128 and B.get_option("donate_min") == -1
    # the non-power-of-two stacks of the batched 64-node round
    old_cap = B.get_option("lds_stack_capacity")
    for cap in (640, 672, 768):
        B.set_option("lds_stack_capacity", cap)
        assert B.get_option("lds_stack_capacity") == cap
    for cap in (560, 639, 700, 896):
        with pytest.raises(B.BpidaError):
            B.set_option("lds_stack_capacity", cap)
    B.set_option("lds_stack_capacity", old_cap)


def test_strerror_covers_codes(B):
    texts = {B.strerror(c) for c in (0, -1, -2, -3, -4, -5, -6)}
    assert len(texts) == 7 and B.strerror(-99) == "unknown status"


def test_last_stats_shape(B):
    s = B.last_stats()
    assert set(s) >= {"rounds", "search_nodes", "spilled", "launches", "search_us"}


def test_mixed_binding_rejects_non_square_states(B):
    import numpy as np
    with pytest.raises(ValueError):
        B.solve_mixed_raw([np.arange(9, dtype=np.uint8), np.arange(10, dtype=np.uint8)])


def test_one_hip_runtime_whatever_the_import_order():
    """The binding loads torch before the library, so the process maps one
    HIP runtime (torch's) even when the binding is imported first."""
    import subprocess
    import sys
    code = ("from paper_1705_02843_amd import bpida\n"
            "import torch\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "print(len(set(l.split()[-1] for l in m if 'libamdhip64' in l)))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
