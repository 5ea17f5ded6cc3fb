"""Python loader for the CPU IDA* oracle (``ida_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.

``build()`` compiles ``ida_oracle.c`` with gcc into ``libida_oracle.so`` next
to it; ``solve()`` runs the oracle over a batch of states.  The arithmetic is
all in the C file (sequential IDA* with the Manhattan distance heuristic, the
final f-limit run to completion; see its header for the readings of the
paper it follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

MAX_ITERS = 64
MAX_PATH = 256
OK, EINVAL, EUNSOLVABLE, ELIMIT, EHCHECK = 0, -1, -2, -3, -4

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ida_oracle.c")
_LIB = os.path.join(_HERE, "libida_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, gcc -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.POINTER
        lib.oracle_solve.argtypes = [p(ctypes.c_uint8), ctypes.c_int32, ctypes.c_int32,
                                     p(ctypes.c_int32), p(ctypes.c_int32), p(ctypes.c_uint64),
                                     p(ctypes.c_int32), p(ctypes.c_int32), ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_solve.restype = ctypes.c_int32
        lib.oracle_solve_paths.argtypes = lib.oracle_solve.argtypes + [p(ctypes.c_uint8)]
        lib.oracle_solve_paths.restype = ctypes.c_int32
        lib.oracle_check_state.argtypes = [p(ctypes.c_uint8), ctypes.c_int32]
        lib.oracle_check_state.restype = ctypes.c_int32
        lib.oracle_manhattan.argtypes = [p(ctypes.c_uint8), ctypes.c_int32]
        lib.oracle_manhattan.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class OracleResult:
    rc: int
    length: np.ndarray   # int32[n], -1 on error
    limits: np.ndarray   # int32[n, 64]
    nodes: np.ndarray    # uint64[n, 64]
    niter: np.ndarray    # int32[n]
    status: np.ndarray   # int32[n]
    path: np.ndarray | None = None  # uint8[n, 256]: moves U, L, R, D = 0..3, 0xFF after

    @property
    def total_nodes(self) -> int:
        return int(self.nodes.sum(dtype=np.uint64))


def solve(states, width: int, nthreads: int = 1, check: bool = False,
          max_limit: int = -1, first_solution: bool = False,
          with_path: bool = False) -> OracleResult:
    """IDA* per instance (all optimal solutions in the final iteration, or
    with ``first_solution`` stopping at its first goal, as Alg. 1 returns).
    ``with_path``: also the moves to the first goal expanded (the
    lexicographically smallest optimal move sequence)."""
    lib = _load()
    st = np.ascontiguousarray(np.asarray(states, dtype=np.uint8).reshape(-1, width * width))
    n = st.shape[0]
    length = np.empty(n, np.int32)
    limits = np.zeros((n, MAX_ITERS), np.int32)
    nodes = np.zeros((n, MAX_ITERS), np.uint64)
    niter = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    path = np.full((n, MAX_PATH), 0xFF, np.uint8) if with_path else None
    if n == 0:
        return OracleResult(OK, length, limits, nodes, niter, status, path)
    rc = lib.oracle_solve_paths(_ptr(st, ctypes.c_uint8), n, width, _ptr(length, ctypes.c_int32),
                                _ptr(limits, ctypes.c_int32), _ptr(nodes, ctypes.c_uint64),
                                _ptr(niter, ctypes.c_int32), _ptr(status, ctypes.c_int32),
                                int(nthreads), int(bool(check)), int(max_limit),
                                int(bool(first_solution)),
                                _ptr(path, ctypes.c_uint8) if with_path else None)
    return OracleResult(int(rc), length, limits, nodes, niter, status, path)


def check_state(state, width: int) -> int:
    st = np.ascontiguousarray(np.asarray(state, dtype=np.uint8).reshape(-1))
    return int(_load().oracle_check_state(_ptr(st, ctypes.c_uint8), width))


def manhattan(state, width: int) -> int:
    st = np.ascontiguousarray(np.asarray(state, dtype=np.uint8).reshape(-1))
    return int(_load().oracle_manhattan(_ptr(st, ctypes.c_uint8), width))
