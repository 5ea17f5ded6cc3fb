"""Seeded synthetic sliding-tile instances (input recipe only).

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark.  It holds no part of the search method: it only draws random walks
of the blank from the goal and, where a workload asks for it, rejects walks by
the Manhattan distance of the state they end in.

Conventions (the paper's 15-puzzle, Sec. 1 and Sec. 3; the goal layout is not
stated there and is fixed here):
  * a state is a row-major ``uint8`` vector of ``w*w`` tiles, 0 is the blank;
  * the goal holds tile ``p`` at position ``p`` (so the blank sits at 0);
  * a move names the direction the blank travels: U=0 (-w), L=1 (-1),
    R=2 (+1), D=3 (+w); the inverse of move ``a`` is ``3 - a``.

Walk recipe: from the goal, at each step pick uniformly (one
``Generator.integers`` draw) among the moves that keep the blank on the board
and do not undo the previous move, taken in U, L, R, D order.  Generators are
``numpy.random.Generator(PCG64(SeedSequence(seed)))``.
"""
from __future__ import annotations

import numpy as np

MOVES = (0, 1, 2, 3)  # U, L, R, D


def goal_state(width: int) -> np.ndarray:
    return np.arange(width * width, dtype=np.uint8)


def _legal_moves(blank: int, width: int, prev: int) -> list[int]:
    r, c = divmod(blank, width)
    out = []
    for a in MOVES:
        if prev >= 0 and a == 3 - prev:
            continue
        if a == 0 and r == 0:
            continue
        if a == 1 and c == 0:
            continue
        if a == 2 and c == width - 1:
            continue
        if a == 3 and r == width - 1:
            continue
        out.append(a)
    return out


_STEP = {0: lambda w: -w, 1: lambda w: -1, 2: lambda w: 1, 3: lambda w: w}


def random_walk(rng: np.random.Generator, width: int, length: int) -> tuple[np.ndarray, list[int]]:
    """Apply ``length`` non-backtracking random blank moves to the goal."""
    s = goal_state(width).copy()
    blank = 0
    prev = -1
    moves = []
    for _ in range(length):
        cands = _legal_moves(blank, width, prev)
        a = cands[int(rng.integers(0, len(cands)))]
        n = blank + _STEP[a](width)
        s[blank], s[n] = s[n], 0
        blank = n
        prev = a
        moves.append(a)
    return s, moves


def manhattan_filter_value(state: np.ndarray, width: int) -> int:
    """Manhattan distance of ``state`` (blank excluded), used only to accept or
    reject a drawn walk for the workloads that constrain it."""
    st = np.asarray(state, dtype=np.int64).reshape(-1)
    pos = np.arange(width * width)
    tiles = st[st != 0]
    p = pos[st != 0]
    return int((np.abs(p // width - tiles // width) + np.abs(p % width - tiles % width)).sum())


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def walks_fixed(n: int, width: int, length: int, seed) -> tuple[np.ndarray, np.ndarray]:
    """``n`` states from walks of exactly ``length`` moves.  Returns
    ``(states uint8[n, w*w], walk_len int32[n])``."""
    rng = _rng(seed)
    out = np.empty((n, width * width), dtype=np.uint8)
    for i in range(n):
        out[i], _ = random_walk(rng, width, length)
    return out, np.full(n, length, dtype=np.int32)


def walks_md_window(n: int, width: int, length: int, md_lo: int, md_hi: int, seed):
    """Walks of ``length`` moves, redrawn until the end state's Manhattan
    distance lies in ``[md_lo, md_hi]``."""
    rng = _rng(seed)
    out = np.empty((n, width * width), dtype=np.uint8)
    i = 0
    while i < n:
        s, _ = random_walk(rng, width, length)
        if md_lo <= manhattan_filter_value(s, width) <= md_hi:
            out[i] = s
            i += 1
    return out, np.full(n, length, dtype=np.int32)


def walks_uniform_len(n: int, width: int, len_lo: int, len_hi: int, md_max, seed):
    """Walk length ``k ~ U{len_lo..len_hi}`` (one draw), then the walk; when
    ``md_max`` is set, a state above it is rejected and both ``k`` and the walk
    are drawn again."""
    rng = _rng(seed)
    out = np.empty((n, width * width), dtype=np.uint8)
    lens = np.empty(n, dtype=np.int32)
    i = 0
    while i < n:
        k = int(rng.integers(len_lo, len_hi + 1))
        s, _ = random_walk(rng, width, k)
        if md_max is not None and manhattan_filter_value(s, width) > md_max:
            continue
        out[i] = s
        lens[i] = k
        i += 1
    return out, lens


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------

def c1_walk40(n: int = 64, seed: int = 1):
    """64 15-puzzle states from 40-move walks."""
    return walks_fixed(n, 4, 40, seed)


def c2_md30_38(n: int = 100, seed: int = 2):
    """100 15-puzzle states from 300-move walks with Manhattan distance in
    [30, 38]: a synthetic stand-in for the paper's 100-instance benchmark set
    (Sec. 3), whose instances are not reproduced here."""
    return walks_md_window(n, 4, 300, 30, 38, seed)


def c3_uneven(n: int = 4096, seed: int = 3):
    """15-puzzle states from walks of length U{20..300}, Manhattan <= 38."""
    return walks_uniform_len(n, 4, 20, 300, 38, seed)


def c4_mixed(n3: int = 2048, n4: int = 2048, n5: int = 256, seed: int = 4):
    """Mixed widths: 3x3 and 4x4 from walks of length U{20..300} (4x4 with
    Manhattan <= 38), 5x5 from 60-move walks.  One child seed per width."""
    s3, s4, s5 = np.random.SeedSequence(seed).spawn(3)
    return {
        3: walks_uniform_len(n3, 3, 20, 300, None, s3),
        4: walks_uniform_len(n4, 4, 20, 300, 38, s4),
        5: walks_fixed(n5, 5, 60, s5),
    }


def c5_poisson(n: int = 4000, rate_hz: float = 200.0, seed: int = 5):
    """Request stream: exponential inter-arrival times (mean 1/rate) and
    instances drawn as in ``c3_uneven``.  Returns (arrival_s float64[n],
    states, walk_len)."""
    ss_t, ss_i = np.random.SeedSequence(seed).spawn(2)
    gaps = _rng(ss_t).exponential(1.0 / rate_hz, size=n)
    states, lens = walks_uniform_len(n, 4, 20, 300, 38, ss_i)
    return np.cumsum(gaps), states, lens


WORKLOADS = {
    "c1_walk40": c1_walk40,
    "c2_md30_38": c2_md30_38,
    "c3_uneven": c3_uneven,
}
