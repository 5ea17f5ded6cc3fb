"""Small, independent sliding-tile helpers used by the tests to pin the oracle.

Nothing here is shared with the oracle or the GPU library: these are separate
graph algorithms (breadth-first search, a layered path-count recurrence) that
fix the values the oracle must reproduce.  Conventions: row-major tuples of
``w*w`` tiles, 0 is the blank, goal = tile p at position p; moves U, L, R, D =
0..3 name the blank's direction, inverse 3 - a.
"""
from __future__ import annotations

from collections import defaultdict, deque

import numpy as np


def goal(w: int) -> tuple:
    return tuple(range(w * w))


def neighbours(state: tuple, w: int):
    """Yield (move, child) for every move that keeps the blank on the board."""
    b = state.index(0)
    r, c = divmod(b, w)
    for a, ok, d in ((0, r > 0, -w), (1, c > 0, -1), (2, c < w - 1, 1), (3, r < w - 1, w)):
        if ok:
            n = b + d
            s = list(state)
            s[b], s[n] = s[n], 0
            yield a, tuple(s)


def manhattan(state, w: int) -> int:
    h = 0
    for p, t in enumerate(state):
        t = int(t)
        if t:
            h += abs(p // w - t // w) + abs(p % w - t % w)
    return h


def bfs_distances(w: int, max_depth: int | None = None) -> dict:
    """Exact shortest distances from the goal (the move graph is undirected)."""
    g = goal(w)
    dist = {g: 0}
    q = deque([g])
    while q:
        s = q.popleft()
        d = dist[s]
        if max_depth is not None and d >= max_depth:
            continue
        for _, c in neighbours(s, w):
            if c not in dist:
                dist[c] = d + 1
                q.append(c)
    return dist


def inversion_parity(state) -> int:
    s = list(state)
    inv = 0
    for i in range(len(s)):
        for j in range(i + 1, len(s)):
            if s[i] > s[j]:
                inv ^= 1
    return inv


def layered_path_count(start: tuple, w: int, limit: int) -> int:
    """Number of non-backtracking move sequences from ``start`` whose every
    prefix ends in a node with depth + Manhattan <= ``limit``, counted by a
    layer-by-layer recurrence over (state, last move) with multiplicities.
    This is the number of nodes an f-limited DFS with parent pruning expands
    when it never stops early."""
    layer = {(start, -1): 1}
    total = 0
    d = 0
    while layer:
        nxt = defaultdict(int)
        for (s, last), mult in layer.items():
            if d + manhattan(s, w) > limit:
                continue
            total += mult
            for a, c in neighbours(s, w):
                if last >= 0 and a == 3 - last:
                    continue
                nxt[(c, a)] += mult
        layer = nxt
        d += 1
    return total


def random_state_at(w: int, moves: list[int]) -> tuple:
    s = goal(w)
    for a in moves:
        for aa, c in neighbours(s, w):
            if aa == a:
                s = c
                break
        else:
            raise ValueError("illegal move")
    return s


def as_array(states) -> np.ndarray:
    return np.asarray(list(states), dtype=np.uint8)


def first_shortest_moves(state: tuple, w: int, dist: dict) -> list:
    """The lexicographically smallest shortest move sequence from ``state`` to
    the goal, from exact distances: at each step the first move (U, L, R, D)
    whose child is one step closer.  Every state on a shortest path from a
    state at distance d is within distance d, so a bounded BFS suffices."""
    out = []
    s = state
    d = dist[s]
    while d > 0:
        for a, c in neighbours(s, w):
            if dist.get(c) == d - 1:
                out.append(a)
                s, d = c, d - 1
                break
        else:
            raise ValueError("no step closer: distances are not exact")
    return out


def replay(state: tuple, w: int, moves) -> tuple:
    """Apply blank moves to a state; raises on a move off the board."""
    s = state
    for a in moves:
        for aa, c in neighbours(s, w):
            if aa == int(a):
                s = c
                break
        else:
            raise ValueError("illegal move %d" % int(a))
    return s
