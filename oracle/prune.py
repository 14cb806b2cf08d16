"""Exact search-space reduction by tile (partition) bounds: definitions.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline); the
GPU library never imports this module.

Section 6 proposes computing only the partitions where an optimal alignment
can lie.  The reading built here keeps that exact with the pairwise bound of
Carrillo and Lipman (1988): for the sum-of-pairs score with a linear gap and
gap-gap columns scoring 0, the score of a k-alignment is the sum over pairs
i < j of the scores of its projections on (i, j), so for any alignment
through cell v

    SP <= B(v) = sum_{i<j} ( P_ij[v_i, v_j] + Q_ij[v_i, v_j] )

where P_ij[a, b] is the optimal pairwise score of the prefixes s_i[:a],
s_j[:b] and Q_ij[a, b] that of the suffixes s_i[a:], s_j[b:].  A cell with
B(v) < L for a lower bound L <= optimum lies on no optimal alignment.

Tiles follow the device grid: along dimension i tile 0 holds the cell
v_i = 0 and tile c >= 1 holds v_i in [(c-1)T + 1, min(cT, n_i)].  A tile is
kept when sum_{i<j} max over its (v_i, v_j) block of (P_ij + Q_ij) >= L, an
upper bound of max B over the tile.

Thresholds.  U = sum_{i<j} P_ij[n_i, n_j] bounds the optimum from above.  The
first pass uses L1 = U - ceil(|U| / 16) - C(k, 2) * cmax (cmax = max(|gap|,
max |sub|)), a guess; a pass whose end score s reaches its threshold is exact
(s <= optimum always, and L <= optimum keeps every optimal cell).  Otherwise
the second pass uses L2 = s when s is the score of a real path (s >= the
closed-form lower bound of every score), else no pruning.
"""
from __future__ import annotations

import itertools

import numpy as np

from .oracle import oracle_fill


def pair_tables(seqs, sub, gap):
    """{(i, j): (P, Q)} for i < j: prefix and suffix optimal pairwise scores,
    int64 arrays of shape (n_i + 1, n_j + 1)."""
    out = {}
    for i, j in itertools.combinations(range(len(seqs)), 2):
        a = np.asarray(seqs[i], np.uint8)
        b = np.asarray(seqs[j], np.uint8)
        P, _ = oracle_fill([a, b], sub, gap)
        R, _ = oracle_fill([a[::-1].copy(), b[::-1].copy()], sub, gap)
        out[(i, j)] = (P, R[::-1, ::-1].copy())
    return out


def upper_bound(seqs, sub, gap):
    """U = sum over pairs of the optimal pairwise score."""
    return int(sum(int(P[-1, -1]) for P, _ in pair_tables(seqs, sub, gap).values()))


def cell_bound(seqs, sub, gap):
    """B(v) for every cell of the k-dimensional tensor (small inputs)."""
    k = len(seqs)
    shape = tuple(len(s) + 1 for s in seqs)
    B = np.zeros(shape, np.int64)
    for (i, j), (P, Q) in pair_tables(seqs, sub, gap).items():
        view = [1] * k
        view[i], view[j] = shape[i], shape[j]
        B = B + (P + Q).reshape(view)
    return B


def tile_ranges(n, T):
    """Cell ranges [lo, hi] of the tiles along one dimension."""
    r = [(0, 0)]
    for c in range(1, 1 + (n + T - 1) // T):
        r.append(((c - 1) * T + 1, min(c * T, n)))
    return r


def tile_bound(seqs, sub, gap, T):
    """Per tile (array over tile coordinates): sum over pairs of the block
    maximum of P_ij + Q_ij, and U."""
    k = len(seqs)
    rng = [tile_ranges(len(s), T) for s in seqs]
    shape = tuple(len(r) for r in rng)
    tot = np.zeros(shape, np.int64)
    U = 0
    for (i, j), (P, Q) in pair_tables(seqs, sub, gap).items():
        U += int(P[-1, -1])
        S = P + Q
        bm = np.empty((shape[i], shape[j]), np.int64)
        for a, (alo, ahi) in enumerate(rng[i]):
            for b, (blo, bhi) in enumerate(rng[j]):
                bm[a, b] = S[alo:ahi + 1, blo:bhi + 1].max()
        view = [1] * k
        view[i], view[j] = shape[i], shape[j]
        tot = tot + bm.reshape(view)
    return tot, U


def tile_keep(seqs, sub, gap, T, L):
    """Boolean array over tile coordinates: tiles kept at threshold L."""
    tot, _ = tile_bound(seqs, sub, gap, T)
    return tot >= L


def first_threshold(U, k, sub, gap):
    """L1 of the first pass (see the module docstring)."""
    cmax = max(abs(int(gap)), int(np.abs(np.asarray(sub, np.int64)).max()))
    return int(U) - (abs(int(U)) + 15) // 16 - (k * (k - 1) // 2) * cmax
