"""Pins for the pruning oracle (oracle/prune.py): the pairwise bound of
Carrillo and Lipman that makes Section 6's partition selection exact.

- the prefix tables are textbook Needleman-Wunsch tables and the suffix
  tables are Needleman-Wunsch scores of the suffixes, both from an
  implementation written independently of the oracle;
- for two sequences the bound of a cell is exactly the best score of any
  alignment through it (enumeration);
- for k = 3, 4 every enumerated alignment scores at most the bound of every
  cell it passes through;
- the tile bound is at least the cell bound of every cell in the tile, and
  equal to the largest one for two sequences;
- at any threshold L <= optimum every optimal alignment runs through kept
  tiles only, so the best alignment restricted to kept tiles is the optimum
  and the lowest-mask rule picks the same one; a pass that reaches its own
  threshold is exact.
"""
import itertools

import numpy as np

from msa_inputs import dna_scoring, protein_scoring
from oracle.brute import enumerate_alignments
from oracle.prune import (cell_bound, first_threshold, pair_tables, tile_bound, tile_keep,
                          tile_ranges, upper_bound)
from tests.nw_reference import nw_score_table
from tests.test_oracle_pins import rand_sym


def _cells_of(masks, lens):
    """Cells visited by an alignment given by its masks (end first)."""
    v = list(lens)
    cells = [tuple(v)]
    for b in masks:
        for i in range(len(v)):
            v[i] -= (b >> i) & 1
        cells.append(tuple(v))
    return cells


def _tile_of(v, T):
    return tuple(0 if x == 0 else (x - 1) // T + 1 for x in v)


def test_tile_ranges_partition_each_dimension():
    for n in range(0, 40):
        for T in (1, 2, 3, 5, 16):
            r = tile_ranges(n, T)
            cells = [x for lo, hi in r for x in range(lo, hi + 1)]
            assert cells == list(range(n + 1))
            assert len(r) == 1 + (n + T - 1) // T
            assert all(_tile_of((x,), T)[0] == c for c, (lo, hi) in enumerate(r)
                       for x in range(lo, hi + 1))


def test_pair_tables_are_textbook_prefix_and_suffix_scores():
    rng = np.random.default_rng(31)
    for trial in range(6):
        sub, gap = (dna_scoring() if trial % 2 else (rand_sym(rng, 4, -3, 4), -2))
        seqs = [rng.integers(0, 4, size=int(rng.integers(0, 9))).astype(np.uint8)
                for _ in range(3)]
        for (i, j), (P, Q) in pair_tables(seqs, sub, gap).items():
            a, b = seqs[i], seqs[j]
            assert np.array_equal(P, nw_score_table(a, b, sub, gap))
            for x in range(len(a) + 1):
                for y in range(len(b) + 1):
                    assert Q[x, y] == nw_score_table(a[x:], b[y:], sub, gap)[-1, -1]


def test_two_sequence_bound_is_best_alignment_through_cell():
    rng = np.random.default_rng(32)
    for trial in range(6):
        sub, gap = (protein_scoring() if trial % 2 else dna_scoring())
        sub = np.asarray(sub)[:4, :4]
        seqs = [rng.integers(0, 4, size=int(rng.integers(0, 6))).astype(np.uint8)
                for _ in range(2)]
        lens = [len(s) for s in seqs]
        best = np.full([n + 1 for n in lens], np.iinfo(np.int64).min, np.int64)
        for score, masks in enumerate_alignments(seqs, sub, gap):
            for v in _cells_of(masks, lens):
                best[v] = max(best[v], score)
        assert np.array_equal(cell_bound(seqs, sub, gap), best)


def test_bound_dominates_every_alignment_k3_k4():
    rng = np.random.default_rng(33)
    shapes = [(3, 3, 2), (2, 3, 3), (2, 2, 2, 2), (1, 3, 2, 2)]
    for trial, lens in enumerate(shapes):
        sub, gap = (dna_scoring() if trial % 2 else (rand_sym(rng, 4, -2, 3), -1))
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
        B = cell_bound(seqs, sub, gap)
        U = upper_bound(seqs, sub, gap)
        opt = None
        for score, masks in enumerate_alignments(seqs, sub, gap):
            opt = score if opt is None else max(opt, score)
            for v in _cells_of(masks, list(lens)):
                assert score <= B[v], (lens, v)
        assert B[(0,) * len(lens)] == U == B[tuple(lens)]
        assert opt <= U


def test_tile_bound_covers_cell_bound():
    rng = np.random.default_rng(34)
    for trial in range(5):
        k = 2 + trial % 3
        sub, gap = protein_scoring()
        seqs = [rng.integers(0, 20, size=int(rng.integers(0, 8))).astype(np.uint8)
                for _ in range(k)]
        T = int(rng.integers(1, 4))
        tot, U = tile_bound(seqs, sub, gap, T)
        B = cell_bound(seqs, sub, gap)
        tmax = np.full(tot.shape, np.iinfo(np.int64).min, np.int64)
        for v in itertools.product(*[range(len(s) + 1) for s in seqs]):
            t = _tile_of(v, T)
            tmax[t] = max(tmax[t], B[v])
        assert np.all(tot >= tmax)
        if k == 2:
            assert np.array_equal(tot, tmax)
        assert U == upper_bound(seqs, sub, gap)


def _restricted_best(seqs, sub, gap, keep, T):
    """Best score over alignments whose cells all lie in kept tiles, and the
    first such alignment (masks, end first) reaching it in mask order."""
    lens = [len(s) for s in seqs]
    best, first = None, None
    for score, masks in enumerate_alignments(seqs, sub, gap):
        if not all(keep[_tile_of(v, T)] for v in _cells_of(masks, lens)):
            continue
        if best is None or score > best:
            best, first = score, masks
    return best, first


def test_pruning_keeps_optimum_and_tie_rule():
    rng = np.random.default_rng(35)
    shapes = [(3, 3, 3), (3, 3, 2), (2, 2, 2, 2), (3, 2, 3)]
    for trial, lens in enumerate(shapes):
        sub, gap = (dna_scoring() if trial % 2 else (rand_sym(rng, 4, -2, 3), -1))
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
        all_ = list(enumerate_alignments(seqs, sub, gap))
        opt = max(s for s, _ in all_)
        first_opt = next(m for s, m in all_ if s == opt)
        U = upper_bound(seqs, sub, gap)
        for T in (1, 2):
            for L in (opt, opt - 1, opt - 3):
                keep = tile_keep(seqs, sub, gap, T, L)
                for s, m in all_:  # every optimal alignment is kept
                    if s == opt:
                        assert all(keep[_tile_of(v, T)] for v in _cells_of(m, list(lens)))
                best, first = _restricted_best(seqs, sub, gap, keep, T)
                assert best == opt and first == first_opt
            # keep sets shrink as L grows; everything is kept far below
            k_lo = tile_keep(seqs, sub, gap, T, opt - 5)
            k_hi = tile_keep(seqs, sub, gap, T, opt + 2)
            assert np.all(k_lo >= k_hi)
            assert np.all(tile_keep(seqs, sub, gap, T, -10 ** 9))
            # the end tile is kept for every L <= U
            end = _tile_of(lens, T)
            assert tile_keep(seqs, sub, gap, T, U)[end]
            # a pass reaching its threshold is exact, whatever the threshold
            for L in range(opt - 4, U + 2):
                keep = tile_keep(seqs, sub, gap, T, L)
                best, _ = _restricted_best(seqs, sub, gap, keep, T)
                if best is not None and best >= L:
                    assert best == opt


def test_first_threshold_rule():
    sub, gap = protein_scoring()
    assert first_threshold(5234, 3, sub, gap) == 5234 - 328 - 3 * max(8, int(np.abs(sub).max()))
    dsub, dgap = dna_scoring()
    assert first_threshold(-17, 4, dsub, dgap) == -17 - 2 - 6 * 2
    assert first_threshold(0, 3, dsub, dgap) == -6
