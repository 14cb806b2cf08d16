"""Pins for the oracle's near-optimal enumeration (Section 6: alignments whose
score lies within a threshold set by the user of the optimum).

- exhaustive enumeration of every alignment of tiny k = 2..4 inputs, filtered
  to scores >= best - delta, in the same order (column masks read from the
  last column to the first, ascending), equals the oracle's list for several
  delta, scores included; a limit returns a prefix of that list;
- delta = 0 gives the co-optimal list (a separate walk over tie sets);
- a delta above any score spread returns every alignment: their number is
  the Delannoy number for k = 2 and the brute-force count for k = 3;
- on larger inputs every returned alignment strips to the inputs, scores what
  is reported (column by column), reaches the threshold, and the list is
  strictly increasing in its end-first mask sequences.
"""
from math import comb

import numpy as np

from msa_inputs import dna_scoring, protein_scoring
from oracle import oracle_coopt, oracle_nearopt
from oracle.brute import brute_force_within, count_alignments
from tests.test_oracle_pins import check_alignment_shape, enc, rand_sym, sp_of_rows


def masks_end_first(rows):
    k = rows.shape[0]
    cols = [sum(1 << i for i in range(k) if rows[i, c] != 0xFF) for c in range(rows.shape[1])]
    return cols[::-1]


def test_nearopt_equals_brute_force_list():
    rng = np.random.default_rng(31)
    sub, gap = dna_scoring()
    cases = [[enc("AG"), enc("GA")], [enc("GATT"), enc("GCAT")],
             [enc("ACG"), enc("AG"), enc("CG")], [enc("TA"), enc("A"), enc("GT"), enc("T")]]
    for _ in range(14):
        k = int(rng.integers(2, 5))
        nmax = {2: 5, 3: 3, 4: 2}[k]
        cases.append([rng.integers(0, 4, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                      for _ in range(k)])
    for trial, seqs in enumerate(cases):
        s, g = (sub, gap) if trial % 3 else (rand_sym(rng, 4, -2, 3), -1)
        for delta in (0, 1, 2, 5, 40):
            best, want = brute_force_within(seqs, s, g, delta)
            opt, got = oracle_nearopt(seqs, s, g, delta, max_paths=len(want) + 2)
            assert opt == best
            assert len(got) == len(want), (trial, delta)
            for (gs, gr), (ws, wr) in zip(got, want):
                assert gs == ws and gr.tolist() == wr
            lim = max(1, len(want) // 3)
            _, got2 = oracle_nearopt(seqs, s, g, delta, max_paths=lim)
            assert [(a, r.tolist()) for a, r in got2] == [(a, r) for a, r in want[:lim]]


def test_nearopt_delta_zero_is_coopt():
    rng = np.random.default_rng(32)
    sub, gap = protein_scoring()
    for _ in range(8):
        k = int(rng.integers(2, 4))
        nmax = 30 if k == 2 else 12
        seqs = [rng.integers(0, 4, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                for _ in range(k)]
        score, rows, _ = oracle_coopt(seqs, sub[:4, :4], gap, max_paths=40)
        opt, got = oracle_nearopt(seqs, sub[:4, :4], gap, 0, max_paths=40)
        assert opt == score and len(got) == len(rows)
        for (gs, gr), r in zip(got, rows):
            assert gs == score and np.array_equal(gr, r)


def test_nearopt_large_delta_returns_every_alignment():
    sub, gap = dna_scoring()
    for m, n in ((0, 0), (1, 3), (3, 3), (4, 2), (5, 4)):
        seqs = [enc("ACGTA"[:m]), enc("GGCAT"[:n])]
        _, got = oracle_nearopt(seqs, sub, gap, 10**6, max_paths=5000)
        delannoy = sum(comb(m, i) * comb(n, i) * 2 ** i for i in range(min(m, n) + 1))
        assert len(got) == delannoy
    seqs = [enc("ACG"), enc("GA"), enc("TC")]
    _, got = oracle_nearopt(seqs, sub, gap, 10**6, max_paths=20000)
    assert len(got) == count_alignments([3, 2, 2])


def test_nearopt_invariants_on_larger_inputs():
    rng = np.random.default_rng(33)
    sub, gap = protein_scoring()
    for k, n, delta in ((2, 40, 12), (3, 14, 10), (4, 6, 8), (5, 4, 6)):
        seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for _ in range(k)]
        opt, got = oracle_nearopt(seqs, sub, gap, delta, max_paths=300)
        assert got and got[0][0] <= opt
        prev = None
        for score, rows in got:
            check_alignment_shape(rows, seqs)
            assert sp_of_rows(rows, sub, gap) == score
            assert opt - delta <= score <= opt
            key = masks_end_first(rows)
            if prev is not None:
                assert key > prev
            prev = key
