"""Pins for the oracle against what the paper and the mathematics fix.

- hand-worked Eq. 1 examples (tests/golden/hand_cases.json);
- exhaustive enumeration of every alignment on tiny inputs (score AND the
  alignment chosen by the lowest-mask tie rule), stored cases H3..H7 and
  random cases;
- k = 2 reduces exactly to textbook Needleman-Wunsch (Eq. 1), including the
  full decision table;
- invariants: self-consistent alignment, identical sequences, an empty
  sequence, permutation and reversal of the inputs, closed-form bounds;
- alignment counts (Delannoy numbers) pin the enumerator itself.
"""
import itertools
import json
from math import comb
from pathlib import Path

import numpy as np
import pytest

from msa_inputs import dna_scoring, protein_scoring, workload
from oracle import GAP, oracle_align, oracle_fill
from oracle.brute import brute_force_align, count_alignments
from tests.nw_reference import needleman_wunsch

GOLDEN = Path(__file__).resolve().parent / "golden"


def enc(s):
    return np.array(["ACGT".index(c) for c in s], dtype=np.uint8)


def dec(row):
    return "".join("-" if x == GAP else "ACGT"[x] for x in row)


def rand_sym(rng, alpha, lo=-5, hi=6):
    m = rng.integers(lo, hi, size=(alpha, alpha))
    m = np.triu(m) + np.triu(m, 1).T
    return m.astype(np.int32)


def sp_of_rows(rows, sub, gap):
    """Sum-of-pairs score of an alignment, column by column (Section 5.2)."""
    rows = np.asarray(rows)
    k, L = rows.shape
    s = 0
    for c in range(L):
        for i in range(k):
            for j in range(i + 1, k):
                x, y = rows[i, c], rows[j, c]
                if x == GAP and y == GAP:
                    continue
                s += gap if (x == GAP or y == GAP) else int(sub[x][y])
    return s


def check_alignment_shape(rows, seqs):
    k, L = rows.shape
    for i in range(k):
        assert np.array_equal(rows[i][rows[i] != GAP], np.asarray(seqs[i]))
    assert not np.any(np.all(rows == GAP, axis=0)), "all-gap column"
    assert max(len(s) for s in seqs) <= L <= sum(len(s) for s in seqs)


@pytest.mark.parametrize("case", json.loads((GOLDEN / "hand_cases.json").read_text())["cases"],
                         ids=lambda c: c["id"])
def test_hand_worked_eq1(case):
    sub, gap = dna_scoring()
    score, rows, _ = oracle_align([enc(s) for s in case["seqs"]], sub, gap)
    assert score == case["score"]
    assert [dec(r) for r in rows] == case["rows"]


@pytest.mark.parametrize("case", json.loads((GOLDEN / "brute_cases.json").read_text())["cases"],
                         ids=lambda c: c["id"])
def test_stored_brute_force_cases(case):
    sub, gap = dna_scoring()
    score, rows, _ = oracle_align([enc(s) for s in case["seqs"]], sub, gap)
    assert score == case["score"]
    assert [dec(r) for r in rows] == case["rows"]


@pytest.mark.parametrize("k,nmax,ncase", [(2, 5, 40), (3, 3, 25), (4, 2, 10)])
def test_random_vs_brute_force(k, nmax, ncase):
    rng = np.random.Generator(np.random.PCG64(100 + k))
    for _ in range(ncase):
        alpha = int(rng.integers(2, 6))
        sub = rand_sym(rng, alpha)
        gap = int(rng.integers(-6, 3))
        seqs = [rng.integers(0, alpha, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                for _ in range(k)]
        score, rows, _ = oracle_align(seqs, sub, gap)
        best, brows, _, _ = brute_force_align(seqs, sub, gap)
        assert score == best, (seqs, sub, gap)
        assert rows.tolist() == brows, (seqs, sub, gap)


def test_k2_equals_needleman_wunsch():
    rng = np.random.Generator(np.random.PCG64(7))
    for trial in range(30):
        if trial % 2:
            sub, gap = dna_scoring()
            alpha = 4
        else:
            sub, gap = protein_scoring()
            alpha = 20
        a = rng.integers(0, alpha, size=int(rng.integers(0, 60))).astype(np.uint8)
        b = rng.integers(0, alpha, size=int(rng.integers(0, 60))).astype(np.uint8)
        score, rows, D = oracle_align([a, b], sub, gap, want_dir=True)
        s2, rows2, T = needleman_wunsch(a, b, sub, gap)
        assert score == s2
        assert rows.tolist() == rows2
        assert np.array_equal(D, T)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_identical_sequences(k):
    rng = np.random.Generator(np.random.PCG64(11 + k))
    for sub, gap, alpha in [(*dna_scoring(), 4), (*protein_scoring(), 20)]:
        n = {2: 30, 3: 14, 4: 6, 5: 4}[k]
        x = rng.integers(0, alpha, size=n).astype(np.uint8)
        score, rows, _ = oracle_align([x] * k, sub, gap)
        assert score == comb(k, 2) * int(sum(int(sub[c][c]) for c in x))
        assert rows.shape == (k, n) and np.all(rows == x[None, :])


def test_empty_sequence_adds_gap_per_residue():
    rng = np.random.Generator(np.random.PCG64(21))
    sub, gap = protein_scoring()
    for k in (2, 3):
        seqs = [rng.integers(0, 20, size=int(rng.integers(1, 12))).astype(np.uint8)
                for _ in range(k)]
        base, _, _ = oracle_align(seqs, sub, gap)
        for pos in range(k + 1):
            ext = seqs[:pos] + [np.zeros(0, np.uint8)] + seqs[pos:]
            s, rows, _ = oracle_align(ext, sub, gap)
            assert s == base + gap * sum(len(q) for q in seqs)
            assert np.all(rows[pos] == GAP)
    s, rows, _ = oracle_align([np.zeros(0, np.uint8)] * 3, sub, gap)
    assert s == 0 and rows.shape == (3, 0)


def test_permutation_and_reversal_invariance():
    rng = np.random.Generator(np.random.PCG64(31))
    sub, gap = protein_scoring()
    for _ in range(6):
        seqs = [rng.integers(0, 20, size=int(rng.integers(0, 10))).astype(np.uint8)
                for _ in range(3)]
        base, rows, _ = oracle_align(seqs, sub, gap)
        assert sp_of_rows(rows, sub, gap) == base
        for perm in itertools.permutations(range(3)):
            s, r, _ = oracle_align([seqs[p] for p in perm], sub, gap)
            assert s == base
            assert sp_of_rows(r, sub, gap) == s
        s, r, _ = oracle_align([q[::-1].copy() for q in seqs], sub, gap)
        assert s == base


@pytest.mark.parametrize("name", ["dna_k3_40"])
def test_self_consistency_and_bounds_workload(name):
    job = workload(name)
    score, rows, _ = oracle_align(job.seqs, job.sub, job.gap)
    check_alignment_shape(rows, job.seqs)
    assert sp_of_rows(rows, job.sub, job.gap) == score
    n = job.lens
    k = job.k
    lo = job.gap * (k - 1) * sum(n)
    hi = max(0, int(job.sub.max())) * sum(min(n[i], n[j]) for i in range(k) for j in range(i + 1, k))
    assert lo <= score <= hi


def test_random_self_consistency_and_bounds():
    rng = np.random.Generator(np.random.PCG64(41))
    for _ in range(40):
        k = int(rng.integers(2, 6))
        alpha = int(rng.integers(2, 21))
        sub = rand_sym(rng, alpha, -4, 8)
        gap = int(rng.integers(-8, 0))
        nmax = {2: 40, 3: 12, 4: 6, 5: 4}[k]
        seqs = [rng.integers(0, alpha, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                for _ in range(k)]
        score, rows, _ = oracle_align(seqs, sub, gap)
        check_alignment_shape(rows, seqs)
        assert sp_of_rows(rows, sub, gap) == score
        lo = gap * (k - 1) * sum(map(len, seqs))
        hi = max(0, int(sub.max())) * sum(min(len(seqs[i]), len(seqs[j]))
                                          for i in range(k) for j in range(i + 1, k))
        assert lo <= score <= hi


def test_decision_tensor_only_uses_in_range_neighbours():
    rng = np.random.Generator(np.random.PCG64(51))
    sub, gap = dna_scoring()
    seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in (5, 0, 7, 3)]
    xi, D = oracle_fill(seqs, sub, gap)
    assert D.flat[0] == 0 and xi.flat[0] == 0
    for v in itertools.product(*[range(len(s) + 1) for s in seqs]):
        if not any(v):
            continue
        b = int(D[v])
        assert 1 <= b < 16
        for i in range(4):
            if (b >> i) & 1:
                assert v[i] >= 1


def test_alignment_counts_are_delannoy():
    # central Delannoy numbers D(n) in 2 and 3 dimensions
    assert [count_alignments([n, n]) for n in range(1, 5)] == [3, 13, 63, 321]
    assert [count_alignments([n, n, n]) for n in range(1, 4)] == [13, 409, 16081]


def test_rejects_invalid_input():
    sub, gap = dna_scoring()
    with pytest.raises(ValueError):
        oracle_align([enc("ACG")], sub, gap)  # k < 2
    with pytest.raises(ValueError):
        oracle_align([enc("AC"), np.array([4], np.uint8)], sub, gap)  # code >= alpha
