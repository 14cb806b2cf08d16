"""Pins for the oracle's end-gap-free variant (the reading of Section 2's
traceback start at the best-scoring cell of the far boundary).

- hand-worked cases (tests/golden/egf_cases.json);
- k = 2 equals textbook overlap (semi-global) alignment, written
  independently in tests/nw_reference.py;
- exhaustive enumeration of every core (any start with some a_i = 0, any end
  with some e_j = n_j, every alignment of the substrings) on tiny k = 3 inputs;
- invariants: the score is the sum-of-pairs score of the returned core, rows
  strip to the inputs, the score is at least 0 and at least the global score
  (gap < 0), identical sequences give the global alignment.
"""
import json
from pathlib import Path

import numpy as np

from msa_inputs import dna_scoring, protein_scoring
from oracle import GAP, oracle_align, oracle_align_egf
from oracle.brute import brute_force_egf_score
from tests.nw_reference import semiglobal_nw_score
from tests.test_oracle_pins import check_alignment_shape, dec, enc, rand_sym, sp_of_rows

GOLDEN = Path(__file__).resolve().parent / "golden"


def test_egf_hand_cases():
    data = json.load(open(GOLDEN / "egf_cases.json"))
    sc = data["scoring"]
    sub = np.full((4, 4), sc["mismatch"], dtype=np.int32)
    np.fill_diagonal(sub, sc["match"])
    for case in data["cases"]:
        seqs = [enc(s) for s in case["seqs"]]
        score, rows, _, core = oracle_align_egf(seqs, sub, sc["gap"])
        assert score == case["score"], case["id"]
        assert [dec(r) for r in rows] == case["rows"], case["id"]
        assert list(core) == case["core"], case["id"]


def test_egf_k2_is_overlap_alignment():
    rng = np.random.default_rng(11)
    for trial in range(60):
        prot = trial % 2 == 1
        sub, gap = protein_scoring() if prot else dna_scoring()
        if trial % 5 == 4:
            sub, gap = rand_sym(rng, 4), int(rng.integers(-4, 0))
        a = rng.integers(0, sub.shape[0], size=int(rng.integers(0, 12))).astype(np.uint8)
        b = rng.integers(0, sub.shape[0], size=int(rng.integers(0, 12))).astype(np.uint8)
        score, rows, _, (c0, c1) = oracle_align_egf([a, b], sub, gap)
        assert score == semiglobal_nw_score(a, b, sub, gap)
        check_alignment_shape(rows, [a, b])
        assert sp_of_rows(rows[:, c0:c1], sub, gap) == score


def test_egf_brute_force_k3():
    rng = np.random.default_rng(12)
    sub, gap = dna_scoring()
    cases = [[enc("AC"), enc("CA"), enc("A")], [enc("GAT"), enc("TA"), enc("AG")]]
    for _ in range(8):
        cases.append([rng.integers(0, 4, size=int(rng.integers(0, 3))).astype(np.uint8)
                      for _ in range(3)])
    for seqs in cases:
        score, rows, _, (c0, c1) = oracle_align_egf(seqs, sub, gap)
        best, n = brute_force_egf_score(seqs, sub, gap)
        assert score == best, [dec(s) for s in seqs]
        assert n >= 1
        check_alignment_shape(rows, seqs)
        assert sp_of_rows(rows[:, c0:c1], sub, gap) == score


def test_egf_invariants():
    rng = np.random.default_rng(13)
    sub, gap = protein_scoring()
    for _ in range(12):
        k = int(rng.integers(2, 5))
        nmax = {2: 30, 3: 12, 4: 6}[k]
        seqs = [rng.integers(0, 20, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                for _ in range(k)]
        score, rows, _, (c0, c1) = oracle_align_egf(seqs, sub, gap)
        gscore = oracle_align(seqs, sub, gap)[0]
        assert score >= 0 and score >= gscore
        check_alignment_shape(rows, seqs)
        assert sp_of_rows(rows[:, c0:c1], sub, gap) == score
        # outside the core every column holds exactly one residue
        outside = np.concatenate([rows[:, :c0], rows[:, c1:]], axis=1)
        assert (np.sum(outside != GAP, axis=0) == 1).all()
    # identical sequences: the whole diagonal, as in the global alignment
    x = rng.integers(0, 20, size=9).astype(np.uint8)
    score, rows, _, core = oracle_align_egf([x, x, x], sub, gap)
    gscore, grows, _ = oracle_align([x, x, x], sub, gap)
    assert score == gscore and np.array_equal(rows, grows) and core == (0, 9)
