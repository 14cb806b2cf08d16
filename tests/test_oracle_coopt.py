"""Pins for the oracle's co-optimal enumeration (Section 6 proposes a
traceback that branches wherever several choices tie).

- exhaustive enumeration of every alignment of tiny k = 2, 3 inputs: the list
  of optimal alignments, in the same order (column masks read from the last
  column to the first, ascending), equals the oracle's list;
- a limit returns a prefix of that list;
- the first alignment is the one the lowest-mask tie rule gives;
- the lowest mask of every cell's tie set is the decision of the plain fill;
- every returned alignment scores the optimum and strips to the inputs.
"""
import numpy as np

from msa_inputs import dna_scoring, protein_scoring
from oracle import oracle_align, oracle_coopt
from oracle.brute import brute_force_align, brute_force_optima
from tests.test_oracle_pins import check_alignment_shape, enc, rand_sym, sp_of_rows


def test_coopt_equals_brute_force_list():
    rng = np.random.default_rng(21)
    sub, gap = dna_scoring()
    cases = [[enc("AG"), enc("GA")], [enc("GATTACA"), enc("GCATGCT")],
             [enc("ACG"), enc("AG"), enc("CG")], [enc("TAG"), enc("AT"), enc("GTA")]]
    for _ in range(12):
        k = int(rng.integers(2, 4))
        nmax = 5 if k == 2 else 3
        cases.append([rng.integers(0, 4, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                      for _ in range(k)])
    for trial, seqs in enumerate(cases):
        s, g = (sub, gap) if trial % 3 else (rand_sym(rng, 4, -2, 3), -1)
        best, optima = brute_force_optima(seqs, s, g)
        score, rows, _ = oracle_coopt(seqs, s, g, max_paths=len(optima) + 3)
        assert score == best
        assert len(rows) == len(optima)
        for r, o in zip(rows, optima):
            assert r.tolist() == o
        # a limit returns a prefix of the list
        lim = max(1, len(optima) // 2)
        _, rows2, _ = oracle_coopt(seqs, s, g, max_paths=lim)
        assert [r.tolist() for r in rows2] == optima[:lim]
        # the count agrees with brute_force_align's
        assert brute_force_align(seqs, s, g)[3] == len(optima)


def test_coopt_first_is_tie_rule_and_ties_extend_decisions():
    rng = np.random.default_rng(22)
    sub, gap = protein_scoring()
    for _ in range(10):
        k = int(rng.integers(2, 4))
        nmax = 25 if k == 2 else 9
        seqs = [rng.integers(0, 4, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                for _ in range(k)]
        s0, r0, d0 = oracle_align(seqs, sub[:4, :4], gap, want_dir=True)
        score, rows, ties = oracle_coopt(seqs, sub[:4, :4], gap, max_paths=8, want_ties=True)
        assert score == s0 and np.array_equal(rows[0], r0)
        lowest = np.array([0] + [(t & -t).bit_length() for t in range(1, 256)], np.uint8)
        assert np.array_equal(lowest[ties], d0)
        seen = set()
        for r in rows:
            check_alignment_shape(r, seqs)
            assert sp_of_rows(r, sub[:4, :4], gap) == score
            seen.add(r.tobytes() + bytes([r.shape[1]]))
        assert len(seen) == len(rows)
