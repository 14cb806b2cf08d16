"""Exhaustive enumeration of every alignment of tiny inputs.

TEST INFRASTRUCTURE ONLY.  An independent pin for the C dynamic programme:
no recurrence, no table, no code shared with it.

An alignment of k sequences is a sequence of columns; each column takes the
next residue from the sequences in a nonempty subset b of {0..k-1} and a gap
from the others (Section 2: a cell of the k-dimensional tensor has 2^k - 1
lower neighbours, one per nonempty subset).  Its score is the sum over
columns of the sum-of-pairs column score of Section 5.2 (residue pair:
substitution score, residue-gap: the gap value, gap-gap: 0).

Enumeration runs from the END of the alignment backwards, trying masks in
ascending order, so alignments are visited in lexicographic order of their
column masks read from the last column to the first.  The first alignment
reaching the maximum score in that order is the one a traceback from the far
corner produces when every cell keeps its lowest maximising mask.
"""
from __future__ import annotations

GAP = 0xFF


def _column_score(col, sub, gap):
    s = 0
    k = len(col)
    for i in range(k):
        for j in range(i + 1, k):
            a, b = col[i], col[j]
            if a is None and b is None:
                continue
            if a is None or b is None:
                s += gap
            else:
                s += sub[a][b]
    return s


def enumerate_alignments(seqs, sub, gap):
    """Yield ``(score, masks_end_first)`` for every alignment of ``seqs``."""
    k = len(seqs)
    seqs = [list(map(int, s)) for s in seqs]
    sub = [list(map(int, r)) for r in sub]
    end = tuple(len(s) for s in seqs)

    def rec(v, score, masks):
        if all(x == 0 for x in v):
            yield score, tuple(masks)
            return
        for b in range(1, 1 << k):
            if any((b >> i) & 1 and v[i] == 0 for i in range(k)):
                continue
            col = [seqs[i][v[i] - 1] if (b >> i) & 1 else None for i in range(k)]
            nv = tuple(v[i] - ((b >> i) & 1) for i in range(k))
            masks.append(b)
            yield from rec(nv, score + _column_score(col, sub, gap), masks)
            masks.pop()

    yield from rec(end, 0, [])


def count_alignments(lens):
    """Number of alignments (monotone paths with nonempty steps)."""
    k = len(lens)

    def rec(v):
        if all(x == 0 for x in v):
            return 1
        n = 0
        for b in range(1, 1 << k):
            if any((b >> i) & 1 and v[i] == 0 for i in range(k)):
                continue
            n += rec(tuple(v[i] - ((b >> i) & 1) for i in range(k)))
        return n

    return rec(tuple(lens))


def brute_force_align(seqs, sub, gap):
    """Return ``(best_score, rows, n_alignments, n_optimal)``.

    ``rows`` is the optimal alignment whose column masks, read from the last
    column to the first, are lexicographically smallest (k lists of codes,
    GAP for gaps), i.e. the one the lowest-mask tie rule selects.
    """
    best = None
    best_masks = None
    n = 0
    n_opt = 0
    for score, masks in enumerate_alignments(seqs, sub, gap):
        n += 1
        if best is None or score > best:
            best, best_masks, n_opt = score, masks, 1
        elif score == best:
            n_opt += 1  # later in lexicographic order: keep the first
    k = len(seqs)
    pos = [0] * k
    rows = [[] for _ in range(k)]
    for b in reversed(best_masks):  # origin to end
        for i in range(k):
            if (b >> i) & 1:
                rows[i].append(int(seqs[i][pos[i]]))
                pos[i] += 1
            else:
                rows[i].append(GAP)
    return best, rows, n, n_opt


def brute_force_egf_score(seqs, sub, gap):
    """Best end-gap-free score by enumeration, independent of any recurrence.

    End-gap-free reading of Section 2's traceback start (the best-scoring cell
    of the far boundary): an alignment may leave a prefix and a suffix of the
    sequences unaligned for free.  The aligned part (the core) aligns the
    substrings s_i[a_i:e_i] where the start a has some a_i = 0 (a prefix of
    every sequence but at least one is skipped) and the end e >= a has some
    e_j = n_j (a suffix of every sequence but at least one is skipped).  The
    score is the best sum-of-pairs score of any core.  Returns
    ``(best_score, n_cores)`` with n_cores the number of (a, e, alignment)
    triples enumerated.
    """
    import itertools

    k = len(seqs)
    seqs = [list(map(int, s)) for s in seqs]
    lens = [len(s) for s in seqs]
    best = None
    n = 0
    for a in itertools.product(*[range(m + 1) for m in lens]):
        if all(x > 0 for x in a):
            continue
        for e in itertools.product(*[range(a[i], lens[i] + 1) for i in range(k)]):
            if all(e[i] < lens[i] for i in range(k)):
                continue
            parts = [s[a[i]:e[i]] for i, s in enumerate(seqs)]
            for score, _ in enumerate_alignments(parts, sub, gap):
                n += 1
                if best is None or score > best:
                    best = score
    return best, n


def brute_force_optima(seqs, sub, gap):
    """Every optimal alignment, in the enumeration order above (lexicographic
    in the column masks read from the last column to the first).  Returns
    ``(best_score, [rows, ...])`` with rows as k lists of codes (GAP for gaps).
    """
    all_ = list(enumerate_alignments(seqs, sub, gap))
    best = max(s for s, _ in all_)
    k = len(seqs)
    out = []
    for score, masks in all_:
        if score != best:
            continue
        pos = [0] * k
        rows = [[] for _ in range(k)]
        for b in reversed(masks):
            for i in range(k):
                if (b >> i) & 1:
                    rows[i].append(int(seqs[i][pos[i]]))
                    pos[i] += 1
                else:
                    rows[i].append(GAP)
        out.append(rows)
    return best, out


def brute_force_within(seqs, sub, gap, delta):
    """Every alignment scoring at least best - ``delta``, in the enumeration
    order above.  Returns ``(best_score, [(score, rows), ...])`` with rows as
    k lists of codes (GAP for gaps)."""
    all_ = list(enumerate_alignments(seqs, sub, gap))
    best = max(s for s, _ in all_)
    k = len(seqs)
    out = []
    for score, masks in all_:
        if score < best - delta:
            continue
        pos = [0] * k
        rows = [[] for _ in range(k)]
        for b in reversed(masks):
            for i in range(k):
                if (b >> i) & 1:
                    rows[i].append(int(seqs[i][pos[i]]))
                    pos[i] += 1
                else:
                    rows[i].append(GAP)
        out.append((score, rows))
    return best, out
