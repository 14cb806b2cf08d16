"""Textbook two-sequence Needleman-Wunsch, written independently of the
oracle as a pin for its k = 2 case.

Eq. 1 of the paper: xi(i,j) = max(xi(i-1,j-1) + sub(a_i, b_j),
xi(i-1,j) + g, xi(i,j-1) + g), with the usual borders xi(i,0) = i*g and
xi(0,j) = j*g.  Ties are resolved in the order "up" (consume a_i only),
"left" (consume b_j only), "diagonal", which is the lowest-mask rule with
bit 0 = first sequence.
"""
from __future__ import annotations

import numpy as np

UP, LEFT, DIAG = 1, 2, 3


def needleman_wunsch(a, b, sub, g):
    n, m = len(a), len(b)
    F = np.zeros((n + 1, m + 1), dtype=np.int64)
    T = np.zeros((n + 1, m + 1), dtype=np.uint8)
    for i in range(1, n + 1):
        F[i, 0] = i * g
        T[i, 0] = UP
    for j in range(1, m + 1):
        F[0, j] = j * g
        T[0, j] = LEFT
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            up = F[i - 1, j] + g
            left = F[i, j - 1] + g
            diag = F[i - 1, j - 1] + int(sub[a[i - 1]][b[j - 1]])
            best, move = up, UP
            if left > best:
                best, move = left, LEFT
            if diag > best:
                best, move = diag, DIAG
            F[i, j] = best
            T[i, j] = move
    ra, rb = [], []
    i, j = n, m
    while i > 0 or j > 0:
        mv = T[i, j]
        if mv == DIAG:
            ra.append(int(a[i - 1])); rb.append(int(b[j - 1])); i -= 1; j -= 1
        elif mv == UP:
            ra.append(int(a[i - 1])); rb.append(0xFF); i -= 1
        else:
            ra.append(0xFF); rb.append(int(b[j - 1])); j -= 1
    return int(F[n, m]), [ra[::-1], rb[::-1]], T


def semiglobal_nw_score(a, b, sub, g):
    """Textbook overlap (semi-global) alignment score of two sequences: end
    gaps are free, i.e. xi(i,0) = xi(0,j) = 0 and the result is the maximum
    over the last row and the last column."""
    n, m = len(a), len(b)
    F = np.zeros((n + 1, m + 1), dtype=np.int64)
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            F[i, j] = max(F[i - 1, j] + g, F[i, j - 1] + g,
                          F[i - 1, j - 1] + int(sub[a[i - 1]][b[j - 1]]))
    return int(max(F[n, :].max(), F[:, m].max()))


def nw_score_table(a, b, sub, g):
    """F[i, j] = best score of aligning a[:i] with b[:j] (the table above)."""
    n, m = len(a), len(b)
    F = np.zeros((n + 1, m + 1), dtype=np.int64)
    for i in range(1, n + 1):
        F[i, 0] = i * g
    for j in range(1, m + 1):
        F[0, j] = j * g
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            F[i, j] = max(F[i - 1, j] + g, F[i, j - 1] + g,
                          F[i - 1, j - 1] + int(sub[a[i - 1]][b[j - 1]]))
    return F
