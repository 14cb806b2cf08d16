"""Oracle for optimal k-sequence alignment by dynamic programming.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU library never does, and this
package never imports the GPU library.

- ``msa_oracle.c``  plain single-threaded C dynamic programme (int64 scores,
  one decision byte per cell, traceback from the far corner), following Eq. 1
  of the paper generalised to 2^k - 1 neighbours (Section 2) with the
  sum-of-pairs column score of Section 5.2.
  ``msa_oracle_align_egf`` is the end-gap-free reading of the traceback start
  (the best cell of the far boundary, Section 2); ``msa_oracle_coopt``
  enumerates co-optimal alignments and ``msa_oracle_nearopt`` the
  alignments within a threshold of the optimum (Section 6).
- ``brute.py``      enumeration of every alignment of tiny inputs, scored
  column by column; the exact optimum and the tie rule by definition.
"""
from .oracle import (  # noqa: F401
    GAP,
    build_oracle_lib,
    oracle_align,
    oracle_align_egf,
    oracle_coopt,
    oracle_fill,
    oracle_nearopt,
    oracle_lib_path,
)
