"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds only input generation (residue codes, substitution
matrices, job lists, arrival times).  It contains none of the alignment
arithmetic, so neither the oracle nor the GPU library depends on the other
through it.  Every generator draws from ``numpy.random.Generator(PCG64(seed))``
and is deterministic across platforms.

Workloads (the paper gives no datasets; these stand in for them):
  dna_k3_40      k=3 DNA, length 40 each, +2/-1, gap -2            (seed 1)
  prot_k3_512    k=3 protein, length 512 each, gap -8              (seed 2)
  prot_k4_128    k=4 protein, length 128 each, gap -8              (seed 3)
  prot_k5_40     k=5 protein, length 40 each, gap -8               (seed 7)
  batch_4096     4096 jobs, k in {3,4}, lengths 16..160, DNA/protein (seed 4)
  served_20000   20000 jobs, k in {3,4,5}, Poisson arrivals       (seeds 5, 6)
"""
from .gen import (  # noqa: F401
    DNA_ALPHABET,
    PROTEIN_ALPHABET,
    Job,
    batch_jobs,
    dna_scoring,
    mutate_from_ancestor,
    poisson_arrivals,
    protein_matrix,
    protein_scoring,
    random_dna,
    served_jobs,
    workload,
    WORKLOADS,
)
