"""Seeded generators for sequences, scoring schemes and job streams."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DNA_ALPHABET = "ACGT"
PROTEIN_ALPHABET = "ARNDCQEGHILKMFPSTWYV"

PROTEIN_MATRIX_SEED = 17


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def dna_scoring():
    """4x4 matrix, +2 on the diagonal and -1 elsewhere; gap -2."""
    sub = np.full((4, 4), -1, dtype=np.int8)
    np.fill_diagonal(sub, 2)
    return sub, -2


def protein_matrix(seed: int = PROTEIN_MATRIX_SEED) -> np.ndarray:
    """Symmetric 20x20 int8: diagonal uniform in 4..11, off-diagonal in -4..3."""
    rng = _rng(seed)
    m = np.zeros((20, 20), dtype=np.int8)
    for i in range(20):
        m[i, i] = rng.integers(4, 12)
    for i in range(20):
        for j in range(i + 1, 20):
            x = rng.integers(-4, 4)
            m[i, j] = x
            m[j, i] = x
    return m


def protein_scoring():
    return protein_matrix(), -8


def random_dna(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 4, size=n).astype(np.uint8)


def mutate_from_ancestor(rng: np.random.Generator, anc: np.ndarray,
                         alpha: int = 20, sub_frac: float = 0.20,
                         indel_frac: float = 0.05) -> np.ndarray:
    """One descendant of ``anc``.

    round(sub_frac * L) distinct positions get a uniformly chosen different
    residue; then 2 * round(indel_frac * L / 2) single-residue indel events
    alternate deletion of a random position and insertion of a random residue
    at a random position, so the length stays exactly L.
    """
    s = anc.astype(np.int64).copy()
    L = len(s)
    nsub = int(round(sub_frac * L))
    if nsub:
        pos = rng.choice(L, size=nsub, replace=False)
        for p in pos:
            r = int(rng.integers(0, alpha - 1))
            s[p] = r if r < s[p] else r + 1
    nev = 2 * int(round(indel_frac * L / 2))
    lst = list(s)
    for e in range(nev):
        if e % 2 == 0 and lst:
            del lst[int(rng.integers(0, len(lst)))]
        else:
            lst.insert(int(rng.integers(0, len(lst) + 1)), int(rng.integers(0, alpha)))
    return np.asarray(lst, dtype=np.uint8)


@dataclass
class Job:
    """One alignment problem: k code arrays, a substitution matrix, a gap."""
    seqs: list
    sub: np.ndarray
    gap: int
    kind: str = ""
    arrival: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def k(self) -> int:
        return len(self.seqs)

    @property
    def lens(self):
        return [len(s) for s in self.seqs]

    @property
    def cells(self) -> int:
        n = 1
        for s in self.seqs:
            n *= len(s) + 1
        return n

    @property
    def neighbour_updates(self) -> int:
        """Number of (cell, in-range lower neighbour) pairs."""
        a = 1
        c = 1
        for s in self.seqs:
            a *= 2 * len(s) + 1
            c *= len(s) + 1
        return a - c


def _dna_job(rng, lens, kind="dna"):
    sub, gap = dna_scoring()
    return Job([random_dna(rng, n) for n in lens], sub, gap, kind)


def _protein_job(rng, lens, kind="protein"):
    sub, gap = protein_scoring()
    L = max(lens) if lens else 0
    anc = rng.integers(0, 20, size=L).astype(np.uint8)
    seqs = [mutate_from_ancestor(rng, anc)[:n] for n in lens]
    return Job(seqs, sub, gap, kind)


def _fixed(name, k, n, seed, protein):
    rng = _rng(seed)
    if protein:
        sub, gap = protein_scoring()
        anc = rng.integers(0, 20, size=n).astype(np.uint8)
        seqs = [mutate_from_ancestor(rng, anc) for _ in range(k)]
        return Job(seqs, sub, gap, name)
    return _dna_job(rng, [n] * k, name)


WORKLOADS = {
    "dna_k3_40": dict(k=3, n=40, seed=1, protein=False),
    "prot_k3_512": dict(k=3, n=512, seed=2, protein=True),
    "prot_k4_128": dict(k=4, n=128, seed=3, protein=True),
    "prot_k5_40": dict(k=5, n=40, seed=7, protein=True),
}


def workload(name: str) -> Job:
    """One of the fixed single-alignment workloads (see module docstring)."""
    w = WORKLOADS[name]
    return _fixed(name, w["k"], w["n"], w["seed"], w["protein"])


def batch_jobs(n_jobs: int = 4096, seed: int = 4, lmin: int = 16,
               lmax: int = 160):
    """Independent jobs: k uniform in {3,4}, each length uniform in
    [lmin, lmax] (uneven within a job), DNA or protein with probability 1/2."""
    rng = _rng(seed)
    jobs = []
    for j in range(n_jobs):
        k = int(rng.integers(3, 5))
        lens = [int(x) for x in rng.integers(lmin, lmax + 1, size=k)]
        if rng.integers(0, 2) == 0:
            job = _dna_job(rng, lens)
        else:
            job = _protein_job(rng, lens)
        job.meta["index"] = j
        jobs.append(job)
    return jobs


SERVED_LENGTHS = {3: (16, 256), 4: (16, 96), 5: (12, 40)}


def served_jobs(n_jobs: int = 20000, seed: int = 5):
    """Job stream for serving: k in {3,4,5} with weights 0.6/0.3/0.1,
    protein scoring, lengths uniform per k (see SERVED_LENGTHS)."""
    rng = _rng(seed)
    jobs = []
    for j in range(n_jobs):
        k = int(rng.choice([3, 4, 5], p=[0.6, 0.3, 0.1]))
        lo, hi = SERVED_LENGTHS[k]
        lens = [int(x) for x in rng.integers(lo, hi + 1, size=k)]
        job = _protein_job(rng, lens)
        job.meta["index"] = j
        jobs.append(job)
    return jobs


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 6) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    return np.cumsum(gaps) - gaps[0]
