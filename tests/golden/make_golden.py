"""Write the stored expected values used by the tests.

Calls only the oracle package (brute-force enumerator and the C dynamic
programme) and the seeded input generators; nothing here touches the GPU
library.  Run from the repository root:

    python tests/golden/make_golden.py            # brute-force cases only
    python tests/golden/make_golden.py --full     # also the large workloads

Outputs:
  brute_cases.json   H3..H7: optimum, tie-rule alignment and alignment counts
                     by exhaustive enumeration (DNA +2/-1, gap -2)
  workloads.json     score, alignment and SHA-256 of the row-major decision
                     tensor of the oracle for the fixed workloads
"""
from __future__ import annotations

import argparse
import hashlib
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from msa_inputs import batch_jobs, dna_scoring, workload  # noqa: E402
from oracle import oracle_align  # noqa: E402
from oracle.brute import brute_force_align  # noqa: E402

HERE = Path(__file__).resolve().parent

BRUTE_CASES = [
    ("H3", ["GATTACA", "GCATGCT"]),
    ("H4", ["A", "A", ""]),
    ("H5", ["ACGT", "ACGT", "ACGT"]),
    ("H6", ["ACG", "AG", "CG"]),
    ("H7", ["TAG", "AT", "GTA"]),
]


def enc(s):
    return np.array(["ACGT".index(c) for c in s], dtype=np.uint8)


def dec(row):
    return "".join("-" if x == 0xFF else "ACGT"[x] for x in row)


def brute_cases():
    sub, gap = dna_scoring()
    out = []
    for cid, seqs in BRUTE_CASES:
        best, rows, n, nopt = brute_force_align([enc(s) for s in seqs], sub, gap)
        out.append(dict(id=cid, seqs=seqs, score=int(best),
                        rows=[dec(r) for r in rows], n_alignments=n,
                        n_optimal=nopt))
        print(cid, best, [dec(r) for r in rows], n, nopt, flush=True)
    doc = {
        "_source": "Exhaustive enumeration of every alignment (oracle/brute.py); "
                   "sum-of-pairs columns (Section 5.2) with the DNA scheme "
                   "+2/-1, gap -2; rows are the optimum selected by the "
                   "lowest-mask tie rule.",
        "scoring": {"alphabet": "ACGT", "match": 2, "mismatch": -1, "gap": -2},
        "cases": out,
    }
    (HERE / "brute_cases.json").write_text(json.dumps(doc, indent=1) + "\n")


def workload_cases(names):
    path = HERE / "workloads.json"
    doc = json.loads(path.read_text()) if path.exists() else {
        "_source": "oracle/msa_oracle.c on the seeded workloads of msa_inputs; "
                   "dir_sha256 is over the row-major decision tensor "
                   "(last sequence fastest, one byte = chosen mask)."}
    for name in names:
        job = workload(name)
        t0 = time.time()
        score, rows, dirt = oracle_align(job.seqs, job.sub, job.gap, want_dir=True)
        dt = time.time() - t0
        doc[name] = dict(
            lens=job.lens, score=score, aln_len=int(rows.shape[1]),
            rows_sha256=hashlib.sha256(np.ascontiguousarray(rows).tobytes()).hexdigest(),
            dir_sha256=hashlib.sha256(np.ascontiguousarray(dirt).tobytes()).hexdigest(),
            oracle_seconds=round(dt, 2))
        print(name, score, rows.shape, round(dt, 1), "s", flush=True)
        path.write_text(json.dumps(doc, indent=1) + "\n")


def batch_largest_case():
    """The largest job of the 4096-job batch (by cells): the oracle's score
    and row hash, for the batched-path test (the other jobs are compared with
    the plain path, itself pinned to the oracle's full decision tensors)."""
    path = HERE / "workloads.json"
    doc = json.loads(path.read_text())
    jobs = batch_jobs(4096)
    idx = int(np.argmax([j.cells for j in jobs]))
    job = jobs[idx]
    t0 = time.time()
    score, rows, _ = oracle_align(job.seqs, job.sub, job.gap)
    dt = time.time() - t0
    doc["batch_4096_largest"] = dict(
        job_index=idx, k=job.k, lens=job.lens, cells=job.cells, score=score,
        aln_len=int(rows.shape[1]),
        rows_sha256=hashlib.sha256(np.ascontiguousarray(rows).tobytes()).hexdigest(),
        oracle_seconds=round(dt, 2))
    print("batch_4096_largest", idx, job.lens, score, rows.shape, round(dt, 1), "s", flush=True)
    path.write_text(json.dumps(doc, indent=1) + "\n")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--only", nargs="*", default=None)
    a = ap.parse_args()
    if a.only is None or "brute" in a.only:
        brute_cases()
    if a.full:
        names = [n for n in ("dna_k3_40", "prot_k3_512", "prot_k4_128")
                 if a.only is None or n in a.only]
        workload_cases(names)
        if a.only is None or "batch_largest" in a.only:
            batch_largest_case()
