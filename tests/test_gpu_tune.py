"""GPU tests of the launch-configuration tuner: every configuration it can
choose (the streaming or the tile fill for k = 3, every workgroup count per
compute unit of the tile fill and of the batched fill) gives the same bytes
-- score, rows and the full decision tensor against the oracle's, batched
results against the plain path -- and the measured choice is one of them.
"""
import sys

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import dna_scoring, protein_scoring
from oracle import oracle_align

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    msa.lib()
    msa.tune_clear()
    yield
    msa.tune_clear()  # later tests in this process use the built-in rule


@pytest.mark.parametrize("lens", [[100, 70, 90], [33, 30, 28, 25], [9, 8, 9, 7, 8]])
def test_every_plain_candidate_gives_the_same_bytes(lens):
    rng = np.random.Generator(np.random.PCG64(9600 + len(lens)))
    sub, gap = protein_scoring()
    seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in lens]
    s0, r0, d0 = oracle_align(seqs, sub, gap, want_dir=True)
    k, m = len(lens), max(lens)
    cands = msa.tune_candidates(msa.MSA_TUNE_PLAIN, k, m)
    assert len(cands) >= 2
    dev = msa.DeviceAligner(lens, sub, gap)
    dev.set_sequences(seqs)
    for variant, wpc in cands:
        say("plain candidate", lens, variant, wpc)
        msa.tune_set(msa.MSA_TUNE_PLAIN, k, m, variant, wpc)
        dev.run()
        s1, r1 = dev.result()
        assert s1 == s0 and np.array_equal(r1, r0), (variant, wpc)
        assert np.array_equal(dev.export_dirs(), d0), (variant, wpc)
    variant, wpc, ms = msa.autotune(lens, sub, gap, reps=2)
    say("autotune", lens, "->", variant, wpc, "%.3f ms" % ms)
    assert (variant, wpc) in cands and ms > 0
    assert msa.tune_get(msa.MSA_TUNE_PLAIN, k, m) == (variant, wpc)
    s1, r1 = msa.align(seqs, sub, gap)
    assert s1 == s0 and np.array_equal(r1, r0)


def small_mixed(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for _ in range(n):
        k = int(rng.integers(2, 6))
        sub, gap = protein_scoring() if rng.integers(0, 2) else dna_scoring()
        nmax = {2: 60, 3: 30, 4: 12, 5: 7}[k]
        jobs.append(([rng.integers(0, sub.shape[0], size=int(rng.integers(0, nmax + 1))).astype(
            np.uint8) for _ in range(k)], sub, gap))
    return jobs


def test_every_batched_candidate_gives_the_same_bytes():
    jobs = small_mixed(9700, 40)
    plain = [msa.align(*j) for j in jobs]
    for k in (3, 5):
        for _, wpc in msa.tune_candidates(msa.MSA_TUNE_BATCH, k, 0):
            say("batched candidate k class of", k, "wpc", wpc)
            msa.tune_set(msa.MSA_TUNE_BATCH, k, 0, 0, wpc)
            res = msa.align_batch(jobs)
            for (st, score, rows), (s0, r0) in zip(res, plain):
                assert st == msa.MSA_OK and score == s0 and np.array_equal(rows, r0)
    choice = msa.autotune_batch(jobs, reps=1)
    say("autotune_batch ->", choice)
    assert choice[0] >= 1 and choice[1] >= 1 and choice[2] == 0 and choice[3] == 0
    res = msa.align_batch(jobs)
    for (st, score, rows), (s0, r0) in zip(res, plain):
        assert st == msa.MSA_OK and score == s0 and np.array_equal(rows, r0)
