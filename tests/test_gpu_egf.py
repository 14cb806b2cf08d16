"""GPU parity of the end-gap-free mode (MSA_END_GAPS_FREE) against the
oracle's end-gap-free variant, bit-exact: score, alignment rows and the full
decision tensor (cells with some v_i = 0 carry no decision).  Shapes span
several tiles with ragged tails; the 513^3 protein workload is checked on
score and rows.
"""
import sys

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import dna_scoring, protein_scoring, workload
from oracle import oracle_align, oracle_align_egf

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
    yield


def check_egf(seqs, sub, gap, want_dir=True):
    lens = [len(s) for s in seqs]
    say("egf case k=%d lens=%s" % (len(seqs), lens))
    s0, r0, d0, _ = oracle_align_egf(seqs, sub, gap, want_dir=want_dir)
    dev = msa.DeviceAligner(lens, sub, gap, end_gaps_free=True)
    dev.set_sequences(seqs)
    dev.run()
    s1, r1 = dev.result()
    assert s1 == s0, (lens, s1, s0)
    assert np.array_equal(r1, r0), lens
    if want_dir:
        d1 = dev.export_dirs()
        assert np.array_equal(d1, d0), (lens, np.argwhere(d1 != d0)[:5])
    return dev


NMAX = {2: 75, 3: 37, 4: 19, 5: 12}


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_egf_random_shapes_full_tensor(k):
    rng = np.random.Generator(np.random.PCG64(7000 + k))
    for trial in range(4):
        sub, gap = protein_scoring() if trial % 2 else dna_scoring()
        seqs = [rng.integers(0, sub.shape[0], size=int(rng.integers(0, NMAX[k] + 1))).astype(
            np.uint8) for _ in range(k)]
        check_egf(seqs, sub, gap)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_egf_tile_boundary_lengths(k):
    T = msa.tile_edge(k)
    rng = np.random.Generator(np.random.PCG64(7100 + k))
    sub, gap = protein_scoring()
    for lens in ([T] * k, [T + 1] * k, [2 * T - 1] + [T] * (k - 1), [1] + [2 * T] * (k - 1)):
        seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in lens]
        check_egf(seqs, sub, gap)


def test_egf_degenerate_and_host_path():
    sub, gap = dna_scoring()
    rng = np.random.Generator(np.random.PCG64(7200))
    cases = [[np.zeros(0, np.uint8)] * 3,
             [np.array([1], np.uint8), np.zeros(0, np.uint8), np.array([2, 3], np.uint8)],
             [np.array([0, 1], np.uint8), np.array([1, 0], np.uint8)]]
    for seqs in cases:
        check_egf(seqs, sub, gap)
    for _ in range(6):
        k = int(rng.integers(2, 5))
        seqs = [rng.integers(0, 4, size=int(rng.integers(0, 14))).astype(np.uint8)
                for _ in range(k)]
        s0, r0, _, _ = oracle_align_egf(seqs, sub, gap)
        s1, r1 = msa.align(seqs, sub, gap, end_gaps_free=True)
        assert s1 == s0 and np.array_equal(r1, r0)


def test_egf_repeated_runs_and_mode_switch():
    rng = np.random.Generator(np.random.PCG64(7300))
    sub, gap = protein_scoring()
    seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in (40, 33, 47)]
    dev = check_egf(seqs, sub, gap, want_dir=False)
    first = dev.result()
    for _ in range(3):
        dev.run()
        s, r = dev.result()
        assert s == first[0] and np.array_equal(r, first[1])
    # the host path keys its cached workspace on the mode as well
    g0, gr0, _ = oracle_align(seqs, sub, gap)
    s1, r1 = msa.align(seqs, sub, gap)
    assert s1 == g0 and np.array_equal(r1, gr0)
    s2, r2 = msa.align(seqs, sub, gap, end_gaps_free=True)
    assert s2 == first[0] and np.array_equal(r2, first[1])


def test_egf_full_size_k3_workload():
    job = workload("prot_k3_512")
    say("egf prot_k3_512 oracle")
    s0, r0, _, _ = oracle_align_egf(job.seqs, job.sub, job.gap)
    dev = msa.DeviceAligner(job.lens, job.sub, job.gap, end_gaps_free=True)
    dev.set_sequences(job.seqs)
    dev.run()
    s1, r1 = dev.result()
    assert s1 == s0 and np.array_equal(r1, r0)


@pytest.mark.parametrize("variant", [1, 2])
def test_egf_k3_both_fills(variant):
    """k = 3 end-gap-free through the streaming fill (variant 1) and the tile
    fill (variant 2), forced through the tuner table: full decision tensor
    equal to the oracle's, shapes spanning several 8 x 64 workgroups and
    16^3 tiles with ragged tails."""
    rng = np.random.Generator(np.random.PCG64(7400 + variant))
    sub, gap = protein_scoring()
    try:
        for lens in ((70, 130, 45), (9, 64, 17), (17, 1, 33), (33, 65, 0)):
            msa.tune_set(msa.MSA_TUNE_PLAIN, 3, max(lens), variant, 0)
            seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in lens]
            check_egf(seqs, sub, gap)
    finally:
        msa.tune_clear()
