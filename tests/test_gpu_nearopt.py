"""GPU parity of the near-optimal mode (MSA_NEAROPT, k <= 6) against the
oracle's enumeration (every global alignment scoring at least opt - delta,
Section 6), bit-exact: the optimum, and the ordered list of alignments with
their scores, up to a limit.  Shapes span several tiles with ragged tails for
every k; delta = 0 is compared with the device's co-optimal list; the 513^3
protein workload is checked for its first 16 alignments within 20 of the
optimum.
"""
import sys

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import dna_scoring, protein_scoring, workload
from oracle import oracle_align, oracle_nearopt

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


def check_nearopt(seqs, sub, gap, delta, max_paths, dev=None):
    lens = [len(s) for s in seqs]
    say("nearopt case k=%d lens=%s delta=%d max_paths=%d" % (len(seqs), lens, delta, max_paths))
    opt0, want = oracle_nearopt(seqs, sub, gap, delta, max_paths)
    if dev is None:
        dev = msa.DeviceAligner(lens, sub, gap, nearopt=True)
    dev.set_sequences(seqs)
    dev.run_nearopt(delta, max_paths)
    opt1, got = dev.result_nearopt()
    assert opt1 == opt0, (lens, opt1, opt0)
    assert len(got) == len(want), (lens, delta, len(got), len(want))
    for p, ((s1, r1), (s0, r0)) in enumerate(zip(got, want)):
        assert s1 == s0 and np.array_equal(r1, r0), (lens, delta, p)
    return dev, got


NMAX = {2: 70, 3: 35, 4: 17, 5: 9, 6: 5}


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
def test_nearopt_random_shapes(k):
    rng = np.random.Generator(np.random.PCG64(9100 + k))
    for trial in range(4):
        sub, gap = protein_scoring() if trial % 2 else dna_scoring()
        seqs = [rng.integers(0, sub.shape[0], size=int(rng.integers(1, NMAX[k] + 1))).astype(
            np.uint8) for _ in range(k)]
        delta = [0, 3, 12, 40][trial]
        check_nearopt(seqs, sub, gap, delta, 40)


def test_nearopt_delta_zero_is_device_coopt_list():
    rng = np.random.Generator(np.random.PCG64(9200))
    sub, gap = dna_scoring()
    for lens in ([40, 33], [20, 18, 21]):
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
        _, got = check_nearopt(seqs, sub, gap, 0, 64)
        co = msa.DeviceAligner(lens, sub, gap, cooptimal=True)
        co.set_sequences(seqs)
        co.run_coopt(64)
        s, rows = co.result_coopt()
        assert len(rows) == len(got)
        for (sc, r1), r0 in zip(got, rows):
            assert sc == s and np.array_equal(r1, r0)


def test_nearopt_edges():
    sub, gap = dna_scoring()
    rng = np.random.Generator(np.random.PCG64(9300))
    # empty sequences, one empty among others, a limit of one, every alignment
    check_nearopt([np.zeros(0, np.uint8)] * 3, sub, gap, 5, 4)
    check_nearopt([np.zeros(0, np.uint8), rng.integers(0, 4, 7).astype(np.uint8),
                   rng.integers(0, 4, 5).astype(np.uint8)], sub, gap, 6, 30)
    seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in (30, 29, 31)]
    check_nearopt(seqs, sub, gap, 10, 1)
    tiny = [rng.integers(0, 4, size=n).astype(np.uint8) for n in (3, 2, 2)]
    _, got = check_nearopt(tiny, sub, gap, 10 ** 6, 5000)
    from oracle.brute import count_alignments
    assert len(got) == count_alignments([3, 2, 2])
    # the same workspace again with other sequences and thresholds (epochs)
    dev = None
    for delta in (0, 7, 2):
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in (25, 40, 18)]
        dev, _ = check_nearopt(seqs, sub, gap, delta, 25, dev)
    # the plain alignment on a near-optimal workspace is the plain one
    dev.run()
    s1, r1 = dev.result()
    s0, r0, _ = oracle_align(seqs, sub, gap)
    assert s1 == s0 and np.array_equal(r1, r0)


def test_nearopt_host_path_and_unprepared_workspace():
    sub, gap = protein_scoring()
    rng = np.random.Generator(np.random.PCG64(9400))
    seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in (14, 12, 15, 13)]
    opt0, want = oracle_nearopt(seqs, sub, gap, 15, 30)
    opt1, got = msa.align_nearopt(seqs, sub, gap, 15, 30)
    assert opt1 == opt0 and len(got) == len(want)
    for (s1, r1), (s0, r0) in zip(got, want):
        assert s1 == s0 and np.array_equal(r1, r0)
    # a workspace prepared for the plain mode is too small for the cell scores
    plain = msa.DeviceAligner([14, 12, 15, 13], sub, gap)
    plain.set_sequences(seqs)
    with pytest.raises(msa.MsaError) as e:
        plain.run_nearopt(5, 4)
    assert e.value.status == msa.MSA_EINVAL


def test_nearopt_full_size_protein_k3():
    job = workload("prot_k3_512")
    check_nearopt(job.seqs, job.sub, job.gap, 20, 16)


def test_coopt_k4_to_6_through_the_nearopt_walk():
    # msa_dp_align_coopt for k = 4..6 lists the delta = 0 alignments
    rng = np.random.Generator(np.random.PCG64(9500))
    sub, gap = dna_scoring()
    for lens in ([12, 10, 11, 9], [6, 7, 5, 6, 7], [4, 3, 4, 4, 3, 4]):
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
        say("coopt via nearopt lens=%s" % lens)
        opt0, want = oracle_nearopt(seqs, sub, gap, 0, 50)
        s1, rows = msa.align_coopt(seqs, sub, gap, 50)
        assert s1 == opt0 and len(rows) == len(want)
        for r1, (s0, r0) in zip(rows, want):
            assert s0 == opt0 and np.array_equal(r1, r0)
