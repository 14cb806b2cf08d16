"""GPU parity of the co-optimal mode (MSA_COOPTIMAL, k <= 3) against the
oracle's co-optimal enumeration, bit-exact: the optimal score, the tie set of
every cell (exported from the device) and the ordered list of co-optimal
alignments, up to a limit.  Shapes span several tiles with ragged tails; the
513^3 protein workload is checked in full (tie tensor and the first 16
alignments).
"""
import sys

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import dna_scoring, protein_scoring, workload
from oracle import oracle_align, oracle_coopt

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


def check_coopt(seqs, sub, gap, max_paths, want_ties=True):
    lens = [len(s) for s in seqs]
    say("coopt case k=%d lens=%s max_paths=%d" % (len(seqs), lens, max_paths))
    s0, rows0, t0 = oracle_coopt(seqs, sub, gap, max_paths, want_ties=want_ties)
    dev = msa.DeviceAligner(lens, sub, gap, cooptimal=True)
    dev.set_sequences(seqs)
    dev.run_coopt(max_paths)
    s1, rows1 = dev.result_coopt()
    assert s1 == s0, (lens, s1, s0)
    assert len(rows1) == len(rows0), (lens, len(rows1), len(rows0))
    for p, (a, b) in enumerate(zip(rows1, rows0)):
        assert np.array_equal(a, b), (lens, p)
    if want_ties:
        t1 = dev.export_dirs()
        assert np.array_equal(t1, t0), (lens, np.argwhere(t1 != t0)[:5])
    return dev, s0, rows0


NMAX = {2: 75, 3: 37}


@pytest.mark.parametrize("k", [2, 3])
def test_coopt_random_shapes(k):
    rng = np.random.Generator(np.random.PCG64(8000 + k))
    for trial in range(5):
        sub, gap = protein_scoring() if trial % 2 else dna_scoring()
        seqs = [rng.integers(0, sub.shape[0], size=int(rng.integers(0, NMAX[k] + 1))).astype(
            np.uint8) for _ in range(k)]
        check_coopt(seqs, sub, gap, max_paths=int(rng.integers(1, 40)))


@pytest.mark.parametrize("k", [2, 3])
def test_coopt_tile_boundary_lengths(k):
    T = msa.tile_edge(k)
    rng = np.random.Generator(np.random.PCG64(8100 + k))
    sub, gap = dna_scoring()  # four letters: many ties
    for lens in ([T] * k, [T + 1] * k, [2 * T - 1] + [T] * (k - 1), [1] + [2 * T] * (k - 1)):
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
        check_coopt(seqs, sub, gap, max_paths=64)


def test_coopt_all_alignments_when_few():
    # small inputs whose whole list fits the limit: every co-optimal alignment
    rng = np.random.Generator(np.random.PCG64(8200))
    sub, gap = dna_scoring()
    for _ in range(8):
        k = int(rng.integers(2, 4))
        seqs = [rng.integers(0, 4, size=int(rng.integers(0, 7))).astype(np.uint8)
                for _ in range(k)]
        _, _, rows0 = check_coopt(seqs, sub, gap, max_paths=100000)
        assert len(rows0) < 100000


def test_coopt_degenerate_cases():
    sub, gap = dna_scoring()
    e = np.zeros(0, np.uint8)
    cases = [[e, e], [e, e, e], [np.array([1], np.uint8), e],
             [np.array([1, 2], np.uint8), e, np.array([3], np.uint8)],
             [np.array([0, 0, 0], np.uint8)] * 3]
    for seqs in cases:
        check_coopt(seqs, sub, gap, max_paths=50)


def test_coopt_workspace_plain_traceback_and_host_path():
    # a co-optimal workspace still runs the plain traceback (lowest tied mask)
    # and the host-buffer entry point returns the same list
    sub, gap = protein_scoring()
    rng = np.random.Generator(np.random.PCG64(8300))
    seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in (40, 33, 47)]
    s0, r0, _ = oracle_align(seqs, sub, gap)
    dev = msa.DeviceAligner([len(s) for s in seqs], sub, gap, cooptimal=True)
    dev.set_sequences(seqs)
    dev.run()
    s1, r1 = dev.result()
    assert s1 == s0 and np.array_equal(r1, r0)
    dsub, dgap = dna_scoring()
    for trial in range(3):
        seqs = [rng.integers(0, 4, size=int(rng.integers(5, 30))).astype(np.uint8)
                for _ in range(2 + trial % 2)]
        s0, rows0, _ = oracle_coopt(seqs, dsub, dgap, 25)
        s1, rows1 = msa.align_coopt(seqs, dsub, dgap, 25)
        assert s1 == s0 and len(rows1) == len(rows0)
        assert all(np.array_equal(a, b) for a, b in zip(rows1, rows0))


def test_coopt_on_plain_workspace_reports_einval():
    # direction bytes of a plain workspace are not tie sets: the device status
    # says so and no alignment is returned
    sub, gap = dna_scoring()
    seqs = [np.array([0, 1, 2, 3], np.uint8), np.array([1, 2, 3], np.uint8)]
    dev = msa.DeviceAligner([4, 3], sub, gap)
    dev.set_sequences(seqs)
    dev.run_coopt(4)
    with pytest.raises(msa.MsaError) as e:
        dev.result_coopt()
    assert e.value.status == msa.MSA_EINVAL
    # the workspace still aligns normally afterwards
    dev.run()
    s1, r1 = dev.result()
    s0, r0, _ = oracle_align(seqs, sub, gap)
    assert s1 == s0 and np.array_equal(r1, r0)


def test_coopt_repeat_runs_same_workspace():
    sub, gap = dna_scoring()
    rng = np.random.Generator(np.random.PCG64(8400))
    lens = [30, 26, 35]
    dev = msa.DeviceAligner(lens, sub, gap, cooptimal=True)
    for _ in range(3):
        seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
        s0, rows0, _ = oracle_coopt(seqs, sub, gap, 20)
        dev.set_sequences(seqs)
        dev.run_coopt(20)
        s1, rows1 = dev.result_coopt()
        assert s1 == s0 and len(rows1) == len(rows0)
        assert all(np.array_equal(a, b) for a, b in zip(rows1, rows0))


def test_coopt_dna_k3_40_workload():
    j = workload("dna_k3_40")
    check_coopt(j.seqs, j.sub, j.gap, max_paths=200)


def test_coopt_full_size_protein_k3_512():
    j = workload("prot_k3_512")
    check_coopt(j.seqs, j.sub, j.gap, max_paths=16)
