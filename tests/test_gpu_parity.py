"""GPU parity: the HIP path against the oracle, bit-exact.

Everything is integer, so the bar is equality: score, alignment rows and the
full decision tensor (every cell's chosen neighbour mask) on seeded inputs
that span several tiles with ragged tails, the edge cases (empty sequences,
lengths at tile boundaries, maximum k), and the full-size workloads against
stored oracle results (tests/golden/workloads.json, written by
tests/golden/make_golden.py from the oracle only).
"""
import hashlib
import json
import sys
from pathlib import Path

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import dna_scoring, protein_scoring, workload
from oracle import oracle_align

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden"


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


def rand_case(rng, k, nmax, protein):
    sub, gap = protein_scoring() if protein else dna_scoring()
    alpha = sub.shape[0]
    seqs = [rng.integers(0, alpha, size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
            for _ in range(k)]
    return seqs, sub, gap


def check_device(seqs, sub, gap, want_dir=True):
    lens = [len(s) for s in seqs]
    say("case k=%d lens=%s gap=%d" % (len(seqs), lens, gap))
    s0, r0, d0 = oracle_align(seqs, sub, gap, want_dir=want_dir)
    dev = msa.DeviceAligner(lens, sub, gap)
    dev.set_sequences(seqs)
    dev.run()
    s1, r1 = dev.result()
    assert s1 == s0, (lens, s1, s0)
    assert np.array_equal(r1, r0), lens
    if want_dir:
        d1 = dev.export_dirs()
        assert np.array_equal(d1, d0), (lens, np.argwhere(d1 != d0)[:5])
    return dev


# lengths per k: several tiles per dimension plus a ragged tail
NMAX = {2: 75, 3: 37, 4: 19, 5: 12, 6: 7, 7: 5, 8: 3}


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
def test_random_shapes_full_tensor(k):
    rng = np.random.Generator(np.random.PCG64(1000 + k))
    for trial in range(4):
        seqs, sub, gap = rand_case(rng, k, NMAX[k], protein=bool(trial % 2))
        check_device(seqs, sub, gap)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_tile_boundary_lengths(k):
    T = msa.tile_edge(k)
    rng = np.random.Generator(np.random.PCG64(2000 + k))
    sub, gap = protein_scoring()
    for lens in ([T] * k, [T + 1] * k, [2 * T] * k, [1] + [T - 1] * (k - 1),
                 [0] + [T + 2] * (k - 1), [2 * T + 1] + [1] * (k - 1)):
        seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in lens]
        check_device(seqs, sub, gap)


def test_three_sequence_column_shapes():
    # Three sequences run as columns along dimension 0, swept in one pass with
    # a ring of layers: long first sequences wrap the ring many times, short
    # ones end inside a tile, and ragged or empty cross-sections change the
    # skew of each column.
    rng = np.random.Generator(np.random.PCG64(2500))
    for lens in ([150, 20, 19], [151, 33, 1], [7, 40, 35], [16, 16, 48], [0, 30, 45],
                 [97, 0, 17], [1, 1, 1], [200, 5, 3], [33, 17, 0]):
        protein = bool(sum(lens) % 2)
        sub, gap = protein_scoring() if protein else dna_scoring()
        seqs = [rng.integers(0, sub.shape[0], size=n).astype(np.uint8) for n in lens]
        check_device(seqs, sub, gap)


def test_empty_and_degenerate():
    sub, gap = dna_scoring()
    e = np.zeros(0, np.uint8)
    a = np.array([0, 1, 2, 3, 0], np.uint8)
    for seqs in ([e, e], [e, e, e], [a, e], [e, a, e], [a[:1], a[:1]], [a, a, a],
                 [a] * 8, [a[:2], e, a[:1], e, a[:3], e, a, e]):
        check_device(seqs, sub, gap)


def test_host_buffer_path_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(3000))
    for k in (2, 3, 4, 5):
        seqs, sub, gap = rand_case(rng, k, NMAX[k], protein=True)
        say("host path k=%d lens=%s" % (k, [len(s) for s in seqs]))
        s0, r0, _ = oracle_align(seqs, sub, gap)
        s1, r1 = msa.align(seqs, sub, gap)
        assert s1 == s0 and np.array_equal(r1, r0)


def test_other_scoring_values():
    rng = np.random.Generator(np.random.PCG64(4000))
    for gap in (-1, 0, 3):
        m = rng.integers(-6, 7, size=(5, 5))
        sub = (np.triu(m) + np.triu(m, 1).T).astype(np.int8)
        seqs = [rng.integers(0, 5, size=int(rng.integers(5, 30))).astype(np.uint8)
                for _ in range(3)]
        check_device(seqs, sub, gap)


def test_repeated_runs_same_workspace():
    job = workload("dna_k3_40")
    dev = check_device(job.seqs, job.sub, job.gap)
    first = dev.result()
    for _ in range(5):
        dev.run()
    s, r = dev.result()
    assert s == first[0] and np.array_equal(r, first[1])


def test_device_detects_bad_code():
    sub, gap = dna_scoring()
    seqs = [np.array([0, 1, 2], np.uint8), np.array([1, 2, 3], np.uint8)]
    dev = msa.DeviceAligner([3, 3], sub, gap)
    bad = [np.array([0, 9, 2], np.uint8), seqs[1]]
    dev.set_sequences(bad)
    dev.run()
    with pytest.raises(msa.MsaError) as e:
        dev.result()
    assert e.value.status == msa.MSA_EINVAL
    dev.set_sequences(seqs)  # the workspace stays usable
    dev.run()
    s, r = dev.result()
    s0, r0, _ = oracle_align(seqs, sub, gap)
    assert s == s0 and np.array_equal(r, r0)


@pytest.mark.parametrize("name", ["dna_k3_40", "prot_k3_512", "prot_k4_128"])
def test_full_size_workloads_against_stored_oracle(name):
    gold = json.loads((GOLDEN / "workloads.json").read_text())[name]
    job = workload(name)
    say("workload", name, job.lens)
    dev = msa.DeviceAligner(job.lens, job.sub, job.gap)
    dev.set_sequences(job.seqs)
    dev.run()
    s, rows = dev.result()
    assert s == gold["score"]
    assert rows.shape[1] == gold["aln_len"]
    assert hashlib.sha256(np.ascontiguousarray(rows).tobytes()).hexdigest() == gold["rows_sha256"]
    d = dev.export_dirs()
    assert hashlib.sha256(np.ascontiguousarray(d).tobytes()).hexdigest() == gold["dir_sha256"]


def test_workspace_prepared_for_other_lengths_is_refused():
    # a workspace prepared for one shape: a call with other lengths (that
    # need no more bytes) returns MSA_EINVAL at once and enqueues nothing
    import ctypes
    from paper_2311_17530_amd._lib import _i32arr
    sub, gap = dna_scoring()
    dev = msa.DeviceAligner([20, 20, 20], sub, gap)
    dev.set_sequences([np.zeros(20, np.uint8)] * 3)
    dev.run()
    s0, _ = dev.result()
    other = [20, 19, 20]
    assert msa.workspace_bytes(other) <= dev.ws_bytes
    rc = msa.lib().msa_dp_align_dev(dev.ws_ptr, dev.ws_bytes, dev.d_seqs.data_ptr(),
                                    _i32arr(other), 3, dev.d_score.data_ptr(),
                                    dev.d_aln.data_ptr(), dev.cap, dev.d_len.data_ptr(),
                                    dev.d_status.data_ptr(), ctypes.c_void_p(dev._stream()))
    assert rc == msa.MSA_EINVAL
    dev.run()  # the prepared shape still runs
    assert dev.result()[0] == s0


def test_streaming_k3_block_edges():
    # The k=3 fill streams lines of 24 rows (three per compute wave) x 64
    # lanes per workgroup: rows and lanes that end one before, on and one
    # after a workgroup or wave edge, several workgroups per dimension, long
    # and empty third sequences, and a gap > 0 (candidate keys that grow) --
    # every cell's decision compared.
    rng = np.random.Generator(np.random.PCG64(2600))
    for lens in ([7, 63, 20], [8, 64, 21], [9, 65, 5], [23, 130, 40], [40, 129, 90],
                 [1, 200, 15], [70, 1, 30], [15, 62, 300], [0, 64, 64], [16, 0, 9],
                 [31, 127, 0], [22, 66, 13], [24, 63, 29], [47, 70, 11], [48, 65, 3]):
        protein = bool(sum(lens) % 2)
        sub, gap = protein_scoring() if protein else dna_scoring()
        seqs = [rng.integers(0, sub.shape[0], size=n).astype(np.uint8) for n in lens]
        check_device(seqs, sub, gap)
    m = rng.integers(-5, 6, size=(4, 4))
    sub = (np.triu(m) + np.triu(m, 1).T).astype(np.int8)
    seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in (25, 70, 33)]
    check_device(seqs, sub, 2)
    # cell (9, 64, 0) takes mask 3 from the left workgroup's halo value of
    # the row above at t = 0 (lane 0, the slot written before step 0)
    r5 = np.random.Generator(np.random.PCG64(5))
    sub, gap = protein_scoring()
    seqs = [r5.integers(0, 20, size=n).astype(np.uint8) for n in (10, 66, 1)]
    check_device(seqs, sub, gap)


def test_streaming_k3_repeated_launches_and_new_sequences():
    # Exchange values carry the launch's epoch: repeated launches on one
    # workspace, with new sequences of the same shape in between, each equal
    # to the oracle.
    rng = np.random.Generator(np.random.PCG64(2700))
    sub, gap = protein_scoring()
    lens = [33, 100, 50]
    dev = msa.DeviceAligner(lens, sub, gap)
    for rep in range(9):
        seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in lens]
        say("launch", rep)
        dev.set_sequences(seqs)
        dev.run()
        s1, r1 = dev.result()
        s0, r0, _ = oracle_align(seqs, sub, gap)
        assert s1 == s0 and np.array_equal(r1, r0)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_streaming_k3_detects_bad_code(which):
    # A residue code >= alpha in any of the three sequences makes the k=3
    # fill report MSA_EINVAL; the workspace stays usable afterwards.
    rng = np.random.Generator(np.random.PCG64(2800 + which))
    sub, gap = dna_scoring()
    lens = [20, 70, 30]
    seqs = [rng.integers(0, 4, size=n).astype(np.uint8) for n in lens]
    dev = msa.DeviceAligner(lens, sub, gap)
    bad = [s.copy() for s in seqs]
    bad[which][lens[which] // 2] = 7
    dev.set_sequences(bad)
    dev.run()
    with pytest.raises(msa.MsaError) as e:
        dev.result()
    assert e.value.status == msa.MSA_EINVAL
    dev.set_sequences(seqs)
    dev.run()
    s, r = dev.result()
    s0, r0, _ = oracle_align(seqs, sub, gap)
    assert s == s0 and np.array_equal(r, r0)


def test_second_fill_without_traceback_finds_no_work():
    # The traceback re-arms the work counter; a fill launched twice in a row
    # finds no work the second time and ends, and the next whole alignment is
    # correct again.
    rng = np.random.Generator(np.random.PCG64(2900))
    sub, gap = protein_scoring()
    for lens in ([30, 90, 40], [20, 20, 20, 20]):
        seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in lens]
        dev = msa.DeviceAligner(lens, sub, gap)
        dev.set_sequences(seqs)
        say("double fill", lens)
        dev.run_fill()
        dev.run_fill()
        dev.run_traceback()
        dev.run()
        s, r = dev.result()
        s0, r0, _ = oracle_align(seqs, sub, gap)
        assert s == s0 and np.array_equal(r, r0)
