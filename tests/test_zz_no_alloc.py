"""GPU test of msa_dp_align_static, the entry point that allocates nothing
(its workspace is a file-scope device array set up by a kernel).

Two calls in a row, the second with a smaller input, each compared bit for
bit (score and rows) with msa_dp_align_dev on a caller workspace and with the
oracle; then the limits that are refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from paper_2311_17530_amd._lib import _i32arr
from msa_inputs import protein_scoring, workload
from oracle import oracle_align

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    msa.lib()
    yield


def run_static(seqs, sub, gap):
    import torch
    lens = [len(s) for s in seqs]
    k = len(seqs)
    cap = max(1, sum(lens))
    flat = np.concatenate([np.asarray(s, np.uint8) for s in seqs]) if sum(lens) else \
        np.zeros(1, np.uint8)
    d_seqs = torch.from_numpy(flat).cuda()
    d_aln = torch.full((k, cap), 0xFF, dtype=torch.uint8, device="cuda")
    d_score = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_len = torch.zeros(1, dtype=torch.int64, device="cuda")
    d_status = torch.full((1,), -99, dtype=torch.int32, device="cuda")
    sub8 = np.ascontiguousarray(np.asarray(sub, np.int8))
    stream = torch.cuda.current_stream().cuda_stream
    rc = msa.lib().msa_dp_align_static(d_seqs.data_ptr(), _i32arr(lens), k, sub8.ctypes.data,
                                       sub8.shape[0], int(gap), d_score.data_ptr(),
                                       d_aln.data_ptr(), cap, d_len.data_ptr(),
                                       d_status.data_ptr(), ctypes.c_void_p(stream))
    assert rc == msa.MSA_OK, rc
    torch.cuda.synchronize()
    assert int(d_status.item()) == msa.MSA_OK
    L = int(d_len.item())
    return int(d_score.item()), d_aln[:, :L].cpu().numpy()


def run_dev(seqs, sub, gap):
    dev = msa.DeviceAligner([len(s) for s in seqs], sub, gap)
    dev.set_sequences(seqs)
    dev.run()
    return dev.result()


def test_static_entry_point_two_calls_second_smaller():
    big = workload("dna_k3_40")
    rng = np.random.Generator(np.random.PCG64(901))
    sub, gap = protein_scoring()
    small = [rng.integers(0, 20, size=n).astype(np.uint8) for n in (23, 17, 29)]
    for name, (seqs, s, g) in (("41^3 DNA", (big.seqs, big.sub, big.gap)),
                               ("24x18x30 protein", (small, sub, gap))):
        say("static call:", name)
        got = run_static(seqs, s, g)
        ref = run_dev(seqs, s, g)
        s0, r0, _ = oracle_align(seqs, s, g)
        assert got[0] == ref[0] == s0
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[1], r0)


def test_static_entry_point_k4_after_k3():
    rng = np.random.Generator(np.random.PCG64(902))
    sub, gap = protein_scoring()
    seqs = [rng.integers(0, 20, size=n).astype(np.uint8) for n in (12, 9, 14, 11)]
    say("static call: k=4 13x10x15x12")
    got = run_static(seqs, sub, gap)
    s0, r0, _ = oracle_align(seqs, sub, gap)
    assert got[0] == s0 and np.array_equal(got[1], r0)


def test_static_limits_refused_before_device():
    sub, gap = protein_scoring()
    sub8 = np.ascontiguousarray(sub.astype(np.int8))
    dummy = ctypes.c_void_p(1 << 20)
    lib = msa.lib()
    # workspace beyond the 32 MiB array
    rc = lib.msa_dp_align_static(dummy, _i32arr([400, 400, 400]), 3, sub8.ctypes.data, 20, gap,
                                 dummy, dummy, 1200, dummy, dummy, None)
    assert rc == msa.MSA_ENOMEM
    # matrices beyond 32 x 32 do not travel by value
    big = np.zeros((40, 40), np.int8)
    rc = lib.msa_dp_align_static(dummy, _i32arr([4, 4]), 2, big.ctypes.data, 40, -1,
                                 dummy, dummy, 8, dummy, dummy, None)
    assert rc == msa.MSA_EINVAL
