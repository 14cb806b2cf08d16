"""GPU tests of the batched and served paths.

Every job's result must equal (a) the oracle and (b) the same job run alone
through the plain path, bit for bit.  The 4096-job workload (k in {3,4},
lengths 16..160, DNA and protein) runs in the same batched launches the
benchmark times and every job is compared with the plain path (itself pinned
to the oracle's full decision tensors); its largest job is compared with the
oracle's stored score and row hash and its smallest jobs with the oracle
directly.  4000 jobs of the served mix go through the server and are
compared with the plain path one by one.
"""
import time

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import batch_jobs, dna_scoring, protein_scoring, served_jobs
from oracle import oracle_align

pytestmark = pytest.mark.gpu

GAP = 0xFF


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    msa.lib()
    yield


def sp_numpy(rows, sub, gap):
    rows = np.asarray(rows, dtype=np.int64)
    k, L = rows.shape
    sub = np.asarray(sub, dtype=np.int64)
    s = 0
    for i in range(k):
        for j in range(i + 1, k):
            a, b = rows[i], rows[j]
            ga, gb = a == GAP, b == GAP
            both = ~ga & ~gb
            s += int(sub[a[both], b[both]].sum())
            s += gap * int((ga ^ gb).sum())
    return s


def check_props(seqs, sub, gap, score, rows):
    k = len(seqs)
    assert rows.shape[0] == k
    for i in range(k):
        assert np.array_equal(rows[i][rows[i] != GAP], np.asarray(seqs[i]))
    assert sp_numpy(rows, sub, gap) == score


def small_mixed(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for _ in range(n):
        k = int(rng.integers(2, 6))
        prot = bool(rng.integers(0, 2))
        sub, gap = protein_scoring() if prot else dna_scoring()
        nmax = {2: 70, 3: 30, 4: 14, 5: 8}[k]
        seqs = [rng.integers(0, sub.shape[0], size=int(rng.integers(0, nmax + 1))).astype(np.uint8)
                for _ in range(k)]
        jobs.append((seqs, sub, gap))
    return jobs


def test_batch_matches_oracle_and_plain_path():
    jobs = small_mixed(5000, 40)
    say("batch of", len(jobs))
    res = msa.align_batch(jobs)
    for (seqs, sub, gap), (st, score, rows) in zip(jobs, res):
        assert st == msa.MSA_OK
        s0, r0, _ = oracle_align(seqs, sub, gap)
        assert score == s0 and np.array_equal(rows, r0), [len(s) for s in seqs]
        s1, r1 = msa.align(seqs, sub, gap)
        assert s1 == score and np.array_equal(r1, rows)


def test_batch_graph_replays_and_permuted_queue_order():
    # Every batched launch replays the launch sequence captured once per arena
    # and k class.  Replays with other device work and synchronisations in
    # between give the plain path's bytes, batch after batch and for batches
    # of other sizes, and so does any order of the jobs: jobs of equal k and
    # scoring keep the caller's order, so a permutation reorders the column
    # queue inside every computation wave.
    import torch
    jobs = small_mixed(5100, 60)
    plain = [msa.align(*j) for j in jobs]
    rng = np.random.Generator(np.random.PCG64(5101))
    for rep, size in enumerate((60, 60, 60, 7, 1, 33)):
        perm = rng.permutation(len(jobs)) if rep else np.arange(len(jobs))
        perm = perm[:size]
        say("batch replay", rep, "jobs", size)
        res = msa.align_batch([jobs[i] for i in perm])
        assert len(res) == size
        for i, (st, score, rows) in zip(perm, res):
            assert st == msa.MSA_OK
            assert score == plain[i][0] and np.array_equal(rows, plain[i][1]), (rep, int(i))
        s, r = msa.align(*jobs[rep])  # eager work between the replays
        torch.cuda.synchronize()
        assert s == plain[rep][0] and np.array_equal(r, plain[rep][1])


def test_batch_small_budget_splits_launches():
    jobs = small_mixed(5001, 30)
    say("batch with small budget")
    full = msa.align_batch(jobs)
    split = msa.align_batch(jobs, hbm_budget_bytes=24 << 20)
    for a, b in zip(full, split):
        assert a[0] == b[0] == msa.MSA_OK
        assert a[1] == b[1] and np.array_equal(a[2], b[2])


def test_batch_reports_per_job_errors():
    sub, gap = dna_scoring()
    good = [np.array([0, 1, 2, 3], np.uint8), np.array([0, 2, 3], np.uint8)]
    bad = [np.array([0, 9], np.uint8), np.array([1], np.uint8)]  # code >= alpha
    res = msa.align_batch([(good, sub, gap), (bad, sub, gap), (good * 2, sub, gap)])
    assert res[0][0] == msa.MSA_OK and res[2][0] == msa.MSA_OK
    assert res[1][0] == msa.MSA_EINVAL
    s0, r0, _ = oracle_align(good, sub, gap)
    assert res[0][1] == s0 and np.array_equal(res[0][2], r0)


def _golden_largest():
    import json
    from pathlib import Path
    doc = json.loads((Path(__file__).resolve().parent / "golden" / "workloads.json").read_text())
    return doc["batch_4096_largest"]


def test_batch_4096_workload():
    """Every one of the 4096 batched jobs equals the plain path bit for bit
    (score and rows); the plain path is itself pinned to the oracle's full
    decision tensors.  The largest job (by cells) also equals the oracle's
    stored score and row hash, and the smallest jobs the oracle directly."""
    import hashlib
    jobs = batch_jobs(4096)
    tuples = [(j.seqs, j.sub, j.gap) for j in jobs]
    say("batch 4096 jobs, cells", sum(j.cells for j in jobs))
    t0 = time.time()
    res = msa.align_batch(tuples)
    say("batch 4096 done in %.2f s" % (time.time() - t0))
    assert all(r[0] == msa.MSA_OK for r in res)
    t0 = time.time()
    equal = 0
    for i, (seqs, sub, gap) in enumerate(tuples):
        s1, r1 = msa.align(seqs, sub, gap)
        if s1 == res[i][1] and np.array_equal(r1, res[i][2]):
            equal += 1
        else:
            say("batched job differs from the plain path:", i, [len(s) for s in seqs])
    say("plain path on 4096 jobs in %.2f s" % (time.time() - t0))
    assert equal == len(tuples)
    g = _golden_largest()
    i = g["job_index"]
    assert list(jobs[i].lens) == g["lens"]
    rows = np.ascontiguousarray(res[i][2])
    assert res[i][1] == g["score"] and rows.shape[1] == g["aln_len"]
    assert hashlib.sha256(rows.tobytes()).hexdigest() == g["rows_sha256"]
    # the oracle itself on the smallest jobs
    order = np.argsort([j.cells for j in jobs])
    for i in list(order[:8]):
        seqs, sub, gap = tuples[i]
        s0, r0, _ = oracle_align(seqs, sub, gap)
        assert res[i][1] == s0 and np.array_equal(res[i][2], r0)


def test_server_alone_equals_mixed():
    jobs = small_mixed(6000, 24)
    probe = jobs[3]
    with msa.Server(hbm_budget_bytes=1 << 30, max_inflight=3, max_jobs_per_launch=8) as srv:
        t = srv.submit(*probe)
        alone = srv.wait(t, 30_000_000)
        tickets = [srv.submit(*j) for j in jobs]
        mixed = [srv.wait(t, 30_000_000) for t in tickets]
    assert alone[0] == msa.MSA_OK
    assert mixed[3][1] == alone[1] and np.array_equal(mixed[3][2], alone[2])
    for (seqs, sub, gap), (st, score, rows) in zip(jobs, mixed):
        assert st == msa.MSA_OK
        s0, r0, _ = oracle_align(seqs, sub, gap)
        assert score == s0 and np.array_equal(rows, r0)


def test_server_stream_of_served_jobs():
    """4000 jobs of the served mix through the server, every one equal to the
    same job run alone through the plain path (score and rows)."""
    jobs = served_jobs(4000, seed=5)
    with msa.Server(max_inflight=4, max_jobs_per_launch=64) as srv:
        tickets = []
        for j in jobs:
            tickets.append(srv.submit(j.seqs, j.sub, j.gap))
        out = [srv.wait(t, 60_000_000) for t in tickets]
        stats = srv.stats()
    bad = {}
    for i, o in enumerate(out):
        if o is None or o[0] != msa.MSA_OK:
            key = "timeout" if o is None else o[0]
            bad.setdefault(key, []).append(i)
    assert not bad, ({s: (len(v), v[:8]) for s, v in bad.items()}, stats)
    t0 = time.time()
    equal = 0
    for j, (_, score, rows) in zip(jobs, out):
        s1, r1 = msa.align(j.seqs, j.sub, j.gap)
        equal += int(s1 == score and np.array_equal(r1, rows))
    say("plain path on %d served jobs in %.2f s" % (len(jobs), time.time() - t0))
    assert equal == len(jobs)
    small = sorted(range(len(jobs)), key=lambda i: jobs[i].cells)[:5]
    for i in small:
        s0, r0, _ = oracle_align(jobs[i].seqs, jobs[i].sub, jobs[i].gap)
        assert out[i][1] == s0 and np.array_equal(out[i][2], r0)


def test_server_reruns_a_launch_that_timed_out():
    """Time-out handling, forced from the host: the first launches of the
    server give up a dependency wait after one tick of the 100 MHz clock
    (every kernel still exits normally).  Their jobs are re-run once and
    return the plain path's alignment; with the short limit on every launch,
    a job whose second launch times out returns MSA_EDEVICE."""
    jobs = served_jobs(400, seed=9)
    plain = [msa.align(j.seqs, j.sub, j.gap) for j in jobs]
    with msa.Server(max_inflight=2, max_jobs_per_launch=64) as srv:
        srv.debug_wait_limit(1, 2)
        tickets = [srv.submit(j.seqs, j.sub, j.gap) for j in jobs[:200]]
        out = [srv.wait(t, 60_000_000) for t in tickets]
        stats = srv.stats()
    say("forced time-outs, first launches only: %s" % stats)
    assert stats["rerun"] > 0 and stats["failed"] == 0, stats
    for (st, score, rows), (s1, r1) in zip(out, plain):
        assert st == msa.MSA_OK and score == s1 and np.array_equal(rows, r1)
    with msa.Server(max_inflight=2, max_jobs_per_launch=64) as srv:
        srv.debug_wait_limit(1, 1 << 20)
        tickets = [srv.submit(j.seqs, j.sub, j.gap) for j in jobs]
        out = [srv.wait(t, 60_000_000) for t in tickets]
        stats = srv.stats()
    say("forced time-outs, every launch: %s" % stats)
    st = [o[0] for o in out]
    assert set(st) <= {msa.MSA_OK, msa.MSA_EDEVICE}, set(st)
    assert st.count(msa.MSA_EDEVICE) == stats["failed"] > 0 and stats["rerun"] > 0, stats
    for (s, score, rows), (s1, r1) in zip(out, plain):
        if s == msa.MSA_OK:
            assert score == s1 and np.array_equal(rows, r1)


def test_server_errors_and_shutdown():
    sub, gap = dna_scoring()
    with msa.Server(hbm_budget_bytes=64 << 20, max_inflight=2) as srv:
        with pytest.raises(msa.MsaError) as e:
            srv.submit([np.array([0, 9], np.uint8), np.array([1], np.uint8)], sub, gap)
        assert e.value.status == msa.MSA_EINVAL
        with pytest.raises(msa.MsaError) as e:  # alone larger than a slot's budget
            big = [np.zeros(400, np.uint8)] * 4
            srv.submit(big, sub, gap)
        assert e.value.status == msa.MSA_ENOMEM
        assert msa.lib().msa_server_poll(srv.h, 987654321, None) == msa.MSA_EINVAL
        t = srv.submit([np.array([0, 1], np.uint8), np.array([1], np.uint8)], sub, gap)
        r = srv.wait(t, 30_000_000)
        assert r[0] == msa.MSA_OK
    # destroy with work still queued or running must not hang
    srv = msa.Server(max_inflight=2)
    for _ in range(10):
        srv.submit(*small_mixed(6100, 1)[0])
    srv.close()
