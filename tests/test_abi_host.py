"""Host-side tests of the C ABI (no GPU needed).

- the shared library loads and exports every function declared in
  include/msa_dp.h;
- the tile-wave enumerator reproduces Table 1 and Table 2 and Eqs. 2-3;
- the closed-form score bounds hold against the oracle;
- argument validation rejects bad input before any device call.
"""
import re
from math import comb
from pathlib import Path

import numpy as np
import pytest

import paper_2311_17530_amd as msa
from msa_inputs import dna_scoring, protein_scoring
from oracle import oracle_align

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "msa_dp.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(msa_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = msa.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(msa.exported_names())


def test_table1_partitions_per_wave():
    # Table 1: unbounded shape, k = 2..9 sequences, waves 1..9; entries are
    # C(w + k - 2, k - 1).  A grid with >= 9 tiles per dimension is unbounded
    # for the first 9 waves.
    table1 = {
        2: [1, 2, 3, 4, 5, 6, 7, 8, 9],
        3: [1, 3, 6, 10, 15, 21, 28, 36, 45],
        4: [1, 4, 10, 20, 35, 56, 84, 120, 165],
        5: [1, 5, 15, 35, 70, 126, 210, 330, 495],
        6: [1, 6, 21, 56, 126, 252, 462, 792, 1287],
        7: [1, 7, 28, 84, 210, 462, 924, 1716, 3003],
        8: [1, 8, 36, 120, 330, 792, 1716, 3432, 6435],
    }
    for k, row in table1.items():
        counts = msa.wave_counts([9] * k)
        assert counts[:9] == row
        assert row == [comb(w + k - 2, k - 1) for w in range(1, 10)]


def test_table2_shape_9999_s3():
    # Table 2: shape (9,9,9,9), partition size S = 3 -> p_i = (9-1)/(3-1) = 4
    # per dimension (Eq. 3), 256 partitions in 13 waves (Eq. 2).
    counts = msa.wave_counts([4, 4, 4, 4])
    assert counts == [1, 4, 10, 20, 31, 40, 44, 40, 31, 20, 10, 4, 1]
    assert sum(counts) == 256  # Eq. 3: prod p_i
    assert len(counts) == 4 + 3 * (4 - 1)  # Eq. 2: p_0 + sum_{i>=1}(p_i - 1)
    assert 9 ** 4 == 6561


def test_library_tile_grid_matches_eq2_eq3():
    # the library's own grid adds the one-cell v_i = 0 layer to the paper's
    # p_i = n_i / T partitions; with that layer removed Eqs. 2-3 hold exactly
    for k in (2, 3, 4, 5):
        T = msa.tile_edge(k)
        lens = [T * m for m in range(1, k + 1)]
        P, waves = msa.tile_grid(lens, T)
        assert P == [1 + n // T for n in lens]
        assert waves == sum(P) - k + 1
        inner = [p - 1 for p in P]
        assert sum(msa.wave_counts(inner)) == int(np.prod(inner))
        assert len(msa.wave_counts(inner)) == inner[0] + sum(p - 1 for p in inner[1:])


def test_score_bounds_hold():
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(30):
        k = int(rng.integers(2, 5))
        sub, gap = (dna_scoring() if rng.integers(0, 2) else protein_scoring())
        alpha = sub.shape[0]
        seqs = [rng.integers(0, alpha, size=int(rng.integers(0, 9))).astype(np.uint8)
                for _ in range(k)]
        lo, hi = msa.score_bounds([len(s) for s in seqs], sub, gap)
        s, _, _ = oracle_align(seqs, sub, gap)
        assert lo <= s <= hi


def test_validation_rejects_before_device():
    sub, gap = dna_scoring()
    a = np.array([0, 1, 2], np.uint8)
    with pytest.raises(msa.MsaError) as e:
        msa.align([a], sub, gap)  # k < 2
    assert e.value.status == msa.MSA_EINVAL
    with pytest.raises(msa.MsaError) as e:
        msa.align([a] * 9, sub, gap)  # k > MAX_K
    assert e.value.status == msa.MSA_EINVAL
    with pytest.raises(msa.MsaError) as e:
        msa.align([a, np.array([4], np.uint8)], sub, gap)  # code >= alpha
    assert e.value.status == msa.MSA_EINVAL
    asym = sub.copy()
    asym[0, 1] = 5
    with pytest.raises(msa.MsaError) as e:
        msa.align([a, a], asym, gap)  # asymmetric matrix
    assert e.value.status == msa.MSA_EINVAL
    big = np.full((4, 4), 127, np.int8)
    with pytest.raises(msa.MsaError) as e:
        msa.align([np.zeros(200000, np.uint8)] * 8, big, -128)  # range check
    assert e.value.status in (msa.MSA_ERANGE, msa.MSA_ENOMEM)


def test_workspace_bytes_and_errors():
    assert msa.workspace_bytes([40, 40, 40]) > 41 ** 3
    with pytest.raises(msa.MsaError):
        msa.workspace_bytes([3])
    with pytest.raises(msa.MsaError):
        msa.workspace_bytes([3, -1])
    assert msa.strerror(msa.MSA_ERANGE).startswith("score range")


def test_mode_flags_rejected_before_device():
    import ctypes
    sub, gap = dna_scoring()
    sub8 = np.ascontiguousarray(sub.astype(np.int8))
    a = np.array([0, 1, 2], np.uint8)
    seqs = [a, a]
    ptrs = (ctypes.c_void_p * 2)(*[s.ctypes.data for s in seqs])
    lens = (ctypes.c_int32 * 2)(3, 3)
    out = np.zeros((2, 6), np.uint8)
    score, alen = ctypes.c_int64(), ctypes.c_int64()
    for flags in (4, 1 | 2):  # an undefined bit; end-gap-free with co-optimal
        rc = msa.lib().msa_dp_align_ex(ptrs, lens, 2, sub8.ctypes.data, 4, gap, flags,
                                       ctypes.byref(score), out.ctypes.data, 6,
                                       ctypes.byref(alen))
        assert rc == msa.MSA_EINVAL
    # end-gap-free keys hold the cell index in 32 bits
    big = [np.zeros(70000, np.uint8)] * 2
    with pytest.raises(msa.MsaError) as e:
        msa.align(big, sub, gap, end_gaps_free=True)
    assert e.value.status == msa.MSA_ERANGE
    ws = 256  # any aligned address: rejected before it is touched
    rc = msa.lib().msa_dp_prepare_ex(ws, 1 << 40, lens, 2, sub8.ctypes.data, 4, gap, 4, None)
    assert rc == msa.MSA_EINVAL


def test_coopt_limits_rejected_before_device():
    # tie sets fit a byte for k <= 3 (the walk's mask stack holds 32768
    # columns); k = 4..6 use the near-optimal walk (4096 columns)
    sub, gap = dna_scoring()
    a = np.array([0, 1, 2], np.uint8)
    with pytest.raises(msa.MsaError) as e:
        msa.align_coopt([a] * 7, sub, gap, 4)  # k = 4..6 go through the near-optimal walk
    assert e.value.status == msa.MSA_EINVAL
    with pytest.raises(msa.MsaError) as e:
        msa.align_coopt([np.zeros(1100, np.uint8)] * 4, sub, gap, 4)
    assert e.value.status == msa.MSA_ERANGE
    with pytest.raises(msa.MsaError) as e:
        msa.align_coopt([a, a], sub, gap, 0)
    assert e.value.status == msa.MSA_EINVAL
    with pytest.raises(msa.MsaError) as e:
        msa.align_coopt([np.zeros(16385, np.uint8)] * 2, sub, gap, 1)
    assert e.value.status == msa.MSA_ERANGE
    with pytest.raises(msa.MsaError) as e:
        _align_ex([a] * 4, sub, gap, msa.MSA_COOPTIMAL)
    assert e.value.status == msa.MSA_EINVAL


def _align_ex(seqs, sub, gap, flags):
    import ctypes
    sub8 = np.ascontiguousarray(np.asarray(sub, np.int8))
    k = len(seqs)
    ptrs = (ctypes.c_void_p * k)(*[s.ctypes.data for s in seqs])
    lens = (ctypes.c_int32 * k)(*[len(s) for s in seqs])
    cap = sum(len(s) for s in seqs)
    out = np.zeros((k, cap), np.uint8)
    score, alen = ctypes.c_int64(), ctypes.c_int64()
    rc = msa.lib().msa_dp_align_ex(ptrs, lens, k, sub8.ctypes.data, sub8.shape[0], gap, flags,
                                   ctypes.byref(score), out.ctypes.data, cap,
                                   ctypes.byref(alen))
    if rc != msa.MSA_OK:
        raise msa.MsaError(rc, "msa_dp_align_ex")


def test_prune_limits_rejected_before_device():
    # pruned mode: 3 <= k <= 6, lengths < 16384, not with end-gap-free
    sub, gap = dna_scoring()
    a = np.array([0, 1, 2], np.uint8)
    for seqs in ([a, a], [a] * 7):
        with pytest.raises(msa.MsaError) as e:
            msa.align(seqs, sub, gap, prune=True)
        assert e.value.status == msa.MSA_EINVAL
    with pytest.raises(msa.MsaError) as e:
        msa.align([np.zeros(16384, np.uint8), a, a], sub, gap, prune=True)
    assert e.value.status == msa.MSA_ERANGE
    with pytest.raises(msa.MsaError) as e:
        _align_ex([a] * 3, sub, gap, msa.MSA_PRUNE | msa.MSA_END_GAPS_FREE)
    assert e.value.status == msa.MSA_EINVAL


def test_prune_workspace_holds_pair_tables():
    # the pruned mode's pairwise tables and queue live in the workspace of
    # every shape it accepts: two int32 tables per pair plus per-tile data
    T = msa.tile_edge(3)
    lens = [40, 33, 47]
    P, _ = msa.tile_grid(lens, T)
    ntiles = int(np.prod(P))
    pairs = [(0, 1), (0, 2), (1, 2)]
    extra = sum(2 * (lens[i] + 1) * (lens[j] + 1) * 4 for i, j in pairs)
    extra += sum(P[i] * P[j] * 4 for i, j in pairs) + ntiles * 5
    base = msa.workspace_bytes([40, 33])  # k = 2: no pruning area
    assert msa.workspace_bytes(lens) >= extra + ntiles * ((T ** 3 + 15) // 16 * 16)
    assert base > 0


def test_pruned_range_covers_minus_infinity_chains():
    # Pruned mode: -infinity halo keys (-2^30) of a kept tile cut off from the
    # origin travel along monotone paths of up to sum(n) cells, one column
    # score (|.| <= colmax = C(k,2) * max(|gap|, max|sub|)) per step, and must
    # stay below every real key (scores >= lo).  The check therefore needs
    # 2^k * (sum(n) * colmax + |lo| + 1) < 2^30 on top of the plain check.
    k = 6
    sub = np.full((4, 4), -127, np.int8)
    np.fill_diagonal(sub, 127)
    gap = -127
    colmax = comb(k, 2) * 127
    # four empty sequences keep the tile grid small; sum(n) is what counts
    for a, fits in ((3302, True), (3303, False)):
        lens = [a, 3303, 0, 0, 0, 0]
        lo, _ = msa.score_bounds(lens, sub, gap)
        need = (2 ** k) * (sum(lens) * colmax + abs(lo) + 1)
        assert (need < 2 ** 30) == fits
        assert msa.check_scoring(lens, sub, gap, 0) == msa.MSA_OK  # plain mode fits both
        want = msa.MSA_OK if fits else msa.MSA_ERANGE
        assert msa.check_scoring(lens, sub, gap, msa.MSA_PRUNE) == want
    # the same range through the entry point that prepares a workspace: the
    # check runs before the (unallocated) workspace is touched
    lens6 = (ctypes_i32(6))(3303, 3303, 0, 0, 0, 0)
    rc = msa.lib().msa_dp_prepare_ex(256, 1 << 40, lens6, k,
                                     np.ascontiguousarray(sub).ctypes.data, 4, gap,
                                     msa.MSA_PRUNE, None)
    assert rc == msa.MSA_ERANGE


def ctypes_i32(n):
    import ctypes
    return ctypes.c_int32 * n


def test_unprepared_or_mismatched_workspace_rejected_before_device():
    # every device-buffer entry point checks that the workspace was prepared
    # for the same shape before it enqueues anything
    import ctypes
    lib = msa.lib()
    fake = 1 << 20  # an aligned address no call has prepared
    lens = (ctypes.c_int32 * 3)(5, 6, 7)
    dummy = ctypes.c_void_p(1 << 21)
    rc = lib.msa_dp_align_dev(fake, 1 << 30, dummy, lens, 3, dummy, dummy, 64, dummy, dummy,
                              None)
    assert rc == msa.MSA_EINVAL
    rc = lib.msa_dp_fill_dev(fake, 1 << 30, dummy, lens, 3, dummy, None)
    assert rc == msa.MSA_EINVAL
    rc = lib.msa_dp_traceback_dev(fake, 1 << 30, dummy, lens, 3, dummy, dummy, 64, dummy, dummy,
                                  None)
    assert rc == msa.MSA_EINVAL
    rc = lib.msa_dp_export_dirs(fake, 1 << 30, lens, 3, dummy, None)
    assert rc == msa.MSA_EINVAL
    rc = lib.msa_dp_coopt_dev(fake, 1 << 30, dummy, lens, 3, 1, dummy, dummy, 64, dummy, dummy,
                              dummy, None)
    assert rc == msa.MSA_EINVAL


def test_nearopt_limits_and_workspace_before_device():
    # near-optimal mode: k <= 6, sum of lengths <= 4096, a mode of its own,
    # delta >= 0, max_paths >= 1; its workspace adds one int32 per cell
    # (padded like the direction blocks) after the plain layout
    sub, gap = dna_scoring()
    a = np.array([0, 1, 2], np.uint8)
    for seqs, delta, mp, want in (([a] * 7, 0, 1, msa.MSA_EINVAL), ([a, a], -1, 1, msa.MSA_EINVAL),
                                  ([a, a], 0, 0, msa.MSA_EINVAL),
                                  ([np.zeros(2049, np.uint8)] * 2, 0, 1, msa.MSA_ERANGE)):
        with pytest.raises(msa.MsaError) as e:
            msa.align_nearopt(seqs, sub, gap, delta, mp)
        assert e.value.status == want
    for lens in ([40, 40, 40], [9, 17, 5, 3], [100, 100]):
        k = len(lens)
        T = msa.tile_edge(k)
        P, _ = msa.tile_grid(lens, T)
        dbs = (T ** k + 15) // 16 * 16
        extra = (int(np.prod(P)) * dbs * 4 + 255) // 256 * 256
        assert msa.workspace_bytes_ex(lens, msa.MSA_NEAROPT) == msa.workspace_bytes(lens) + extra
        assert msa.workspace_bytes_ex(lens, 0) == msa.workspace_bytes(lens)
    for flags in (msa.MSA_NEAROPT | msa.MSA_PRUNE, msa.MSA_NEAROPT | msa.MSA_COOPTIMAL, 16):
        with pytest.raises(msa.MsaError) as e:
            msa.workspace_bytes_ex([10, 10, 10], flags)
        assert e.value.status == msa.MSA_EINVAL
    import ctypes
    sub8 = np.ascontiguousarray(sub.astype(np.int8))
    lens = (ctypes.c_int32 * 3)(10, 10, 10)
    plain = msa.workspace_bytes([10, 10, 10])
    ws = 256  # any aligned address: a workspace too small for the mode is rejected first
    rc = msa.lib().msa_dp_prepare_ex(ws, plain, lens, 3, sub8.ctypes.data, 4, gap,
                                     msa.MSA_NEAROPT, None)
    assert rc == msa.MSA_EINVAL


def test_tuner_table_without_device():
    # the table keys by (architecture, kind, k, length bucket); a bucket holds
    # longest lengths 2^(b-1) .. 2^b - 1; no device is touched
    msa.tune_clear()
    assert msa.tune_get(msa.MSA_TUNE_PLAIN, 3, 512) == (0, 0)
    msa.tune_set(msa.MSA_TUNE_PLAIN, 3, 512, 2, 3)
    assert msa.tune_get(msa.MSA_TUNE_PLAIN, 3, 1023) == (2, 3)
    assert msa.tune_get(msa.MSA_TUNE_PLAIN, 3, 511) == (0, 0)
    assert msa.tune_get(msa.MSA_TUNE_PLAIN, 4, 512) == (0, 0)
    msa.tune_set(msa.MSA_TUNE_BATCH, 3, 0, 0, 2)  # the class of k = 2..4
    assert msa.tune_get(msa.MSA_TUNE_BATCH, 2, 7) == (0, 2)
    assert msa.tune_get(msa.MSA_TUNE_BATCH, 5, 0) == (0, 0)
    for args in ((2, 3, 10, 0, 0), (0, 9, 10, 0, 0), (0, 3, -1, 0, 0), (0, 3, 10, 3, 0),
                 (0, 3, 10, 1, 65), (1, 3, 10, 1, 1)):
        with pytest.raises(msa.MsaError) as e:
            msa.tune_set(*args)
        assert e.value.status == msa.MSA_EINVAL
    msa.tune_clear()
    assert msa.tune_get(msa.MSA_TUNE_PLAIN, 3, 512) == (0, 0)


def test_server_debug_wait_limit_rejects_bad_arguments():
    lib = msa.lib()
    # a null server and bad values are refused before anything touches a device
    assert lib.msa_server_debug_wait_limit(None, 1, 1) == msa.MSA_EINVAL
    assert lib.msa_server_stats(None, None, 0) == msa.MSA_EINVAL
