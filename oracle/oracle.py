"""ctypes front-end for the C oracle (``msa_oracle.c``).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

The C code is compiled with plain ``gcc -O2`` (no OpenMP, no intrinsics) into
``oracle/_build/libmsa_oracle.so``.  ``build_oracle_lib()`` compiles it; the
loader builds it on first use when the shared object is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

GAP = 0xFF  # gap symbol in alignment rows

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "msa_oracle.c"
_OUT_DIR = _HERE / "_build"
_LIB = _OUT_DIR / "libmsa_oracle.so"
_lib = None


def oracle_lib_path() -> Path:
    return _LIB


def build_oracle_lib(force: bool = True) -> Path:
    """Compile the oracle with gcc -O2 (single thread, no intrinsics)."""
    if _LIB.exists() and not force:
        return _LIB
    _OUT_DIR.mkdir(exist_ok=True)
    tmp = _LIB.with_suffix(f".so.tmp{os.getpid()}")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", str(tmp), str(_SRC)]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB.exists():
        build_oracle_lib()
    lib = ctypes.CDLL(str(_LIB))
    lib.msa_oracle_align.restype = ctypes.c_int
    lib.msa_oracle_align.argtypes = [
        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.msa_oracle_align_egf.restype = ctypes.c_int
    lib.msa_oracle_align_egf.argtypes = lib.msa_oracle_align.argtypes + [
        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.msa_oracle_coopt.restype = ctypes.c_int
    lib.msa_oracle_coopt.argtypes = [
        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
    lib.msa_oracle_nearopt.restype = ctypes.c_int
    lib.msa_oracle_nearopt.argtypes = [
        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]
    lib.msa_oracle_fill.restype = ctypes.c_int
    lib.msa_oracle_fill.argtypes = [
        ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p,
        ctypes.c_void_p]
    _lib = lib
    return lib


def _marshal(seqs, sub):
    seqs = [np.ascontiguousarray(np.asarray(s, dtype=np.uint8)) for s in seqs]
    k = len(seqs)
    lens = (ctypes.c_int32 * k)(*[len(s) for s in seqs])
    ptrs = (ctypes.c_void_p * k)(*[s.ctypes.data if len(s) else None for s in seqs])
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int32))
    alpha = sub.shape[0]
    if sub.shape != (alpha, alpha):
        raise ValueError("substitution matrix must be square")
    return seqs, k, lens, ptrs, sub, alpha


def oracle_align(seqs, sub, gap: int, want_dir: bool = False):
    """Optimal alignment of ``seqs`` (list of uint8 code arrays).

    Returns ``(score, rows, dir)``: ``rows`` is a (k, L) uint8 array with GAP
    for gaps; ``dir`` (only if ``want_dir``) is the decision tensor of shape
    (n_0+1, ..., n_{k-1}+1) holding the chosen neighbour mask per cell.
    """
    lib = _load()
    seqs, k, lens, ptrs, sub, alpha = _marshal(seqs, sub)
    total = int(sum(len(s) for s in seqs))
    cap = max(total, 1)
    aln = np.full((k, cap), GAP, dtype=np.uint8)
    shape = tuple(len(s) + 1 for s in seqs)
    dirt = np.zeros(shape, dtype=np.uint8) if want_dir else None
    score = ctypes.c_int64(0)
    alen = ctypes.c_int64(0)
    rc = lib.msa_oracle_align(
        k, lens, ptrs, alpha, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(gap), ctypes.byref(score),
        dirt.ctypes.data if dirt is not None else None,
        aln.ctypes.data, cap, ctypes.byref(alen))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    rows = aln[:, : alen.value].copy()
    return int(score.value), rows, dirt


def oracle_align_egf(seqs, sub, gap: int, want_dir: bool = False):
    """End-gap-free optimal alignment (see ``msa_oracle_align_egf``).

    Returns ``(score, rows, dir, (core_begin, core_end))``; the score is the
    sum-of-pairs score of ``rows[:, core_begin:core_end]``.
    """
    lib = _load()
    seqs, k, lens, ptrs, sub, alpha = _marshal(seqs, sub)
    total = int(sum(len(s) for s in seqs))
    cap = max(total, 1)
    aln = np.full((k, cap), GAP, dtype=np.uint8)
    shape = tuple(len(s) + 1 for s in seqs)
    dirt = np.zeros(shape, dtype=np.uint8) if want_dir else None
    score = ctypes.c_int64(0)
    alen = ctypes.c_int64(0)
    cb = ctypes.c_int64(0)
    ce = ctypes.c_int64(0)
    rc = lib.msa_oracle_align_egf(
        k, lens, ptrs, alpha, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(gap), ctypes.byref(score),
        dirt.ctypes.data if dirt is not None else None,
        aln.ctypes.data, cap, ctypes.byref(alen), ctypes.byref(cb), ctypes.byref(ce))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    rows = aln[:, : alen.value].copy()
    return int(score.value), rows, dirt, (int(cb.value), int(ce.value))


def oracle_coopt(seqs, sub, gap: int, max_paths: int, want_ties: bool = False):
    """Up to ``max_paths`` co-optimal alignments (see ``msa_oracle_coopt``).

    Returns ``(score, [rows, ...], ties)``; fewer than ``max_paths`` alignments
    means all of them.  ``ties`` (if requested) holds bit b - 1 for every
    maximising mask b of each cell."""
    lib = _load()
    seqs, k, lens, ptrs, sub, alpha = _marshal(seqs, sub)
    total = int(sum(len(s) for s in seqs))
    cap = max(total, 1)
    aln = np.full((max_paths, k, cap), GAP, dtype=np.uint8)
    alen = np.zeros(max_paths, dtype=np.int64)
    shape = tuple(len(s) + 1 for s in seqs)
    ties = np.zeros(shape, dtype=np.uint8) if want_ties else None
    score = ctypes.c_int64(0)
    npaths = ctypes.c_int32(0)
    rc = lib.msa_oracle_coopt(
        k, lens, ptrs, alpha, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(gap), int(max_paths), ctypes.byref(score),
        ties.ctypes.data if ties is not None else None, aln.ctypes.data, cap,
        alen.ctypes.data, ctypes.byref(npaths))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    rows = [aln[p, :, : alen[p]].copy() for p in range(npaths.value)]
    return int(score.value), rows, ties


def oracle_nearopt(seqs, sub, gap: int, delta: int, max_paths: int):
    """Up to ``max_paths`` alignments scoring at least opt - ``delta`` (see
    ``msa_oracle_nearopt``).

    Returns ``(opt, [(score, rows), ...])``; fewer than ``max_paths``
    alignments means all of them."""
    lib = _load()
    seqs, k, lens, ptrs, sub, alpha = _marshal(seqs, sub)
    total = int(sum(len(s) for s in seqs))
    cap = max(total, 1)
    aln = np.full((max_paths, k, cap), GAP, dtype=np.uint8)
    alen = np.zeros(max_paths, dtype=np.int64)
    scores = np.zeros(max_paths, dtype=np.int64)
    score = ctypes.c_int64(0)
    npaths = ctypes.c_int32(0)
    rc = lib.msa_oracle_nearopt(
        k, lens, ptrs, alpha, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(gap), int(delta), int(max_paths), ctypes.byref(score), scores.ctypes.data,
        aln.ctypes.data, cap, alen.ctypes.data, ctypes.byref(npaths))
    if rc != 0:
        raise ValueError("oracle rejected the input")
    out = [(int(scores[p]), aln[p, :, : alen[p]].copy()) for p in range(npaths.value)]
    return int(score.value), out


def oracle_fill(seqs, sub, gap: int):
    """Full int64 score tensor and decision tensor (no traceback)."""
    lib = _load()
    seqs, k, lens, ptrs, sub, alpha = _marshal(seqs, sub)
    shape = tuple(len(s) + 1 for s in seqs)
    xi = np.zeros(shape, dtype=np.int64)
    dirt = np.zeros(shape, dtype=np.uint8)
    rc = lib.msa_oracle_fill(
        k, lens, ptrs, alpha, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(gap), xi.ctypes.data, dirt.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the input")
    return xi, dirt
