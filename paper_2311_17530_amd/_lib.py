"""ctypes binding of ``libmsa_dp.so`` (argument marshalling only).

Every step of the alignment runs in the library's HIP kernels; this module
only converts Python/numpy/torch arguments into pointers and sizes.  PyTorch
supplies device memory and streams.  If the shared library is missing the
import of any entry point raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

import os

PKG = Path(__file__).resolve().parent
# MSA_LIB overrides the library path (a variant built with extra flags)
LIB_PATH = Path(os.environ.get("MSA_LIB", str(PKG / "_lib" / "libmsa_dp.so")))

MAX_K = 8
GAP = 0xFF

MSA_OK, MSA_EINVAL, MSA_ERANGE, MSA_ENOMEM, MSA_EDEVICE, MSA_EAGAIN, MSA_ESHUTDOWN = (
    0, -1, -2, -3, -4, -5, -6)

_lib = None

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_vp = ctypes.c_void_p


class MsaError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().msa_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class MsaJob(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32),
                ("seqs", c_vp * MAX_K),
                ("lens", ctypes.c_int32 * MAX_K),
                ("submat", c_vp),
                ("alpha", ctypes.c_int32),
                ("gap", ctypes.c_int32)]


class MsaResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32),
                ("score", ctypes.c_int64),
                ("aln", c_vp),
                ("aln_cap", ctypes.c_int64),
                ("aln_len", ctypes.c_int64)]


# alignment mode flags (msa_dp_align_ex / msa_dp_prepare_ex)
MSA_END_GAPS_FREE = 1
MSA_COOPTIMAL = 2
MSA_PRUNE = 4
MSA_NEAROPT = 8
# launch-configuration tuner kinds
MSA_TUNE_PLAIN = 0
MSA_TUNE_BATCH = 1

_SIGS = {
    "msa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "msa_dp_align": (ctypes.c_int, [ctypes.POINTER(c_vp), c_i32p, ctypes.c_int32, c_vp,
                                    ctypes.c_int32, ctypes.c_int32, c_i64p, c_vp,
                                    ctypes.c_int64, c_i64p]),
    "msa_dp_align_ex": (ctypes.c_int, [ctypes.POINTER(c_vp), c_i32p, ctypes.c_int32, c_vp,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                       c_i64p, c_vp, ctypes.c_int64, c_i64p]),
    "msa_dp_align_coopt": (ctypes.c_int, [ctypes.POINTER(c_vp), c_i32p, ctypes.c_int32, c_vp,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          c_i64p, c_vp, ctypes.c_int64, c_vp, c_i32p]),
    "msa_dp_align_nearopt": (ctypes.c_int, [ctypes.POINTER(c_vp), c_i32p, ctypes.c_int32, c_vp,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_int32, c_i64p, c_vp, c_vp, ctypes.c_int64,
                                            c_vp, c_i32p]),
    "msa_dp_workspace_bytes": (ctypes.c_int64, [c_i32p, ctypes.c_int32]),
    "msa_dp_workspace_bytes_ex": (ctypes.c_int64, [c_i32p, ctypes.c_int32, ctypes.c_uint32]),
    "msa_dp_prepare": (ctypes.c_int, [c_vp, ctypes.c_int64, c_i32p, ctypes.c_int32, c_vp,
                                      ctypes.c_int32, ctypes.c_int32, c_vp]),
    "msa_dp_prepare_ex": (ctypes.c_int, [c_vp, ctypes.c_int64, c_i32p, ctypes.c_int32, c_vp,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, c_vp]),
    "msa_dp_align_dev": (ctypes.c_int, [c_vp, ctypes.c_int64, c_vp, c_i32p, ctypes.c_int32,
                                        c_vp, c_vp, ctypes.c_int64, c_vp, c_vp, c_vp]),
    "msa_dp_align_static": (ctypes.c_int, [c_vp, c_i32p, ctypes.c_int32, c_vp, ctypes.c_int32,
                                           ctypes.c_int32, c_vp, c_vp, ctypes.c_int64, c_vp,
                                           c_vp, c_vp]),
    "msa_dp_fill_dev": (ctypes.c_int, [c_vp, ctypes.c_int64, c_vp, c_i32p, ctypes.c_int32,
                                       c_vp, c_vp]),
    "msa_dp_traceback_dev": (ctypes.c_int, [c_vp, ctypes.c_int64, c_vp, c_i32p,
                                            ctypes.c_int32, c_vp, c_vp, ctypes.c_int64, c_vp,
                                            c_vp, c_vp]),
    "msa_dp_export_dirs": (ctypes.c_int, [c_vp, ctypes.c_int64, c_i32p, ctypes.c_int32,
                                          c_vp, c_vp]),
    "msa_dp_export_prune": (ctypes.c_int, [c_vp, ctypes.c_int64, c_i32p, ctypes.c_int32,
                                           c_vp, c_vp, c_vp]),
    "msa_dp_coopt_dev": (ctypes.c_int, [c_vp, ctypes.c_int64, c_vp, c_i32p, ctypes.c_int32,
                                        ctypes.c_int32, c_vp, c_vp, ctypes.c_int64, c_vp,
                                        c_vp, c_vp, c_vp]),
    "msa_dp_nearopt_dev": (ctypes.c_int, [c_vp, ctypes.c_int64, c_vp, c_i32p, ctypes.c_int32,
                                          ctypes.c_int64, ctypes.c_int32, c_vp, c_vp, c_vp,
                                          ctypes.c_int64, c_vp, c_vp, c_vp, c_vp]),
    "msa_dp_align_batch": (ctypes.c_int, [ctypes.POINTER(MsaJob), ctypes.c_int32,
                                          ctypes.POINTER(MsaResult), ctypes.c_int64]),
    "msa_server_create": (c_vp, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "msa_server_submit": (ctypes.c_int, [c_vp, ctypes.POINTER(MsaJob),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "msa_server_poll": (ctypes.c_int, [c_vp, ctypes.c_uint64, ctypes.POINTER(MsaResult)]),
    "msa_server_wait": (ctypes.c_int, [c_vp, ctypes.c_uint64, ctypes.POINTER(MsaResult),
                                       ctypes.c_int64]),
    "msa_server_destroy": (None, [c_vp]),
    "msa_server_stats": (ctypes.c_int, [c_vp, c_i64p, ctypes.c_int32]),
    "msa_server_debug_wait_limit": (ctypes.c_int, [c_vp, ctypes.c_int64, ctypes.c_int32]),
    "msa_dp_score_bounds": (ctypes.c_int, [c_i32p, ctypes.c_int32, c_vp, ctypes.c_int32,
                                           ctypes.c_int32, c_i64p, c_i64p]),
    "msa_dp_check_scoring": (ctypes.c_int, [c_i32p, ctypes.c_int32, c_vp, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_uint32]),
    "msa_dp_tune_set": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32]),
    "msa_dp_tune_get": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, c_i32p]),
    "msa_dp_tune_clear": (None, []),
    "msa_dp_tune_candidates": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              c_i32p, ctypes.c_int32]),
    "msa_dp_autotune": (ctypes.c_int, [c_i32p, ctypes.c_int32, c_vp, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, c_i32p,
                                       ctypes.POINTER(ctypes.c_float)]),
    "msa_dp_autotune_batch": (ctypes.c_int, [ctypes.POINTER(MsaJob), ctypes.c_int32,
                                             ctypes.c_int32, c_i32p]),
    "msa_dp_tile_edge": (ctypes.c_int32, [ctypes.c_int32]),
    "msa_dp_tile_grid": (ctypes.c_int32, [c_i32p, ctypes.c_int32, ctypes.c_int32, c_i32p]),
    "msa_dp_wave_counts": (ctypes.c_int32, [c_i32p, ctypes.c_int32, c_i64p, ctypes.c_int32]),
}


def lib():
    """Load the library (raises FileNotFoundError when it was not built).

    PyTorch (when installed) is imported first: its wheel ships its own HIP
    runtime under the same soname, and the library must bind to that copy.
    Loaded the other way round, the process would hold two HIP runtimes,
    torch could not initialise its device afterwards, and device pointers and
    streams would not be shared between the two."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2311_17530_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        h = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def exported_names():
    return list(_SIGS)


def _i32arr(xs):
    return (ctypes.c_int32 * len(xs))(*[int(x) for x in xs])


def _check(rc, what):
    if rc != MSA_OK:
        raise MsaError(rc, what)


# ---------------------------------------------------------------------------
# host helpers
# ---------------------------------------------------------------------------
def strerror(status: int) -> str:
    return lib().msa_strerror(int(status)).decode()


def score_bounds(lens, sub, gap):
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    lo, hi = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().msa_dp_score_bounds(_i32arr(lens), len(lens), sub.ctypes.data, sub.shape[0],
                                   int(gap), ctypes.byref(lo), ctypes.byref(hi))
    _check(rc, "msa_dp_score_bounds")
    return lo.value, hi.value


def check_scoring(lens, sub, gap, flags: int = 0) -> int:
    """Status of ``msa_dp_check_scoring`` (host only: shape, scoring, mode
    flags and the closed-form key range of that mode)."""
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    return int(lib().msa_dp_check_scoring(_i32arr(lens), len(lens), sub.ctypes.data,
                                          sub.shape[0], int(gap), int(flags)))


def tile_edge(k: int) -> int:
    return int(lib().msa_dp_tile_edge(int(k)))


def tile_grid(lens, tile):
    out = (ctypes.c_int32 * len(lens))()
    w = lib().msa_dp_tile_grid(_i32arr(lens), len(lens), int(tile), out)
    if w < 0:
        raise MsaError(w, "msa_dp_tile_grid")
    return list(out), int(w)


def wave_counts(p):
    cap = sum(p) + 1
    out = (ctypes.c_int64 * cap)()
    w = lib().msa_dp_wave_counts(_i32arr(p), len(p), out, cap)
    if w < 0:
        raise MsaError(w, "msa_dp_wave_counts")
    return [int(x) for x in out[:w]]


def workspace_bytes(lens) -> int:
    n = int(lib().msa_dp_workspace_bytes(_i32arr(lens), len(lens)))
    if n < 0:
        raise MsaError(n, "msa_dp_workspace_bytes")
    return n


# ---------------------------------------------------------------------------
# plain path, host buffers
# ---------------------------------------------------------------------------
def align(seqs, sub, gap, end_gaps_free: bool = False, prune: bool = False):
    """Optimal alignment through ``msa_dp_align_ex`` (host buffers);
    ``end_gaps_free`` selects MSA_END_GAPS_FREE, ``prune`` MSA_PRUNE.

    Returns ``(score, rows)`` with rows a (k, L) uint8 array (GAP for gaps)."""
    seqs = [np.ascontiguousarray(np.asarray(s, dtype=np.uint8)) for s in seqs]
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    k = len(seqs)
    cap = max(1, sum(len(s) for s in seqs))
    out = np.full((k, cap), GAP, dtype=np.uint8)
    ptrs = (c_vp * k)(*[s.ctypes.data if len(s) else None for s in seqs])
    score, alen = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().msa_dp_align_ex(ptrs, _i32arr([len(s) for s in seqs]), k, sub.ctypes.data,
                               sub.shape[0], int(gap),
                               (MSA_END_GAPS_FREE if end_gaps_free else 0)
                               | (MSA_PRUNE if prune else 0),
                               ctypes.byref(score), out.ctypes.data, cap, ctypes.byref(alen))
    _check(rc, "msa_dp_align_ex")
    return int(score.value), out[:, : alen.value].copy()


def align_coopt(seqs, sub, gap, max_paths: int):
    """Up to ``max_paths`` co-optimal alignments through ``msa_dp_align_coopt``.

    Returns ``(score, [rows, ...])``; fewer than ``max_paths`` alignments means
    all of them (alignment 0 is ``align``'s)."""
    seqs = [np.ascontiguousarray(np.asarray(s, dtype=np.uint8)) for s in seqs]
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    k = len(seqs)
    cap = max(1, sum(len(s) for s in seqs))
    out = np.full((int(max_paths), k, cap), GAP, dtype=np.uint8)
    lens_out = np.zeros(max(1, int(max_paths)), dtype=np.int64)
    ptrs = (c_vp * k)(*[s.ctypes.data if len(s) else None for s in seqs])
    score, npaths = ctypes.c_int64(), ctypes.c_int32()
    rc = lib().msa_dp_align_coopt(ptrs, _i32arr([len(s) for s in seqs]), k, sub.ctypes.data,
                                  sub.shape[0], int(gap), int(max_paths), ctypes.byref(score),
                                  out.ctypes.data, cap, lens_out.ctypes.data,
                                  ctypes.byref(npaths))
    _check(rc, "msa_dp_align_coopt")
    return int(score.value), [out[p, :, : lens_out[p]].copy() for p in range(npaths.value)]


def align_nearopt(seqs, sub, gap, delta: int, max_paths: int):
    """Up to ``max_paths`` alignments scoring at least opt - ``delta`` through
    ``msa_dp_align_nearopt``.

    Returns ``(opt, [(score, rows), ...])``; fewer than ``max_paths``
    alignments means all of them."""
    seqs = [np.ascontiguousarray(np.asarray(s, dtype=np.uint8)) for s in seqs]
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    k = len(seqs)
    cap = max(1, sum(len(s) for s in seqs))
    out = np.full((int(max_paths), k, cap), GAP, dtype=np.uint8)
    lens_out = np.zeros(max(1, int(max_paths)), dtype=np.int64)
    scores = np.zeros(max(1, int(max_paths)), dtype=np.int64)
    ptrs = (c_vp * k)(*[s.ctypes.data if len(s) else None for s in seqs])
    score, npaths = ctypes.c_int64(), ctypes.c_int32()
    rc = lib().msa_dp_align_nearopt(ptrs, _i32arr([len(s) for s in seqs]), k, sub.ctypes.data,
                                    sub.shape[0], int(gap), int(delta), int(max_paths),
                                    ctypes.byref(score), scores.ctypes.data, out.ctypes.data,
                                    cap, lens_out.ctypes.data, ctypes.byref(npaths))
    _check(rc, "msa_dp_align_nearopt")
    return int(score.value), [(int(scores[p]), out[p, :, : lens_out[p]].copy())
                              for p in range(npaths.value)]


def workspace_bytes_ex(lens, flags: int) -> int:
    """``msa_dp_workspace_bytes_ex``: workspace bytes for a mode."""
    n = lib().msa_dp_workspace_bytes_ex(_i32arr(lens), len(lens), int(flags))
    if n < 0:
        raise MsaError(int(n), "msa_dp_workspace_bytes_ex")
    return int(n)


def tune_set(kind: int, k: int, max_len: int, variant: int, wpc: int):
    """Store a launch configuration for (kind, k, length bucket of max_len)
    (``msa_dp_tune_set``)."""
    _check(lib().msa_dp_tune_set(int(kind), int(k), int(max_len), int(variant), int(wpc)),
           "msa_dp_tune_set")


def tune_get(kind: int, k: int, max_len: int):
    """``(variant, wpc)`` stored for the key, (0, 0) for the built-in rule."""
    out = (ctypes.c_int32 * 2)()
    _check(lib().msa_dp_tune_get(int(kind), int(k), int(max_len), out), "msa_dp_tune_get")
    return int(out[0]), int(out[1])


def tune_clear():
    lib().msa_dp_tune_clear()


def tune_candidates(kind: int, k: int, max_len: int):
    """The (variant, wpc) pairs the tuner tries for the key."""
    n = lib().msa_dp_tune_candidates(int(kind), int(k), int(max_len), None, 0)
    if n < 0:
        raise MsaError(int(n), "msa_dp_tune_candidates")
    out = (ctypes.c_int32 * (2 * n))()
    lib().msa_dp_tune_candidates(int(kind), int(k), int(max_len), out, 2 * n)
    return [(int(out[2 * i]), int(out[2 * i + 1])) for i in range(n)]


def autotune(lens, sub, gap, reps: int = 3):
    """Time every candidate fill of this shape (``msa_dp_autotune``), store the
    fastest and return ``(variant, wpc, best_ms)``."""
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    out = (ctypes.c_int32 * 2)()
    ms = ctypes.c_float()
    _check(lib().msa_dp_autotune(_i32arr(lens), len(lens), sub.ctypes.data, sub.shape[0],
                                 int(gap), int(reps), out, ctypes.byref(ms)), "msa_dp_autotune")
    return int(out[0]), int(out[1]), float(ms.value)


def autotune_batch(jobs, reps: int = 2):
    """Time every candidate workgroup count of the batched fill on these jobs
    (``msa_dp_autotune_batch``); returns the choice per k class."""
    keep = []
    arr = (MsaJob * len(jobs))(*[_make_job(s, m, g, keep) for s, m, g in jobs])
    out = (ctypes.c_int32 * 4)()
    _check(lib().msa_dp_autotune_batch(arr, len(jobs), int(reps), out), "msa_dp_autotune_batch")
    return [int(x) for x in out]


# ---------------------------------------------------------------------------
# plain path, device buffers (torch provides memory and the stream)
# ---------------------------------------------------------------------------
class DeviceAligner:
    """Device-resident alignment of one fixed shape and scoring.

    Owns a torch-allocated workspace and output tensors on ``device``; ``run``
    enqueues one alignment on the current torch stream (asynchronous)."""

    def __init__(self, lens, sub, gap, device="cuda", end_gaps_free: bool = False,
                 cooptimal: bool = False, prune: bool = False, nearopt: bool = False):
        import torch
        self.torch = torch
        self.lens = [int(x) for x in lens]
        self.k = len(self.lens)
        self.device = torch.device(device)
        self.sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
        self.gap = int(gap)
        flags = ((MSA_END_GAPS_FREE if end_gaps_free else 0)
                 | (MSA_COOPTIMAL if cooptimal else 0) | (MSA_PRUNE if prune else 0)
                 | (MSA_NEAROPT if nearopt else 0))
        self.ws_bytes = workspace_bytes_ex(self.lens, flags)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.cap = max(1, sum(self.lens))
        self.d_seqs = torch.zeros(max(1, sum(self.lens)), dtype=torch.uint8, device=self.device)
        self.d_aln = torch.full((self.k, self.cap), GAP, dtype=torch.uint8, device=self.device)
        self.d_score = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.d_len = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=self.device)
        rc = lib().msa_dp_prepare_ex(self.ws_ptr, self.ws_bytes, _i32arr(self.lens), self.k,
                                     self.sub.ctypes.data, self.sub.shape[0], self.gap,
                                     flags, self._stream())
        _check(rc, "msa_dp_prepare_ex")

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def set_sequences(self, seqs):
        flat = np.concatenate([np.asarray(s, dtype=np.uint8) for s in seqs]) if sum(
            self.lens) else np.zeros(1, np.uint8)
        if [len(s) for s in seqs] != self.lens:
            raise ValueError("sequence lengths differ from the prepared shape")
        self.d_seqs[: len(flat)].copy_(self.torch.from_numpy(flat))

    def run(self):
        rc = lib().msa_dp_align_dev(self.ws_ptr, self.ws_bytes, self.d_seqs.data_ptr(),
                                    _i32arr(self.lens), self.k, self.d_score.data_ptr(),
                                    self.d_aln.data_ptr(), self.cap, self.d_len.data_ptr(),
                                    self.d_status.data_ptr(), self._stream())
        _check(rc, "msa_dp_align_dev")

    def run_fill(self):
        rc = lib().msa_dp_fill_dev(self.ws_ptr, self.ws_bytes, self.d_seqs.data_ptr(),
                                   _i32arr(self.lens), self.k, self.d_score.data_ptr(),
                                   self._stream())
        _check(rc, "msa_dp_fill_dev")

    def run_traceback(self):
        rc = lib().msa_dp_traceback_dev(self.ws_ptr, self.ws_bytes, self.d_seqs.data_ptr(),
                                        _i32arr(self.lens), self.k, self.d_score.data_ptr(),
                                        self.d_aln.data_ptr(), self.cap, self.d_len.data_ptr(),
                                        self.d_status.data_ptr(), self._stream())
        _check(rc, "msa_dp_traceback_dev")

    def run_coopt(self, max_paths: int):
        """Enqueue the fill and the enumeration of up to ``max_paths``
        co-optimal alignments (``msa_dp_coopt_dev``); read them with
        ``result_coopt``."""
        if getattr(self, "_co_max", 0) != max_paths:
            t = self.torch
            self._co_max = int(max_paths)
            self.d_co_aln = t.full((self._co_max, self.k, self.cap), GAP, dtype=t.uint8,
                                   device=self.device)
            self.d_co_len = t.zeros(max(1, self._co_max), dtype=t.int64, device=self.device)
            self.d_co_np = t.zeros(1, dtype=t.int32, device=self.device)
        rc = lib().msa_dp_coopt_dev(self.ws_ptr, self.ws_bytes, self.d_seqs.data_ptr(),
                                    _i32arr(self.lens), self.k, int(max_paths),
                                    self.d_score.data_ptr(), self.d_co_aln.data_ptr(), self.cap,
                                    self.d_co_len.data_ptr(), self.d_co_np.data_ptr(),
                                    self.d_status.data_ptr(), self._stream())
        _check(rc, "msa_dp_coopt_dev")

    def result_coopt(self):
        """Synchronise and return ``(score, [rows, ...])`` of ``run_coopt``."""
        self.torch.cuda.current_stream(self.device).synchronize()
        st = int(self.d_status.item())
        if st != MSA_OK:
            raise MsaError(st, "device status")
        n = int(self.d_co_np.item())
        lens = self.d_co_len[:n].cpu().numpy()
        aln = self.d_co_aln[:n].cpu().numpy()
        return int(self.d_score.item()), [aln[p, :, : lens[p]].copy() for p in range(n)]

    def run_nearopt(self, delta: int, max_paths: int):
        """Enqueue the fill and the walk of up to ``max_paths`` alignments
        scoring at least opt - ``delta`` (``msa_dp_nearopt_dev``); read them
        with ``result_nearopt``."""
        t = self.torch
        if getattr(self, "_no_max", 0) != max_paths:
            self._no_max = int(max_paths)
            self.d_no_aln = t.full((self._no_max, self.k, self.cap), GAP, dtype=t.uint8,
                                   device=self.device)
            self.d_no_len = t.zeros(max(1, self._no_max), dtype=t.int64, device=self.device)
            self.d_no_sc = t.zeros(max(1, self._no_max), dtype=t.int64, device=self.device)
            self.d_no_np = t.zeros(1, dtype=t.int32, device=self.device)
        rc = lib().msa_dp_nearopt_dev(self.ws_ptr, self.ws_bytes, self.d_seqs.data_ptr(),
                                      _i32arr(self.lens), self.k, int(delta), int(max_paths),
                                      self.d_score.data_ptr(), self.d_no_sc.data_ptr(),
                                      self.d_no_aln.data_ptr(), self.cap,
                                      self.d_no_len.data_ptr(), self.d_no_np.data_ptr(),
                                      self.d_status.data_ptr(), self._stream())
        _check(rc, "msa_dp_nearopt_dev")

    def result_nearopt(self):
        """Synchronise and return ``(opt, [(score, rows), ...])`` of
        ``run_nearopt``."""
        self.torch.cuda.current_stream(self.device).synchronize()
        st = int(self.d_status.item())
        if st != MSA_OK:
            raise MsaError(st, "device status")
        n = int(self.d_no_np.item())
        lens = self.d_no_len[:n].cpu().numpy()
        sc = self.d_no_sc[:n].cpu().numpy()
        aln = self.d_no_aln[:n].cpu().numpy()
        return int(self.d_score.item()), [(int(sc[p]), aln[p, :, : lens[p]].copy())
                                          for p in range(n)]

    def result(self):
        """Synchronise and return ``(score, rows)`` (raises on device status)."""
        self.torch.cuda.current_stream(self.device).synchronize()
        st = int(self.d_status.item())
        if st != MSA_OK:
            raise MsaError(st, "device status")
        L = int(self.d_len.item())
        rows = self.d_aln[:, :L].cpu().numpy()
        return int(self.d_score.item()), rows

    def export_prune(self):
        """Pruned mode: ``(keep, info)`` of the last fill -- keep flags over
        the tile grid (array of the tile-grid shape) and
        ``{"U", "L", "kept", "passes"}``."""
        t = self.torch
        P, _ = tile_grid(self.lens, tile_edge(self.k))
        keep = t.zeros(int(np.prod(P)), dtype=t.uint8, device=self.device)
        info = t.zeros(4, dtype=t.int64, device=self.device)
        rc = lib().msa_dp_export_prune(self.ws_ptr, self.ws_bytes, _i32arr(self.lens), self.k,
                                       keep.data_ptr(), info.data_ptr(), self._stream())
        _check(rc, "msa_dp_export_prune")
        self.torch.cuda.current_stream(self.device).synchronize()
        v = [int(x) for x in info.cpu().tolist()]
        return (keep.cpu().numpy().reshape(P).astype(bool),
                {"U": v[0], "L": v[1], "kept": v[2], "passes": v[3]})

    def export_dirs(self):
        """Row-major decision tensor of the last run: the neighbour mask per
        cell, or the tie set per cell (bit b - 1 for mask b) when the aligner
        was made with ``cooptimal``."""
        shape = tuple(n + 1 for n in self.lens)
        out = self.torch.empty(int(np.prod(shape)), dtype=self.torch.uint8, device=self.device)
        rc = lib().msa_dp_export_dirs(self.ws_ptr, self.ws_bytes, _i32arr(self.lens), self.k,
                                      out.data_ptr(), self._stream())
        _check(rc, "msa_dp_export_dirs")
        self.torch.cuda.current_stream(self.device).synchronize()
        return out.cpu().numpy().reshape(shape)


# ---------------------------------------------------------------------------
# batched and served paths
# ---------------------------------------------------------------------------
def _make_job(seqs, sub, gap, keep):
    seqs = [np.ascontiguousarray(np.asarray(s, dtype=np.uint8)) for s in seqs]
    sub = np.ascontiguousarray(np.asarray(sub, dtype=np.int8))
    keep.append((seqs, sub))
    j = MsaJob()
    j.k = len(seqs)
    for i, s in enumerate(seqs):
        j.seqs[i] = s.ctypes.data if len(s) else None
        j.lens[i] = len(s)
    j.submat = sub.ctypes.data
    j.alpha = sub.shape[0]
    j.gap = int(gap)
    return j


def align_batch(jobs, hbm_budget_bytes: int = 0):
    """Align many jobs (each ``(seqs, sub, gap)``) in persistent launches.

    Returns a list of ``(status, score, rows)``."""
    keep = []
    n = len(jobs)
    cj = (MsaJob * n)()
    cr = (MsaResult * n)()
    outs = []
    for i, (seqs, sub, gap) in enumerate(jobs):
        cj[i] = _make_job(seqs, sub, gap, keep)
        cap = max(1, sum(len(s) for s in seqs))
        buf = np.full((len(seqs), cap), GAP, dtype=np.uint8)
        outs.append(buf)
        cr[i].aln = buf.ctypes.data
        cr[i].aln_cap = cap
    rc = lib().msa_dp_align_batch(cj, n, cr, int(hbm_budget_bytes))
    _check(rc, "msa_dp_align_batch")
    res = []
    for i in range(n):
        r = cr[i]
        res.append((int(r.status), int(r.score), outs[i][:, : r.aln_len].copy()))
    return res


class Server:
    """Continuous-batching alignment server (``msa_server_*``)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_inflight: int = 4,
                 max_jobs_per_launch: int = 256):
        self.h = lib().msa_server_create(int(hbm_budget_bytes), int(max_inflight),
                                         int(max_jobs_per_launch))
        if not self.h:
            raise MsaError(MSA_EDEVICE, "msa_server_create")
        self._caps = {}

    def submit(self, seqs, sub, gap) -> int:
        keep = []
        j = _make_job(seqs, sub, gap, keep)
        t = ctypes.c_uint64()
        rc = lib().msa_server_submit(self.h, ctypes.byref(j), ctypes.byref(t))
        _check(rc, "msa_server_submit")
        self._caps[t.value] = (len(seqs), max(1, sum(len(s) for s in seqs)))
        return int(t.value)

    def _result(self, ticket, timeout_us=None):
        k, cap = self._caps[ticket]
        buf = np.full((k, cap), GAP, dtype=np.uint8)
        r = MsaResult()
        r.aln = buf.ctypes.data
        r.aln_cap = cap
        if timeout_us is None:
            rc = lib().msa_server_poll(self.h, ticket, ctypes.byref(r))
        else:
            rc = lib().msa_server_wait(self.h, ticket, ctypes.byref(r), int(timeout_us))
        if rc == MSA_EAGAIN:
            return None
        del self._caps[ticket]
        return int(r.status), int(r.score), buf[:, : r.aln_len].copy()

    def poll(self, ticket):
        return self._result(ticket)

    def wait(self, ticket, timeout_us=-1):
        return self._result(ticket, timeout_us)

    def stats(self):
        """``{"launches", "jobs", "busy_us", "span_us", "queued", "failed",
        "last_failure", "max_pause_us", "rerun"}`` so far."""
        out = (ctypes.c_int64 * 9)()
        _check(lib().msa_server_stats(self.h, out, 9), "msa_server_stats")
        return dict(zip(("launches", "jobs", "busy_us", "span_us", "queued", "failed",
                         "last_failure", "max_pause_us", "rerun"), [int(x) for x in out]))

    def debug_wait_limit(self, ticks: int, launches: int):
        """The next ``launches`` launches time out a dependency wait after
        ``ticks`` ticks of the 100 MHz clock (``msa_server_debug_wait_limit``)."""
        _check(lib().msa_server_debug_wait_limit(self.h, int(ticks), int(launches)),
               "msa_server_debug_wait_limit")

    def close(self):
        if self.h:
            lib().msa_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
