"""Benchmark of the k-D DP alignment hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

A step is one whole alignment of the k=3 protein workload (three sequences of
length 512, 513^3 cells): the fill (every cell, one direction byte per cell)
followed by the traceback and the expansion of the gapped rows, with inputs
already resident in HBM.  Prints one JSON line:

  value        GCUPS = cells / step time / 1e9 (whole step, fill + traceback)
  roofline     dominant kernel (the fill): algorithmic integer ops per launch
               (2 per neighbour update: one add, one max) / its average launch
               time measured with HIP events on its stream, against the int32
               VALU peak 256 CU * 64 lanes * 2.4 GHz
  cpu_baseline the oracle (plain single-threaded C) timed on this host on the
               full k=3 / 512 alignment

The same numbers for the k=4 / 128 workload (129^4 cells), the k=3 DNA / 40
workload (41^3 cells, a latency case), the k=3 workload in end-gap-free mode, the k=3 workload's co-optimal mode (tie-set
fill plus the first 16 co-optimal alignments), its near-optimal mode (fill
with cell scores plus the first 16 alignments within 20 of the optimum) and
both workloads in the exact
pruned mode (pairwise bounds, tile selection and the kept tiles' fill, all
inside fill_ms; same score and alignment) are reported under "extra"; "batched" gives jobs/s of the 4096-job workload through the batched
persistent launches (beside sequential plain calls), "served" the saturated
throughput and p50/p99 latency of a 20000-job Poisson stream through the
server at 0.7 and 0.9 times that rate.  Only one GPU is used: --gpus above 1 is
rejected.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12  # 39.3 T int32 lane-ops/s
PEAK_HBM_GBS = 8000.0
MAIN = "prot_k3_512"
EXTRA = ["prot_k4_128", "prot_k5_40", "dna_k3_40"]
# Served stream: fixed Poisson arrival rates (jobs/s), the same on every run
# so that p50/p99 compare across runs and machines.
SERVED_RATES = (4000.0, 7000.0)


def time_workload(name, steps, warmup, end_gaps_free=False, prune=False):
    import torch
    import paper_2311_17530_amd as msa
    from msa_inputs import workload

    job = workload(name)
    dev = msa.DeviceAligner(job.lens, job.sub, job.gap, end_gaps_free=end_gaps_free, prune=prune)
    dev.set_sequences(job.seqs)
    torch.cuda.synchronize()
    for _ in range(warmup):
        dev.run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        dev.run_fill()
        e1.record(stream)
        dev.run_traceback()
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fill_ms = [a.elapsed_time(b) for a, b, _ in ev]
    tb_ms = [b.elapsed_time(c) for _, b, c in ev]
    score, rows = dev.result()
    ms_per_step = wall * 1e3 / steps
    cells = job.cells
    nu = job.neighbour_updates
    fill_avg = float(np.mean(fill_ms))
    extra = {}
    if prune:
        keep, info = dev.export_prune()
        extra = dict(tiles=int(keep.size), tiles_kept=info["kept"], passes=info["passes"],
                     upper_bound=info["U"], threshold=info["L"])
    return dict(
        workload=name + (" end-gap-free" if end_gaps_free else "") + (" pruned" if prune else ""),
        k=job.k, lens=job.lens, **extra,
        cells=cells, neighbour_updates=nu,
        ms_per_step=ms_per_step, fill_ms_avg=fill_avg, fill_ms_min=float(np.min(fill_ms)),
        traceback_ms_avg=float(np.mean(tb_ms)),
        gcups=cells / (ms_per_step / 1e3) / 1e9,
        fill_gcups=cells / (fill_avg / 1e3) / 1e9,
        nu_per_s=nu / (ms_per_step / 1e3),
        fill_tops=2 * nu / (fill_avg / 1e3) / 1e12,
        score=score, aln_len=int(rows.shape[1]),
        tile_edge=msa.tile_edge(job.k))


def time_coopt(name, steps, warmup, max_paths=16):
    """Whole step of the co-optimal mode: the fill keeping tie sets, then the
    enumeration of the first ``max_paths`` co-optimal alignments."""
    import torch
    import paper_2311_17530_amd as msa
    from msa_inputs import workload

    job = workload(name)
    dev = msa.DeviceAligner(job.lens, job.sub, job.gap, cooptimal=True)
    dev.set_sequences(job.seqs)
    for _ in range(warmup):
        dev.run_coopt(max_paths)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        dev.run_coopt(max_paths)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    score, alns = dev.result_coopt()
    ms_per_step = wall * 1e3 / steps
    return dict(workload=name + " co-optimal", k=job.k, lens=job.lens, cells=job.cells,
                max_paths=max_paths, alignments=len(alns), ms_per_step=ms_per_step,
                step_ms_avg=float(np.mean(step_ms)),
                gcups=job.cells / (ms_per_step / 1e3) / 1e9, score=score)


def time_nearopt(name, steps, warmup, delta=20, max_paths=16):
    """Whole step of the near-optimal mode: the fill keeping cell scores, then
    the walk of the first ``max_paths`` alignments within ``delta`` of the
    optimum."""
    import torch
    import paper_2311_17530_amd as msa
    from msa_inputs import workload

    job = workload(name)
    dev = msa.DeviceAligner(job.lens, job.sub, job.gap, nearopt=True)
    dev.set_sequences(job.seqs)
    for _ in range(warmup):
        dev.run_nearopt(delta, max_paths)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        dev.run_nearopt(delta, max_paths)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in ev]
    opt, alns = dev.result_nearopt()
    ms_per_step = wall * 1e3 / steps
    return dict(workload=name + f" near-optimal (delta {delta})", k=job.k, lens=job.lens,
                cells=job.cells, max_paths=max_paths, alignments=len(alns),
                ms_per_step=ms_per_step, step_ms_avg=float(np.mean(step_ms)),
                gcups=job.cells / (ms_per_step / 1e3) / 1e9, score=opt,
                lowest_score=min(s for s, _ in alns))


def bench_batched(n_jobs=4096, n_plain=256):
    """Jobs/s of the batched persistent launches on the 4096-job workload
    (host buffers in and out, staging included), next to the same jobs run one
    at a time through the plain path (first n_plain jobs)."""
    import paper_2311_17530_amd as msa
    from msa_inputs import batch_jobs

    jobs = batch_jobs(n_jobs)
    tuples = [(j.seqs, j.sub, j.gap) for j in jobs]
    msa.align_batch(tuples[:64])  # warm-up: arena allocation, code load
    t0 = time.perf_counter()
    res = msa.align_batch(tuples)
    dt = time.perf_counter() - t0
    ok = sum(r[0] == 0 for r in res)
    cells = sum(j.cells for j in jobs)
    msa.align(*tuples[0])
    t1 = time.perf_counter()
    for t in tuples[:n_plain]:
        msa.align(*t)
    dtp = time.perf_counter() - t1
    return {"jobs": n_jobs, "ok": ok, "seconds": round(dt, 4),
            "jobs_per_s": round(n_jobs / dt, 2), "gcups": round(cells / dt / 1e9, 3),
            "sequential_plain_jobs_per_s": round(n_plain / dtp, 2),
            "sequential_plain_sample": f"first {n_plain} jobs, one msa_dp_align call each",
            "speedup_vs_sequential": round((n_jobs / dt) / (n_plain / dtp), 2)}


def bench_served(n_jobs=20000, rates=SERVED_RATES, max_inflight=4, max_jobs=256,
                 n_plain=1000):
    """Served path on the 20000-job mix.

    Jobs are marshalled into C job structs before any timing, so the timed
    windows hold only the library's submit calls and the device work.
    - saturated: every job submitted at t=0 by one thread while another
      thread waits for the results in order; jobs/s over the wall time, and
      the server's own device-busy time (union of its launches' device
      intervals, HIP events) beside it, with the host's share (submit calls)
      timed separately;
    - streams: Poisson arrivals at each fixed rate in `rates` (jobs/s), per
      job latency from its arrival to its result (p50/p99);
    - sequential: the first `n_plain` jobs of the mix one at a time through
      the plain path (one msa_dp_align call each)."""
    import paper_2311_17530_amd as msa
    from msa_inputs import served_jobs

    jobs = served_jobs(n_jobs)
    cells = sum(j.cells for j in jobs)
    pre = _Marshalled(jobs)
    out = {"jobs": n_jobs, "cells": cells,
           "max_inflight_launches": max_inflight, "max_jobs_per_launch": max_jobs}
    with msa.Server(max_inflight=max_inflight, max_jobs_per_launch=max_jobs) as srv:
        for i in range(32):  # warm-up: arenas, code load
            srv.wait(srv.submit(jobs[i].seqs, jobs[i].sub, jobs[i].gap))
        st0 = srv.stats()
        wall, submit_s, status = pre.run_saturated(srv)
        st1 = srv.stats()
        busy = (st1["busy_us"] - st0["busy_us"]) / 1e6
        ok = int((status == 0).sum())
        failed = {str(int(c)): int((status == c).sum()) for c in np.unique(status) if c != 0}
        out.update({"ok": ok, "failed_by_status": failed,
                    "saturated_jobs_per_s": round(n_jobs / wall, 2),
                    "saturated_gcups": round(cells / wall / 1e9, 3),
                    "saturated_seconds": round(wall, 4),
                    "submit_seconds": round(submit_s, 4),
                    "device_busy_seconds": round(busy, 4),
                    "device_busy_fraction": round(busy / wall, 3),
                    "device_jobs_per_s": round(n_jobs / busy, 2) if busy > 0 else None,
                    "launches": st1["launches"] - st0["launches"],
                    "device_max_pause_us": st1["max_pause_us"],
                    "rerun_after_timeout": st1["rerun"] - st0["rerun"]})
        streams = [pre.run_stream(srv, rate) for rate in rates]
    out["streams"] = streams
    if streams:
        out.update({"arrival_rate_per_s": streams[0]["arrival_rate_per_s"],
                    "jobs_per_s": streams[0]["jobs_per_s"],
                    "latency_ms_p50": streams[0]["latency_ms_p50"],
                    "latency_ms_p99": streams[0]["latency_ms_p99"]})
    if n_plain:
        msa.align(jobs[0].seqs, jobs[0].sub, jobs[0].gap)
        t0 = time.perf_counter()
        for j in jobs[:n_plain]:
            msa.align(j.seqs, j.sub, j.gap)
        dt = time.perf_counter() - t0
        out["sequential_plain_jobs_per_s"] = round(n_plain / dt, 2)
        out["sequential_plain_sample"] = f"first {n_plain} jobs, one msa_dp_align call each"
        out["speedup_vs_sequential"] = round(out["saturated_jobs_per_s"] / (n_plain / dt), 2)
    return out


class _Marshalled:
    """Jobs of a stream as C job structs and result buffers, built once."""

    def __init__(self, jobs):
        import ctypes

        import paper_2311_17530_amd as msa
        from paper_2311_17530_amd._lib import MsaResult, _make_job
        self.ctypes = ctypes
        self.msa = msa
        self.keep = []
        self.n = len(jobs)
        self.cj = [_make_job(j.seqs, j.sub, j.gap, self.keep) for j in jobs]
        caps = [max(1, sum(j.lens)) for j in jobs]
        self.bufs = [np.empty((j.k, c), np.uint8) for j, c in zip(jobs, caps)]
        self.res = [MsaResult() for _ in jobs]
        for r, b, c in zip(self.res, self.bufs, caps):
            r.aln = b.ctypes.data
            r.aln_cap = c

    def _waiter(self, srv, tick, ready, t_done, status):
        lib = self.msa.lib()
        for i in range(self.n):
            ready.acquire()
            rc = lib.msa_server_wait(srv.h, tick[i], self.ctypes.byref(self.res[i]), -1)
            t_done[i] = time.perf_counter()
            status[i] = rc

    def _go(self, srv, arrivals):
        import threading
        lib = self.msa.lib()
        ct = self.ctypes
        n = self.n
        tick = [0] * n
        t_sub = np.zeros(n)
        t_done = np.zeros(n)
        status = np.zeros(n, dtype=np.int64)
        ready = threading.Semaphore(0)
        th = threading.Thread(target=self._waiter, args=(srv, tick, ready, t_done, status))
        th.start()
        t = ct.c_uint64()
        submit_s = 0.0
        start = time.perf_counter()
        for i in range(n):
            if arrivals is not None:
                now = time.perf_counter() - start
                if arrivals[i] > now:
                    time.sleep(arrivals[i] - now)
            t0 = time.perf_counter()
            rc = lib.msa_server_submit(srv.h, ct.byref(self.cj[i]), ct.byref(t))
            submit_s += time.perf_counter() - t0
            if rc != 0:
                raise self.msa.MsaError(rc, "msa_server_submit")
            t_sub[i] = t0 if arrivals is None else start + arrivals[i]
            tick[i] = t.value
            ready.release()
        th.join()
        return start, t_sub, t_done, status, submit_s

    def run_saturated(self, srv):
        start, _, t_done, status, submit_s = self._go(srv, None)
        return float(t_done.max() - start), submit_s, status

    def run_stream(self, srv, rate):
        from msa_inputs import poisson_arrivals
        arr = poisson_arrivals(self.n, rate)
        start, t_sub, t_done, status, _ = self._go(srv, arr)
        span = t_done.max() - start
        lat = (t_done - t_sub) * 1e3
        return {"arrival_rate_per_s": rate, "ok": int((status == 0).sum()),
                "failed_by_status": {str(int(c)): int((status == c).sum())
                                     for c in np.unique(status) if c != 0},
                "jobs_per_s": round(self.n / span, 2),
                "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                "latency_ms_p99": round(float(np.percentile(lat, 99)), 3)}


TRAFFIC_SOURCES = ("msa_sweep3.hip", "msa_internal.h", "msa_plan.cpp", "msa_runtime.cpp")


def measured_traffic():
    """HBM bytes per launch of the k=3 fill from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a device copy), or
    None when the kernel, plan or launch sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "fill_k3_prot512_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_17530_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = dict(ln.split(": ", 1) for ln in text.splitlines() if ": " in ln and not ln.startswith(" "))
    if vals.get("source_sha256 (" + " + ".join(TRAFFIC_SOURCES) + ")") != h.hexdigest():
        return None
    return int(vals["traffic_bytes_per_launch"])


def host_cpu():
    """Model name, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(reps=3):
    """The oracle (plain single-threaded C) on the full k=3 / 512 alignment,
    median of `reps` runs with the calling thread pinned to one CPU."""
    from msa_inputs import workload
    from oracle import build_oracle_lib, oracle_align

    build_oracle_lib(force=False)
    job = workload(MAIN)
    old = os.sched_getaffinity(0)
    cpu = min(old)
    os.sched_setaffinity(0, {cpu})
    try:
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle_align(job.seqs, job.sub, job.gap)
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    dt = float(np.median(times))
    return {"value": job.cells / dt / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full {MAIN} alignments (fill + traceback, {job.cells} cells "
                      f"each), median {dt:.2f} s, one thread pinned to CPU {cpu}, gcc -O2",
            "seconds": [round(t, 3) for t in times]}


def sclk_during(fn, seconds=0.4):
    """GPU shader clock (MHz) read with rocm-smi while `fn` runs back to back
    on the device; None when rocm-smi is not usable here."""
    import subprocess
    import threading

    import torch
    stop = threading.Event()
    errors = []

    def spin():
        try:
            while not stop.is_set():
                fn()
                torch.cuda.synchronize()
        except Exception as exc:  # noqa: BLE001 -- re-raised below
            errors.append(exc)

    th = threading.Thread(target=spin)
    th.start()
    try:
        time.sleep(seconds)
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True,
                           text=True, timeout=20)
        data = json.loads(r.stdout) if r.returncode == 0 else {}
    except Exception:  # noqa: BLE001 -- the clock is context only
        data = {}
    finally:
        stop.set()
        th.join()
    if errors:
        raise errors[0]
    for card in data.values():
        if isinstance(card, dict):
            for key, val in card.items():
                if ("sclk" in key.lower() and isinstance(val, str)
                        and "mhz" in val.lower()):
                    digits = "".join(c for c in val if c.isdigit())
                    if digits:
                        return int(digits)
    return None


def _sclk_main():
    import paper_2311_17530_amd as msa
    from msa_inputs import workload
    job = workload(MAIN)
    dev = msa.DeviceAligner(job.lens, job.sub, job.gap)
    dev.set_sequences(job.seqs)
    return sclk_during(dev.run)  # whole alignments: a fill is always followed by its traceback


def copy_probe(nbytes, steps):
    """Plain device-to-device copy of a known size: the reference for scaling
    the FETCH_SIZE / WRITE_SIZE hardware counters into HBM bytes."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "launches": steps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-clock", action="store_true",
                    help="skip the shader-clock reading (profiling runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device copy of BYTES (counter calibration)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-job batch")
    ap.add_argument("--no-served", action="store_true", help="skip the 20000-job server run")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs each alignment on a "
              "single MI355X and has no multi-GPU path (use --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.copy_probe:
        copy_probe(a.copy_probe, a.steps)
        return
    main_r = time_workload(MAIN, a.steps, a.warmup)
    extra = {}
    if not a.no_extra:
        for name in EXTRA:
            extra[name] = time_workload(name, a.steps, a.warmup)
        # the end-gap-free mode on the same workload (same fill, zero faces,
        # far-face maximum, traceback to the first face)
        extra[MAIN + "_end_gaps_free"] = time_workload(MAIN, a.steps, a.warmup, True)
        # co-optimal mode: tie-set fill and the first 16 co-optimal alignments
        extra[MAIN + "_cooptimal"] = time_coopt(MAIN, a.steps, a.warmup)
        # near-optimal mode: fill with cell scores, the first 16 alignments
        # within 20 of the optimum
        extra[MAIN + "_nearopt"] = time_nearopt(MAIN, a.steps, a.warmup)
        # pruned mode (exact): pairwise bounds, tile selection, kept tiles only;
        # the fill time covers the whole sequence
        for name in [MAIN] + EXTRA:
            extra[name + "_pruned"] = time_workload(name, a.steps, a.warmup, prune=True)
    achieved = main_r["fill_tops"]
    traffic = measured_traffic()
    fill_s = main_r["fill_ms_avg"] / 1e3
    line = {
        "metric": "GCUPS",
        "value": round(main_r["gcups"], 3),
        "unit": "Gcell/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": MAIN, "k": 3, "lens": main_r["lens"],
                   "cells": main_r["cells"], "neighbour_updates": main_r["neighbour_updates"],
                   "tile_edge": main_r["tile_edge"], "scoring": "20x20 int8 seed 17, gap -8"},
        "neighbour_updates_per_s": main_r["nu_per_s"],
        "fill_ms": round(main_r["fill_ms_avg"], 4),
        "traceback_ms": round(main_r["traceback_ms_avg"], 4),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_INT32_TOPS, 2), "unit": "Tops/s",
                     "frac": round(achieved / PEAK_INT32_TOPS, 4), "traffic": traffic,
                     "hbm_gbs": round(traffic / fill_s / 1e9, 1) if traffic else None,
                     "hbm_frac": round(traffic / fill_s / 1e9 / PEAK_HBM_GBS, 4)
                     if traffic else None,
                     "algorithmic_bytes": main_r["cells"],
                     "algorithmic_hbm_frac": round(main_r["cells"] / fill_s / 1e9 / PEAK_HBM_GBS,
                                                   4),
                     "kernel": "sweep3_kernel (k=3 streaming fill: 24 rows, three per compute "
                               "wave, x 64 lanes per workgroup, one workgroup per CU)",
                     "ops_per_launch": 2 * main_r["neighbour_updates"]},
        "extra": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in extra.items()},
    }
    line["host"] = host_cpu()
    line["sclk_mhz_during_fill"] = None if a.no_clock else _sclk_main()
    if not a.no_batched:
        line["batched"] = bench_batched()
    if not a.no_served:
        line["served"] = bench_served()
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
