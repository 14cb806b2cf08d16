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
fill plus the first 16 co-optimal alignments) and both workloads in the exact
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
EXTRA = ["prot_k4_128", "dna_k3_40"]


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


def bench_served(n_jobs=20000, loads=(0.7, 0.9), max_inflight=4, max_jobs=256):
    """Served path: saturated throughput X (all jobs submitted at once), then
    Poisson streams at load * X for each load, with per-job latency from
    arrival to result."""
    import paper_2311_17530_amd as msa
    from msa_inputs import served_jobs

    jobs = served_jobs(n_jobs)
    cells = sum(j.cells for j in jobs)
    with msa.Server(max_inflight=max_inflight, max_jobs_per_launch=max_jobs) as srv:
        for j in jobs[:32]:  # warm-up
            srv.wait(srv.submit(j.seqs, j.sub, j.gap))
        t0 = time.perf_counter()
        tickets = [srv.submit(j.seqs, j.sub, j.gap) for j in jobs]
        for t in tickets:
            srv.wait(t)
        sat = n_jobs / (time.perf_counter() - t0)
        streams = [_served_stream(srv, jobs, load, sat) for load in loads]
    if not streams:
        return {"jobs": n_jobs, "saturated_jobs_per_s": round(sat, 2)}
    first = streams[0]
    return {"jobs": n_jobs, "ok": first["ok"],
            "saturated_jobs_per_s": round(sat, 2), "saturated_gcups": round(cells / (n_jobs / sat) / 1e9, 3),
            "arrival_rate_per_s": first["arrival_rate_per_s"], "load": first["load"],
            "jobs_per_s": first["jobs_per_s"],
            "latency_ms_p50": first["latency_ms_p50"], "latency_ms_p99": first["latency_ms_p99"],
            "streams": streams,
            "max_inflight_launches": max_inflight, "max_jobs_per_launch": max_jobs}


def _served_stream(srv, jobs, load, sat):
    """One Poisson stream of `jobs` at load * sat jobs/s through `srv`."""
    import threading

    from msa_inputs import poisson_arrivals

    n_jobs = len(jobs)
    rate = load * sat
    arr = poisson_arrivals(n_jobs, rate)
    tick = [None] * n_jobs
    t_sub = np.zeros(n_jobs)
    t_done = np.zeros(n_jobs)
    status = np.zeros(n_jobs, dtype=np.int64)
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(n_jobs):
            ready.acquire()
            r = srv.wait(tick[i])
            t_done[i] = time.perf_counter()
            status[i] = r[0]

    th = threading.Thread(target=waiter)
    th.start()
    start = time.perf_counter()
    for i, j in enumerate(jobs):
        now = time.perf_counter() - start
        if arr[i] > now:
            time.sleep(arr[i] - now)
        t_sub[i] = time.perf_counter()
        tick[i] = srv.submit(j.seqs, j.sub, j.gap)
        ready.release()
    th.join()
    span = t_done.max() - start
    lat = (t_done - t_sub) * 1e3
    return {"load": load, "arrival_rate_per_s": round(rate, 2), "ok": int((status == 0).sum()),
            "jobs_per_s": round(n_jobs / span, 2),
            "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)), 3)}


def measured_traffic():
    """HBM bytes per launch of the k=3 fill from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a device copy), or
    None when the kernel or launch sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "fill_k3_prot512_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in ("msa_kernels.hip", "msa_runtime.cpp"):
        with open(os.path.join(ROOT, "paper_2311_17530_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = dict(ln.split(": ", 1) for ln in text.splitlines() if ": " in ln and not ln.startswith(" "))
    if vals.get("source_sha256 (msa_kernels.hip + msa_runtime.cpp)") != h.hexdigest():
        return None
    return int(vals["traffic_bytes_per_launch"])


def cpu_baseline():
    from msa_inputs import workload
    from oracle import build_oracle_lib, oracle_align

    build_oracle_lib(force=False)
    job = workload(MAIN)
    t0 = time.perf_counter()
    oracle_align(job.seqs, job.sub, job.gap)
    dt = time.perf_counter() - t0
    return {"value": job.cells / dt / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": f"one full {MAIN} alignment (fill + traceback, "
                      f"{job.cells} cells) in {dt:.2f} s, single thread, gcc -O2"}


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
        # pruned mode (exact): pairwise bounds, tile selection, kept tiles only;
        # the fill time covers the whole sequence
        for name in [MAIN] + EXTRA:
            extra[name + "_pruned"] = time_workload(name, a.steps, a.warmup, prune=True)
    achieved = main_r["fill_tops"]
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
                     "frac": round(achieved / PEAK_INT32_TOPS, 4), "traffic": measured_traffic(),
                     "kernel": "fill_kernel<3,256,2> (k=3, T=16, one line per lane)",
                     "ops_per_launch": 2 * main_r["neighbour_updates"]},
        "extra": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                      for kk, vv in v.items()} for k, v in extra.items()},
    }
    if not a.no_batched:
        line["batched"] = bench_batched()
    if not a.no_served:
        line["served"] = bench_served()
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
