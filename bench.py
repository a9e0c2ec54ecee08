#!/usr/bin/env python3
"""Benchmark of the gfx950 Vietoris-Rips filtration front end (dim <= 2).

One step = one whole build (distances, ranks, threshold, triangles, ordered
output) of the headline workload: 4000 points of an 8-component Gaussian
mixture in R^64 (int8, int8 MFMA Gram), thresholded at the 10th-percentile
edge rank (799800 edges, 94017474 triangles).  Inputs are resident in HBM
before the timed region; outputs stay on the device.  The metric is filtered
simplices per second, n + K + T per build.

Before the line is printed, the last timed build's edges and every triangle
key are compared with the CPU oracle's (built on the host's threads, which is
also the CPU baseline); the line carries "parity": "bit-exact" only if every
element matches, and the run fails otherwise.

Prints ONE JSON line.  Only N = 1 GPU is supported.  Under "extra" the
line also carries side measurements: the 1000-point noisy circle, the
512-cloud batch, a Poisson request stream, a 1088 x 1088 Hamming matrix
(dissimilarity input), the per-column order of a 2000 x 1999 array, the
pairs of dimension 0 and the apparent pairs of dimension 1, tetrahedra
counts, the F2 product and sum of 16384 x 16384 sparse matrices, one
end-to-end figure with the outputs copied to the host, and event-timed
single builds.  --workload runs one of them alone.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak

# HBM bytes per launch of the triangle writer from rocprofv3 FETCH_SIZE and
# WRITE_SIZE, each scaled by what the counter reads for a 256 MiB device copy
# (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000), keyed by workload; `src` is the
# SHA-256 prefix of the writer's sources the counters were taken on, and the
# figure is dropped (null) once those sources change.
TRAFFIC = {
    "mixture4000": {"bytes": 1623461114, "src": "998cef403ad17f91"},
    "circle1000": {"bytes": 77664551, "src": "998cef403ad17f91"},
    "batched512": {"bytes": 29110745100, "src": "998cef403ad17f91"},
}
WRITER_SOURCES = ("k_triangles.hip", "vr_device.h")

# Fixed arrival rate of the serving stream: 0.7 x the plain one-at-a-time
# build's capacity on this stream, measured once on MI355X (2488-2520
# builds/s back to back), then kept for every later run.
SERVE_QPS = 1750.0


def _writer_sha() -> str:
    h = hashlib.sha256()
    for name in WRITER_SOURCES:
        with open(os.path.join(ROOT, "paper_1809_04424_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(workload):
    tr = TRAFFIC.get(workload)
    return tr["bytes"] if tr and tr["src"] == _writer_sha() else None


def _workload(name):
    import workloads

    return {"circle1000": workloads.noisy_circle, "mixture4000": workloads.mixture,
            "plain64": workloads.plain64}[name]()


def _time_builds(vr, torch, pts, thr, steps, warmup, build=None, keep_last=False):
    """Time `steps` whole builds; HIP events bracket only the triangle write
    (on the build's stream), so its average launch duration is measured live.
    Each result is freed once the next build has been issued, as a caller
    consuming results would; its events have completed by then.  With
    keep_last the last result is returned too (for the parity gate)."""
    build = build or vr.build
    prev = None
    for _ in range(max(warmup, 2)):  # two results alive at once, as in the timed loop
        r = build(pts, thr, timing="write")
        if prev is not None:
            prev.free()
        prev = r
    torch.cuda.synchronize()
    if prev is not None:
        prev.free()
    tw = []
    prev = None
    t0 = time.perf_counter()
    for _ in range(steps):
        r = build(pts, thr, timing="write")
        if prev is not None:
            tw.append(prev.stage_ms()["tri_write"])
            prev.free()
        prev = r
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tw.append(prev.stage_ms()["tri_write"])
    counts = prev.counts
    if keep_last:
        return (t1 - t0), counts, sum(tw) / len(tw), prev
    prev.free()
    torch.cuda.synchronize()
    return (t1 - t0), counts, sum(tw) / len(tw)


def _stage_breakdown(vr, torch, pts, thr, reps=10):
    """Untimed builds with events between all stages (events add small gaps)."""
    acc = {}
    for _ in range(reps):
        r = vr.build(pts, thr, timing=True)
        for k, v in r.stage_ms().items():
            acc.setdefault(k, []).append(v)
        r.free()
    torch.cuda.synchronize()
    return {k: round(sum(v) / len(v), 5) for k, v in acc.items()}


def _host_threads():
    """Threads for the oracle: the host's CPU share for one GPU (16), or fewer
    where the host has fewer cores."""
    return max(1, min(16, os.cpu_count() or 1))


def _cpu_baseline(cloud, threads):
    """The oracle's whole build of the headline cloud (distances, ranks,
    threshold, every triangle in filtration order), timed on `threads` host
    threads and on one; returns the baseline and the threaded build, which
    the parity gate then compares with the device's output."""
    import oracle

    oracle.lib()
    t0 = time.perf_counter()
    f = oracle.build_mt(cloud.points, cloud.thr, threads)
    tn = time.perf_counter() - t0
    t0 = time.perf_counter()
    f1 = oracle.build_mt(cloud.points, cloud.thr, 1)
    t1 = time.perf_counter() - t0
    simp = f.n + f.K + f.T
    assert (f1.K, f1.T) == (f.K, f.T)
    del f1
    return {"value": simp / tn, "unit": "simplices/s", "cores": threads, "kind": "oracle",
            "sample": f"one complete build of {cloud.name} by the C oracle (distances by rows of pairs, sortperm, "
                      f"rank matrix, the triangles of each value sorted; distances and triangles split over "
                      f"{threads} threads): {tn:.2f} s; host reports {os.cpu_count()} cores",
            "single_thread": {"value": simp / t1, "seconds": round(t1, 3)}}, f


def _parity_gate(res, f):
    """Every kept edge (endpoints, squared length) and every triangle key of
    the device's result against the oracle's filtration; True when all match."""
    import numpy as np

    n, K, T = res.counts
    if (n, K, T) != (f.n, f.K, f.T):
        return False
    ij = res.edge_ij().cpu().numpy()
    if not (np.array_equal(ij[:, 0], f.ei) and np.array_equal(ij[:, 1], f.ej)
            and np.array_equal(res.edge_q().cpu().numpy(), f.eq)):
        return False
    keys = res.tri_key().cpu().numpy().view(np.uint64)
    t = f.tris.astype(np.uint64)
    want = (t[:, 0] << np.uint64(39)) | (t[:, 1] << np.uint64(26)) | (t[:, 2] << np.uint64(13)) | t[:, 3]
    return bool(np.array_equal(keys, want))


def _batched(vr, torch, reps=3, tune=True):
    """512 R^3 clouds (n log-uniform in [50, 2000], 5th-25th percentile) as
    one batched build, against the same clouds built one call at a time."""
    import workloads

    clouds = workloads.batched()
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    thrs = [c.thr for c in clouds]
    torch.cuda.synchronize()
    tuned = vr.autotune(pts, thrs) if tune else None  # one-time, untimed
    vr.build_batch(pts, thrs).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b = vr.build_batch(pts, thrs)
        simp = sum(sum(it.counts) for it in b)
        b.free()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    print(f"[bench] batched512: {tb * 1e3:.2f} ms per batch", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for p, t in zip(pts, thrs):
        vr.build(p, t).free()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    print(f"[bench] batched512: {ts * 1e3:.2f} ms one cloud at a time", file=sys.stderr, flush=True)
    return {"value": simp / tb, "unit": "simplices/s", "ms_per_batch": 1e3 * tb, "simplices": simp,
            "schedule": list(tuned) if tuned else "default",
            "clouds": len(clouds), "points": sum(c.n for c in clouds),
            "per_cloud_builds": {"value": simp / ts, "ms": 1e3 * ts}, "speedup_vs_per_cloud": ts / tb}


def _pcts(lat):
    lat = sorted(lat)
    pick = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]  # noqa: E731
    return {"p50_ms": round(1e3 * pick(0.50), 4), "p99_ms": round(1e3 * pick(0.99), 4),
            "mean_ms": round(1e3 * sum(lat) / len(lat), 4)}


def _serving(vr, torch, qps=None, requests=2000, warm=100, slots=4, max_batch=32):
    """Poisson stream of clouds (n log-uniform in [100, 5000], d in {2, 3, 16,
    64}, 5th-20th percentile): the plain build (FIFO, one at a time) and the
    continuous-batching request loop at the same fixed QPS.  Latency is
    completion (outputs on the device) minus scheduled arrival; the first
    `warm` requests are excluded from the statistics."""
    import workloads
    from paper_1809_04424_amd.serve import Server

    stream = workloads.serving_stream(requests=requests, qps=1.0)  # arrival times scale as 1/qps
    clouds = [c for _, c in stream]
    unit_t = [t for t, _ in stream]
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    torch.cuda.synchronize()
    for p, c in zip(pts[:warm], clouds[:warm]):
        vr.build(p, c.thr).free()
    torch.cuda.synchronize()
    # capacity of the plain build: back to back, FIFO
    t0 = time.perf_counter()
    simp = []
    for p, c in zip(pts, clouds):
        r = vr.build(p, c.thr)
        simp.append(sum(r.counts))
        r.free()
    torch.cuda.synchronize()
    mu = requests / (time.perf_counter() - t0)
    if not qps:
        qps = max(1.0, round(0.7 * mu))
    arr = [t / qps for t in unit_t]
    print(f"[bench] serving: plain capacity {mu:.1f} req/s, fixed QPS {qps}", file=sys.stderr, flush=True)

    def _sleep_until(t):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    # plain: one build at a time, in arrival order
    start = time.perf_counter() + 0.02
    done = []
    s = torch.cuda.current_stream()
    for a, p, c in zip(arr, pts, clouds):
        _sleep_until(start + a)
        r = vr.build(p, c.thr)
        s.synchronize()
        done.append(time.perf_counter())
        r.free()
    lat_plain = [d - (start + a) for d, a in zip(done, arr)]
    span_plain = done[-1] - (start + arr[warm])
    print("[bench] serving: plain FIFO done", file=sys.stderr, flush=True)

    # served: continuous batching
    with Server(slots=slots, max_batch=max_batch, keep_results=False) as srv:
        start = time.perf_counter() + 0.02
        reqs = []
        for a, p, c in zip(arr, pts, clouds):
            _sleep_until(start + a)
            reqs.append(srv.submit(p, c.thr, arrival=start + a))
        for r in reqs:
            r.wait(timeout=300)
    lat_srv = [r.latency for r in reqs]
    span_srv = max(r.t_done for r in reqs[warm:]) - reqs[warm].arrival
    assert all(sum(r.counts) == n for r, n in zip(reqs, simp)), "served counts differ from plain builds"
    print("[bench] serving: request loop done", file=sys.stderr, flush=True)
    # saturation: every request waiting at once, so the loop batches as far
    # as its byte budget and batch limit allow; capacity = requests / span
    with Server(slots=slots, max_batch=max_batch, keep_results=False) as srv2:
        t0 = time.perf_counter()
        sreqs = [srv2.submit(p, c.thr, arrival=t0) for p, c in zip(pts, clouds)]
        for r in sreqs:
            r.wait(timeout=300)
        t_sat = max(r.t_done for r in sreqs) - t0
    assert all(sum(r.counts) == n for r, n in zip(sreqs, simp)), "served counts differ from plain builds"
    sat_sizes = [r.batch_size for r in sreqs]
    print("[bench] serving: saturation done", file=sys.stderr, flush=True)
    total = sum(simp[warm:])
    sizes = [r.batch_size for r in reqs]
    return {"qps": qps, "plain_capacity_rps": round(mu, 2), "requests": requests, "warmup_requests": warm,
            "simplices": total,
            "capacity": {"plain_rps": round(mu, 2), "plain_simplices_per_s": sum(simp) * mu / requests,
                         "served_rps": round(requests / t_sat, 2), "served_simplices_per_s": sum(simp) / t_sat,
                         "served_mean_batch": round(sum(sat_sizes) / len(sat_sizes), 3),
                         "served_over_plain": round(requests / t_sat / mu, 3)},
            "plain_fifo": dict(_pcts(lat_plain[warm:]), simplices_per_s=total / span_plain),
            "served": dict(_pcts(lat_srv[warm:]), simplices_per_s=total / span_srv, slots=slots,
                           max_batch=max_batch, batches=srv.batches,
                           mean_batch=round(sum(sizes) / len(sizes), 3), peak_bytes=srv.peak_bytes)}


def _copy_calibration(torch, mib=256):
    """A plain device copy of known size, so FETCH_SIZE / WRITE_SIZE of other
    kernels can be scaled to bytes (launched only with --copy-calib)."""
    n = mib * 1024 * 1024
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"[copy-calib] copied {n} bytes", file=sys.stderr, flush=True)


def _main_batched(vr, torch, args):
    """The 512-cloud workload as the timed step: one batched build."""
    import workloads

    clouds = workloads.batched()
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    thrs = [c.thr for c in clouds]
    torch.cuda.synchronize()
    tuned = _schedule(vr, args, pts, thrs)  # one-time, untimed
    prev = None
    for _ in range(max(args.warmup, 2)):  # two results alive at once, as in the timed loop
        b = vr.build_batch(pts, thrs, timing="write")
        if prev is not None:
            prev.free()
        prev = b
    torch.cuda.synchronize()
    prev.free()
    tw = []
    prev = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b = vr.build_batch(pts, thrs, timing="write")
        if prev is not None:
            tw.append(prev.stage_ms()["tri_write"])
            prev.free()
        prev = b
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tw.append(prev.stage_ms()["tri_write"])
    counts = [it.counts for it in prev]
    prev.free()
    n, K, T = (sum(c[i] for c in counts) for i in range(3))
    simp = n + K + T
    tri_ms = sum(tw) / len(tw)
    alg = _enum_bytes(n, K, T, sum(c[0] ** 2 for c in counts))
    achieved = alg / (tri_ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "filtered simplices/sec (VR dim<=2, bit-exact)", "value": simp * args.steps / el,
        "unit": "simplices/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batched512_r3", "clouds": len(clouds), "points": n, "kept_edges": K,
                   "triangles": T, "simplices_per_step": simp,
                   "schedule": list(tuned) if tuned else "default"},
        "roofline": {"bound": "hbm", "kernel": "k_tri_write", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic("batched512"),
                     "algorithmic_bytes": int(alg), "avg_ms": round(tri_ms, 5),
                     "fused_edge_bytes": int(_edge_bytes(K))}}), flush=True)


def _schedule(vr, args, pts, thr):
    """The main workload's schedule: pinned with --schedule, else tuned once
    (untimed), else the library's default."""
    if args.schedule:
        sched = tuple(int(x) for x in args.schedule.split(","))
        vr.set_schedule(pts, thr, sched)
        return sched
    return vr.autotune(pts, thr) if not args.no_tune else None


def _hamming(vr, torch, tune=True, steps=5, warmup=2, sched=None):
    """Dissimilarity-matrix input: pairwise Hamming distances of 1088 synthetic
    binary sequences (the shape of the paper's sequence example), every pair
    kept: C(1088, 3) = 214 million triangles per build."""
    import workloads

    M = torch.from_numpy(workloads.hamming_matrix(1088, 1088)).to("cuda:0")
    thr = ("full", 0, 1)
    if sched:
        vr.set_schedule(M, thr, sched, matrix=True)
        sch = sched
    else:
        sch = vr.autotune(M, thr, matrix=True) if tune else None
    el, cnt, tw = _time_builds(vr, torch, M, thr, steps, warmup, build=vr.build_matrix)
    a = _enum_bytes(cnt[0], cnt[1], cnt[2], cnt[0] ** 2)
    del M
    return {"value": sum(cnt) * steps / el, "unit": "simplices/s", "ms_per_step": 1e3 * el / steps,
            "steps": steps, "counts": list(cnt), "schedule": list(sch) if sch else "default",
            "input": "int32 1088 x 1088 Hamming matrix of 96-bit sequences, full threshold",
            "tri_write_ms": round(tw, 5),
            "tri_write_frac_hbm": round(a / (tw * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if tw > 0 else None}


def _column_order(vr, torch, reps=20):
    """Per-column stable order of 2000 columns x 1999 entries (the shape of a
    complete 2000-point graph's rank matrix), values uniform in 0..1999000.
    HIP events on the current stream bracket each call (all of its kernels)."""
    import workloads

    colptr, v = workloads.full_columns(2000, 2000, 1999, 1999000)
    cp = torch.from_numpy(colptr).to("cuda:0")
    vv = torch.from_numpy(v).to("cuda:0")
    z = torch.empty(len(v), dtype=torch.int64, device="cuda:0")
    for _ in range(3):
        vr.column_order(cp, vv, out=z)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        vr.column_order(cp, vv, out=z)
        e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
    nnz, ncols = len(v), len(colptr) - 1
    alg = 12 * nnz + 8 * (ncols + 1)  # values in, slots out, column pointers in
    return {"entries_per_s": nnz / (ms * 1e-3), "ms_per_call": round(ms, 5), "wall_ms_per_call": round(1e3 * wall, 5),
            "ncols": ncols, "nnz": nnz, "algorithmic_bytes": alg,
            "frac_hbm": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def _event_median(vr, torch, pts, thr, reps=20, warmup=3):
    """Median over `reps` builds of the time between HIP events recorded on
    the torch stream just before and just after each vr.build call (the call
    enqueues every kernel of the build on that stream), after `warmup`
    builds."""
    for _ in range(warmup):
        vr.build(pts, thr).free()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = vr.build(pts, thr)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
        r.free()
    ts.sort()
    return {"median_ms": round(ts[reps // 2], 5), "min_ms": round(ts[0], 5), "max_ms": round(ts[-1], 5),
            "reps": reps, "warmup": warmup}


def _with_d2h(vr, torch, pts, thr, steps=20, warmup=3):
    """End to end with the outputs copied to the host: each step builds, then
    copies the edge endpoints, edge lengths and triangle keys into pinned
    host buffers (allocated once, before timing) and waits for the copies.
    The library's boundary keeps outputs on the device; this is the rate a
    caller that needs them on the host sees over PCIe."""
    r = vr.build(pts, thr)
    torch.cuda.synchronize()
    n, K, T = r.counts
    r.free()
    h_ij = torch.empty((K, 2), dtype=torch.int32, pin_memory=True)
    h_q = torch.empty(K, dtype=torch.int64, pin_memory=True)
    h_tri = torch.empty(T, dtype=torch.int64, pin_memory=True)

    def step():
        r = vr.build(pts, thr)
        h_ij.copy_(r.edge_ij(), non_blocking=True)
        h_q.copy_(r.edge_q(), non_blocking=True)
        h_tri.copy_(r.tri_key(), non_blocking=True)
        torch.cuda.current_stream().synchronize()
        r.free()

    for _ in range(warmup):
        step()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    el = time.perf_counter() - t0
    out_bytes = 8 * K + 8 * K + 8 * T
    return {"value": (n + K + T) * steps / el, "unit": "simplices/s", "ms_per_step": 1e3 * el / steps,
            "output_bytes_per_step": out_bytes, "d2h_GBps": out_bytes * steps / el / 1e9}


def _schur(vr, torch, reps=10):
    """S = D + C E over F2 (the Schur complement step) for 16384 x 16384
    sparse matrices in compressed columns: C with 32 entries per column on
    average, E and D with 8, seeded.  HIP events on the current stream around
    each whole call (count, scan, the host's read of the entry count, write).
    `xors` counts the row additions: every entry of D plus, for every entry
    (k, j) of E, the entries of column k of C."""
    import numpy as np

    import workloads

    m = k = n = 16384
    C = workloads.f2_csc(101, m, k, 32, empty=0.0)
    E = workloads.f2_csc(102, k, n, 8, empty=0.0)
    D = workloads.f2_csc(103, m, n, 8, empty=0.0)
    lens_c = np.diff(C[0])
    xors = int(len(D[1]) + lens_c[E[1]].sum())
    dev = lambda x: (torch.from_numpy(x[0]).to("cuda:0"), torch.from_numpy(x[1]).to("cuda:0"))
    Cd, Ed, Dd = dev(C), dev(E), dev(D)
    for _ in range(2):
        vr.blockprodsum(m, Cd, Ed, Dd)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        cp, _ = vr.blockprodsum(m, Cd, Ed, Dd)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[reps // 2]
    return {"ms_per_call": round(ms, 5), "m": m, "k": k, "n": n, "xors": xors, "nnz_S": int(cp[-1].item()),
            "xors_per_s": xors / (ms * 1e-3)}


def _apparent(vr, torch, reps=20):
    """Apparent pairs of dimension 1 on the circle1000 build: one pass over
    the triangle keys (8 T bytes in, 4 K out), timed with HIP events on the
    current stream.  Also counts the edges left to a column-serial stage:
    neither paired with a vertex (dimension 0) nor apparent."""
    c = _workload("circle1000")
    pts = torch.from_numpy(c.points).to("cuda:0")
    r = vr.build(pts, c.thr)
    for _ in range(2):
        vr.pairs_dim1_apparent(r)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        app = vr.pairs_dim1_apparent(r)
        e1.record()
    torch.cuda.synchronize()
    ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
    e_low, _ = vr.pairs_dim0(r)
    n, K, T = r.counts
    n_app = int((app >= 0).sum().item())
    n_neg = int((e_low >= 0).sum().item())
    r.free()
    alg = 8 * T + 4 * K
    return {"ms_per_call": round(ms, 5), "apparent_pairs": n_app, "edges_paired_dim0": n_neg,
            "edges_left": K - n_app - n_neg, "frac_hbm": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def _tetra(vr, torch, reps=10):
    """Tetrahedra per largest edge of the circle1000 build (dimension 3),
    timed with HIP events on the current stream."""
    c = _workload("circle1000")
    pts = torch.from_numpy(c.points).to("cuda:0")
    r = vr.build(pts, c.thr)
    for _ in range(2):
        vr.tetra_counts(r)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        cnt = vr.tetra_counts(r)
        e1.record()
    torch.cuda.synchronize()
    ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
    total = int(cnt.sum().item())
    # the listing: offsets, the host's read of the total, the ordered write
    # (16 bytes per tetrahedron)
    _, keys = vr.tetrahedra(r)
    del keys
    torch.cuda.synchronize()
    lt = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, keys = vr.tetrahedra(r)
        e1.record()
        e1.synchronize()
        lt.append(e0.elapsed_time(e1))
        del keys
    r.free()
    lms = sorted(lt)[1]
    return {"ms_per_call": round(ms, 5), "tetrahedra": total, "tetrahedra_per_s": total / (ms * 1e-3),
            "list_ms_per_call": round(lms, 5), "list_GBps": 16 * total / (lms * 1e-3) / 1e9}


def _pairs_dim0(vr, torch, reps=20, workload="circle1000"):
    """Dimension-0 persistence pairs of a build: above 512 points a spanning
    forest in rank order (one work-group: every edge's roots found in
    parallel, at most n - 1 serial unions), timed with HIP events on the
    current stream around each call; the rate is kept edges per second."""
    c = _workload(workload)
    pts = torch.from_numpy(c.points).to("cuda:0")
    r = vr.build(pts, c.thr)
    for _ in range(2):
        vr.pairs_dim0(r)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        vr.pairs_dim0(r)
        e1.record()
    torch.cuda.synchronize()
    ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
    n, K, _ = r.counts
    r.free()
    return {"ms_per_call": round(ms, 5), "n": n, "K": K, "edges_per_s": K / (ms * 1e-3)}


def _pairs_dim1(vr, torch, reps=5, workload="circle1000"):
    """All persistence pairs of dimension 1 and the barcode of dimensions 0
    and 1 of a build (dimension-0 pairs first, as the clearing needs them):
    the apparent pairs in one pass over the keys, then the remaining edge
    columns in rounds that reduce every unsettled column at once.  Wall
    time of the
    three calls (each synchronises for its status), median of reps."""
    c = _workload(workload)
    pts = torch.from_numpy(c.points).to("cuda:0")
    r = vr.build(pts, c.thr)
    torch.cuda.synchronize()
    ts = []
    for i in range(reps + 1):
        t0 = time.perf_counter()
        e_low, _ = vr.pairs_dim0(r)
        toe = vr.pairs_dim1(r, e_low)
        bars, ess2 = vr.barcode(r, e_low, toe)
        torch.cuda.synchronize()
        if i:
            ts.append(time.perf_counter() - t0)
    n, K, T = r.counts
    app = vr.pairs_dim1_apparent(r)
    n_app = int((app >= 0).sum().item())
    n_dim0 = int((e_low >= 0).sum().item())
    n_pair1 = int((toe >= 0).sum().item())
    b = bars.cpu()
    inf = 2 ** 63 - 1
    betti = [int(((b[:, 0] == 0) & (b[:, 2] == inf)).sum()), int(((b[:, 0] == 1) & (b[:, 2] == inf)).sum()), ess2]
    r.free()
    return {"ms_per_call": round(1e3 * sorted(ts)[len(ts) // 2], 4), "n": n, "K": K, "T": T,
            "apparent_pairs": n_app, "columns_reduced": K - n_app - n_dim0, "pairs_dim1": n_pair1,
            "positive_bars_dim1": int(((b[:, 0] == 1) & (b[:, 2] != inf)).sum()), "betti": betti}


def _dim3(vr, torch, reps=3, workload="circle1000"):
    """Dimension 3 (Section 3's bettimax = 2): a maxdim-3 build (the
    triangles, then the tetrahedra counted, scanned, read back and listed)
    and the pairs of dimension 2 (triangles with tetrahedra: apparent pairs
    one wave per triangle, the rest reduced as in dimension 1).  Wall times,
    median of reps; the pairs of dimensions 0 and 1 come first (clearing)."""
    c = _workload(workload)
    pts = torch.from_numpy(c.points).to("cuda:0")
    tb, tp = [], []
    for i in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = vr.build(pts, c.thr, maxdim=3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e_low, _ = vr.pairs_dim0(r)
        toe = vr.pairs_dim1(r, e_low)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tt = vr.pairs_dim2(r, toe)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if i:
            tb.append(t1 - t0)
            tp.append(t3 - t2)
        n, K, T = r.counts
        T3 = r.T3
        paired = int((tt >= 0).sum().item())
        r.free()
    mb, mp = sorted(tb)[len(tb) // 2], sorted(tp)[len(tp) // 2]
    return {"build_ms": round(1e3 * mb, 3), "n": n, "K": K, "T": T, "T3": T3,
            "simplices_per_s": (n + K + T + T3) / mb, "pairs_dim2_ms": round(1e3 * mp, 3), "pairs_dim2": paired}


def _enum_bytes(n, K, T, n2):
    """Algorithmic bytes of the triangle enumeration: triangle keys out (8 T),
    kept ranks in (8 K), the adjacency once (n^2/8 over the clouds)."""
    return 8 * T + 8 * K + n2 / 8.0


def _edge_bytes(K):
    """Bytes of the public edge arrays the writer's grid also emits: 8 K in
    (packed endpoints and length), 16 K out (endpoints, int64 length)."""
    return 24 * K


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixture4000",
                    choices=["circle1000", "mixture4000", "plain64", "batched512", "hamming1088", "colorder2000",
                             "pairs0", "pairs1", "schur16384"],
                    help="mixture4000 (the benchmark line, with side measurements), circle1000, plain64, "
                         "batched512 (one batched build of 512 clouds), or one side measurement alone: "
                         "hamming1088 (matrix input), colorder2000 (column order), pairs0 (dimension-0 pairs and dimension-1 apparent pairs), "
                         "pairs1 (dimension-1 reduction and barcode; dimension 3 and its pairs), "
                         "schur16384 (F2 product and sum)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline and the parity gate")
    ap.add_argument("--no-extra", action="store_true", help="skip the side measurements")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-cloud batched side measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (Poisson stream) side measurement")
    ap.add_argument("--qps", type=float, default=SERVE_QPS,
                    help="serving QPS; 0 measures 0.7 x the plain build's capacity instead")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 256 MiB plain copy")
    ap.add_argument("--no-tune", action="store_true", help="skip the one-time schedule autotuning")
    ap.add_argument("--schedule", default=None,
                    help="pin the main workload's schedule (six comma-separated values, as reported in config) "
                         "instead of tuning it")
    ap.add_argument("--stages", action="store_true", help="print per-stage times to stderr")
    ap.add_argument("--breakdown-reps", type=int, default=10, help="untimed builds for the stage breakdown (0: skip)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(splitting a build over several GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1809_04424_amd as vr

    vr.lib()
    if args.copy_calib:
        _copy_calibration(torch)
    if args.workload == "batched512":
        _main_batched(vr, torch, args)
        return
    if args.workload == "hamming1088":  # the matrix-input workload alone (profiling)
        print(json.dumps({"workload": "hamming1088_full_matrix",
                          **_hamming(vr, torch, tune=not args.no_tune, steps=args.steps, warmup=args.warmup,
                                     sched=tuple(int(x) for x in args.schedule.split(",")) if args.schedule
                                     else None)}),
              flush=True)
        return
    if args.workload == "pairs0":  # pairs of circle1000 alone (profiling)
        print(json.dumps({"workload": "pairs_dim0_circle1000", **_pairs_dim0(vr, torch, reps=args.steps),
                          "pairs_dim1_barcode": _pairs_dim1(vr, torch),
                          "apparent_dim1": _apparent(vr, torch, reps=args.steps),
                          "tetra_counts": _tetra(vr, torch, reps=args.steps)}), flush=True)
        return
    if args.workload == "pairs1":  # the dimension-1 reduction and barcode alone (profiling)
        print(json.dumps({"workload": "pairs_dim1_barcode",
                          "circle1000": _pairs_dim1(vr, torch, reps=args.steps),
                          "mixture4000": _pairs_dim1(vr, torch, reps=args.steps, workload="mixture4000"),
                          "dim3_circle1000": _dim3(vr, torch, reps=args.steps)}), flush=True)
        return
    if args.workload == "schur16384":  # the F2 product and sum alone (profiling)
        print(json.dumps({"workload": "schur_f2_16384", **_schur(vr, torch, reps=args.steps)}), flush=True)
        return
    if args.workload == "colorder2000":  # the per-column order alone (profiling)
        print(json.dumps({"workload": "column_order_2000x1999", **_column_order(vr, torch, reps=args.steps)}),
              flush=True)
        return
    cloud = _workload(args.workload)
    pts = torch.from_numpy(cloud.points).to("cuda:0")
    torch.cuda.synchronize()

    tuned = _schedule(vr, args, pts, cloud.thr)  # one-time, untimed
    el, counts, tri_ms, last = _time_builds(vr, torch, pts, cloud.thr, args.steps, args.warmup, keep_last=True)
    n, K, T = counts
    simplices = n + K + T
    value = simplices * args.steps / el
    ms_step = 1e3 * el / args.steps
    # the CPU baseline's build doubles as the reference of the parity gate
    cpu, parity = None, None
    if not args.no_cpu:
        cpu, f = _cpu_baseline(cloud, _host_threads())
        ok = _parity_gate(last, f)
        del f
        if not ok:
            last.free()
            print(f"bench.py: the device's build of {cloud.name} differs from the oracle's", file=sys.stderr)
            sys.exit(1)
        parity = "bit-exact"
    last.free()
    torch.cuda.synchronize()
    st = _stage_breakdown(vr, torch, pts, cloud.thr, args.breakdown_reps) if args.breakdown_reps > 0 else {}
    if args.stages:
        print(json.dumps({"stages_ms": st}), file=sys.stderr, flush=True)

    enum = _enum_bytes(n, K, T, n * n)
    achieved = enum / (tri_ms * 1e-3) / 1e9 if tri_ms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": "k_tri_write", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(args.workload),
                "algorithmic_bytes": int(enum), "avg_ms": round(tri_ms, 5),
                "fused_edge_bytes": int(_edge_bytes(K)),
                "frac_with_edges": round((enum + _edge_bytes(K)) / (tri_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                if tri_ms > 0 else None}

    extra = {}
    if not args.no_extra and args.workload == "mixture4000":
        c2 = _workload("circle1000")
        p2 = torch.from_numpy(c2.points).to("cuda:0")
        t2s = vr.autotune(p2, c2.thr) if not args.no_tune else None
        e2, cnt2, t2 = _time_builds(vr, torch, p2, c2.thr, 20, 3)
        a2 = _enum_bytes(cnt2[0], cnt2[1], cnt2[2], cnt2[0] ** 2)
        extra["circle1000_r3_p20"] = {
            "value": sum(cnt2) * 20 / e2, "unit": "simplices/s", "ms_per_step": 1e3 * e2 / 20,
            "counts": list(cnt2), "schedule": list(t2s) if t2s else "default",
            "tri_write_ms": round(t2, 5), "tri_write_traffic": _traffic("circle1000"),
            "tri_write_frac_hbm": round(a2 / (t2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if t2 > 0 else None,
            "stages_ms": _stage_breakdown(vr, torch, p2, c2.thr, reps=3) if args.breakdown_reps > 0 else {}}
        extra["hamming1088_full_matrix"] = _hamming(vr, torch, tune=not args.no_tune)
        extra["column_order_2000x1999"] = _column_order(vr, torch)
        extra["pairs_dim0_circle1000"] = _pairs_dim0(vr, torch)
        extra["pairs_dim0_mixture4000"] = _pairs_dim0(vr, torch, workload="mixture4000")
        extra["pairs_dim1_barcode_circle1000"] = _pairs_dim1(vr, torch)
        extra["pairs_dim1_barcode_mixture4000"] = _pairs_dim1(vr, torch, reps=3, workload="mixture4000")
        extra["dim3_circle1000"] = _dim3(vr, torch)
        extra["pairs_dim1_apparent_circle1000"] = _apparent(vr, torch)
        extra["tetra_counts_circle1000"] = _tetra(vr, torch)
        extra["schur_f2_16384"] = _schur(vr, torch)
        extra["mixture4000_outputs_to_host"] = _with_d2h(vr, torch, pts, cloud.thr, steps=5, warmup=1)
        extra["mixture4000_event_timed"] = _event_median(vr, torch, pts, cloud.thr)
        del p2

    if not args.no_batch and args.workload == "mixture4000":
        extra["batched512_r3"] = _batched(vr, torch, tune=not args.no_tune)
    if not args.no_serve and args.workload == "mixture4000":
        extra["serving_poisson"] = _serving(vr, torch, qps=args.qps)

    line = {
        "metric": "filtered simplices/sec (VR dim<=2, bit-exact)",
        "value": value,
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": cloud.name, "n": n, "d": cloud.d, "coords": str(cloud.points.dtype),
                   "threshold": f"{cloud.thr[0]} {cloud.thr[1]}/{cloud.thr[2]}", "kept_edges": K,
                   "triangles": T, "simplices_per_build": simplices,
                   "schedule": list(tuned) if tuned else "default",
                   "timed_loop": "repeat builds of one shape: after the first, each build enqueues its "
                                 "triangle write before the host reads the counts"},
        "roofline": roofline,
        "stages_ms": st,
    }
    if parity:
        line["parity"] = parity
    if extra:
        line["extra"] = extra
    if cpu:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
