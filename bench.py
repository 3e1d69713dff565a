"""Throughput of the FHT + bend-limited DP polyline detector on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config 4096x4096]

One step is one whole detection (band FHT of all k bands, the DP over every
band boundary, the argmax and the backtrace) of one seeded synthetic image
that is already resident in HBM.  The default workload is the 4096x4096
uint16 image with k = 32 bands of 128 rows and a bend bound of 8 shifts.
Prints one JSON line.  The CPU oracle is timed on a bounded sample of the
same workload beside it.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch of each kernel family on the 4096x4096 uint16 image
# (k = 32, bend 8), from two rocprofv3 --pmc runs of `bench.py --probe`
# (FETCH_SIZE, then WRITE_SIZE), each scaled by what the same counter reads
# for a copy of a known size in the same run (`bench.py --summarize-counters`).
# Valid only for the kernel source they were taken on (sha256 of the file);
# otherwise the traffic is unknown and reported as null.
TRAFFIC = {
    "fht_reg_kernel": {"source": "paper_1912_01884_amd/csrc/fhtp_fht.hip",
                      "source_sha256": "e7eee6e6575463104e02e08783cd3137e37f8275f260b872fb3e9b5f019fc535",
                      "fetch_bytes": 36827289, "write_bytes": 142582784},
    "dp_pair_fixed": {"source": "paper_1912_01884_amd/csrc/fhtp_dp.hip",
                     "source_sha256": "a6bf6ca8288b017f2832837c1fe9d972cf6ff7e6104683c978afdf24e9237859",
                     "fetch_bytes": 13988813, "write_bytes": 6653440},
    "dp_step_fixed": {"source": "paper_1912_01884_amd/csrc/fhtp_dp.hip",
                     "source_sha256": "a6bf6ca8288b017f2832837c1fe9d972cf6ff7e6104683c978afdf24e9237859",
                     "fetch_bytes": 8680520, "write_bytes": 6144},
    "walk": {"source": "paper_1912_01884_amd/csrc/fhtp_dp.hip",
            "source_sha256": "a6bf6ca8288b017f2832837c1fe9d972cf6ff7e6104683c978afdf24e9237859",
            "fetch_bytes": 67448, "write_bytes": 192},
}


def byte_model(h, w, k, bpp):
    """Algorithmic HBM bytes of one detection with materialised band tables.

    The image is read once, the tables [k][2n-1][w+n] are written once by the
    FHT and read once by the DP (int32 cells, or uint16 where 8-bit pixels
    keep every line sum below 2^16), and one back-pointer per DP cell and
    band boundary is written ((k-1)(2n-1)w of them, one byte each while 2n-1
    fits a byte, else two).  The DP's value planes are not counted: the
    dataflow keeps them in cache, and their traffic is reported apart.
    """
    n = h // k
    D, W = 2 * n - 1, w + n
    ab = 1 if D <= 256 else 2
    image = h * w * bpp
    # 8-bit pixels and bands of at most 256 rows: bands 0..k-2 are stored as
    # uint16 (every line sum fits), the last one as int32
    narrow = k - 1 if (bpp == 1 and n <= 256 and k >= 2) else 0
    tb = 2 if narrow else 4  # bytes of a table cell of the bands the DP steps read
    tables = D * W * (2 * narrow + 4 * (k - narrow))
    backptr = max(k - 1, 0) * D * w * ab
    return {"image": image, "tables_write": tables, "tables_read": tables, "backptr": backptr,
            "total": image + 2 * tables + backptr, "fht_kernel": image + tables,
            "dp_per_band": tb * D * W + D * w * ab, "table_read_per_band": tb * D * W,
            "backptr_per_band": D * w * ab, "v_plane": 4 * D * w, "table_cell_bytes": tb}


def time_events(fn, reps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps  # ms per call


def cpu_baseline(img, k, bend, seconds):
    """The oracle on all host cores, repeated on the same image for about
    `seconds`; returns the baseline entry and the oracle's answer."""
    import oracle
    h, w = img.shape
    runs = 0
    t0 = time.perf_counter()
    while True:
        res = oracle.detect_polyline(img, k, bend=bend)
        runs += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return ({"value": round(h * w * runs / el / 1e6, 3), "unit": "Mpix/s",
             "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
             "sample": f"{runs} full detection(s) of the {h}x{w} image, {el:.1f} s"},
            (int(res[0]), [int(v) for v in res[1]]))


SINGLE_THREAD_SNIPPET = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle, synth
out = {}
for name, secs in (("64x64", float(sys.argv[2])), ("1024x1024", float(sys.argv[2]))):
    s = synth.make_config(name)
    runs, t0 = 0, time.perf_counter()
    while True:
        oracle.detect_polyline(s.image, s.k, bend=s.bend)
        runs += 1
        el = time.perf_counter() - t0
        if el >= secs:
            break
    out[name] = {"value": round(s.h * s.w * runs / el / 1e6, 3), "unit": "Mpix/s",
                 "ms_per_detection": round(el / runs * 1e3, 3), "cores": oracle.num_threads(),
                 "sample": f"{runs} detection(s), {el:.1f} s"}
print(json.dumps(out))
"""


def cpu_single_thread(seconds):
    """The oracle on one host core (OMP_NUM_THREADS=1, a child process) on the
    64x64 and 1024x1024 workloads."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", SINGLE_THREAD_SNIPPET, ROOT, str(seconds)],
                       capture_output=True, text=True, env=env, timeout=120)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def single_detections(step, stream, reps, flush=None):
    """Per-detection times (ms) of `reps` detections, each timed alone with
    events; `flush` (outside the timed region) evicts the caches first."""
    import torch
    out = []
    for _ in range(reps):
        if flush is not None:
            flush()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step()
        b.record(stream)
        b.synchronize()
        out.append(a.elapsed_time(b))
    out.sort()
    return {"median": round(out[len(out) // 2], 4), "min": round(out[0], 4), "reps": reps}


def mixed_batch(n_images, reps, dev, stream, tune=True, plan_out=None):
    """The mixed-size workload: images/s one detection at a time vs one batched call.

    Both paths get prebuilt arguments and preallocated workspaces, so the
    comparison is between the library's two entry points, not Python overhead.
    With `tune`, the autotuner first picks the launch shapes for this workload
    (both paths then run with them).
    """
    import ctypes as C

    import torch

    import synth
    from paper_1912_01884_amd import autotune, fhtp

    batch = synth.make_mixed_batch(n_images)
    imgs = [torch.from_numpy(s.image).to(dev) for s in batch]
    tuning = None
    if tune:
        res = autotune.tune(imgs, [s.k for s in batch], bends=[s.bend for s in batch], reps=3,
                            stream=stream)
        tuning = res.as_dict()
        if plan_out:
            autotune.save(res, plan_out, workload=f"mixed-size batch of {n_images} images")
    jobs, keep = fhtp.make_jobs(imgs, [s.k for s in batch], bends=[s.bend for s in batch])
    L = fhtp.lib()
    sptr = int(stream.cuda_stream)
    # plain path: one workspace big enough for the largest image, reused in stream order
    single_ws = max(fhtp.detect_workspace_bytes(j.dtype, j.h, j.w, j.k, j.bend) for j in jobs)
    ws1 = torch.empty(single_ws, dtype=torch.uint8, device=dev)
    args1 = [(j.img, j.dtype, j.h, j.w, j.k, j.bend, C.c_void_p(ws1.data_ptr()), single_ws,
              j.score, j.xs, C.c_void_p(sptr)) for j in jobs]

    def plain():
        for a in args1:
            rc = L.fhtp_detect_polyline(*a)
            if rc != 0:
                raise RuntimeError(f"detect_polyline failed: {rc}")

    arr = (fhtp.Job * len(jobs))(*jobs)
    nb = fhtp.batch_workspace_bytes(jobs)
    wsb = torch.empty(nb, dtype=torch.uint8, device=dev)

    def batched():
        rc = L.fhtp_detect_batch(arr, len(jobs), C.c_void_p(wsb.data_ptr()), nb, C.c_void_p(sptr))
        if rc != 0:
            raise RuntimeError(f"detect_batch failed: {rc}")

    plain()
    batched()
    torch.cuda.synchronize()
    ms_plain = time_events(plain, reps, stream)
    ms_batch = time_events(batched, reps, stream)
    first = [(int(sc.cpu()[0]), x.cpu().tolist()) for sc, x in keep]

    # The steady state: the same batch recorded once as a HIP graph
    # (fhtp_plan_create / _capture) and replayed with fhtp_plan_launch.
    plan = fhtp.Plan(imgs, [s.k for s in batch], bends=[s.bend for s in batch],
                     scores=[sc for sc, _ in keep], xss=[x for _, x in keep], ws=wsb)
    for sc, x in keep:
        sc.fill_(-1)
        x.fill_(-1)
    plan.launch(stream)
    torch.cuda.synchronize()
    same = [(int(sc.cpu()[0]), x.cpu().tolist()) for sc, x in keep] == first
    ms_graph = time_events(lambda: plan.launch(stream), reps, stream)
    plan.destroy()
    mpix = sum(s.h * s.w for s in batch) / 1e6
    best = min(ms_batch, ms_graph)
    return {"images": n_images, "mpix_per_batch": round(mpix, 2),
            "plain_images_per_s": round(n_images / (ms_plain * 1e-3), 1),
            "batched_images_per_s": round(n_images / (ms_batch * 1e-3), 1),
            "graph_images_per_s": round(n_images / (ms_graph * 1e-3), 1),
            "plain_ms": round(ms_plain, 3), "batched_ms": round(ms_batch, 3),
            "graph_ms": round(ms_graph, 3), "graph_identical_to_batched": same,
            "speedup": round(ms_plain / ms_batch, 2),
            "graph_speedup": round(ms_plain / ms_graph, 2),
            "batched_mpix_per_s": round(mpix / (best * 1e-3), 1),
            "tuning": tuning}


def serving(dev, rates, count, streams=4, max_batch=256):
    """Open-loop Poisson arrivals of the mixed-size requests: continuous batching vs plain.

    Requests are the 256 mixed-size images (device resident) in a seeded
    random order; arrivals are a Poisson stream at each rate (and all at once
    for the saturation run).  Latency is host-observed completion minus the
    scheduled arrival.  The two servers must return identical results.
    """
    import numpy as np
    import torch

    import synth
    from paper_1912_01884_amd import fhtp
    from paper_1912_01884_amd.serve import (FhtpBackend, PlainServer, Request, Server,
                                            poisson_arrivals, run_open_loop)

    batch = synth.make_mixed_batch(256)
    imgs = [torch.from_numpy(s.image).to(dev) for s in batch]
    pick = np.random.default_rng([191201884, 5, 998]).integers(0, len(batch), size=count)
    scores = torch.zeros((2, count), dtype=torch.int32, device=dev)
    xss = torch.zeros((2, count, 17), dtype=torch.int32, device=dev)
    max_bytes = max(fhtp.detect_workspace_bytes(s.dtype_code, s.h, s.w, s.k, fhtp.make_bend(s.bend))
                    for s in batch)
    backend = FhtpBackend(dev, arena_bytes=8 << 30, streams=streams)
    plain = PlainServer(dev, max_request_bytes=max_bytes)
    torch.cuda.synchronize()

    def requests(which):
        out = []
        for i, q in enumerate(pick):
            s = batch[q]
            out.append(Request(img=imgs[q], k=s.k, bend=s.bend, score=scores[which, i:i + 1],
                               xs=xss[which, i, :s.k + 1], rid=i))
        return out

    res = {}
    for rate in rates:
        arr = poisson_arrivals(rate, count, [191201884, 5, 999])
        srv = Server(backend, streams=streams, max_batch=max_batch)
        a = run_open_loop(srv, requests(0), arr, timeout=300)
        a["groups"] = srv.groups_launched
        b = run_open_loop(plain, requests(1), arr, timeout=300)
        torch.cuda.synchronize()
        same = bool(torch.equal(scores[0], scores[1]) and torch.equal(xss[0], xss[1]))
        key = "saturation" if rate == float("inf") else f"{int(rate)}_per_s"
        res[key] = {"server": a, "plain": b, "identical_results": same,
                    "throughput_ratio": round(a["images_per_s"] / b["images_per_s"], 2)}
        scores.zero_()
        xss.zero_()
    res["requests_per_rate"] = count
    res["streams"] = streams
    res["max_group"] = max_batch
    return res




def source_sha(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_of(family):
    """Counter bytes (fetched + written) per launch of a kernel family on the
    4096x4096 workload, or None when not taken on the current source."""
    t = TRAFFIC.get(family)
    if not t or source_sha(t["source"]) != t["source_sha256"]:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def kernel_alg_bytes(family, model, launches):
    """Algorithmic bytes of one launch of a kernel family in one detection
    (the byte model's per-unit figures times the units one launch handles)."""
    if family == "fht_reg_kernel" and launches == 1:
        return model["fht_kernel"]  # the image read, every band's table written
    per_band = model["dp_per_band"]  # a band's table read, its back-pointers written
    bands = {"dp_pair_fixed": 2, "dp_triple_fixed": 3, "dp_step_fixed": 1,
             "dp_step_generic": 1}.get(family)
    return None if bands is None else bands * per_band


def kernel_breakdown(step, reps):
    """Per-kernel launch times of `reps` detections, from the library's event
    brackets (fhtp_timing_start / _stop) on the launch stream."""
    import torch
    from paper_1912_01884_amd import fhtp
    torch.cuda.synchronize()
    fhtp.timing_start()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    fam = fhtp.timing_stop()
    return {name: {"launches_per_detection": round(n / reps, 3),
                   "avg_launch_us": round(ms * 1e3 / n, 3),
                   "us_per_detection": round(ms * 1e3 / reps, 3)}
            for name, (n, ms) in fam.items()}


def roofline_of(family, info, model, headline=True):
    """Roofline entry of a kernel family; the counter traffic (taken on the
    4096x4096 workload) only for that workload."""
    per = info["launches_per_detection"]
    alg = kernel_alg_bytes(family, model, per)
    if alg is None:
        return None
    t = info["avg_launch_us"] * 1e-6
    gbps = alg / t / 1e9
    out = {"bound": "hbm", "kernel": family, "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS,
           "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
           "traffic": traffic_of(family) if headline else None,
           "algorithmic_bytes": alg, "avg_launch_us": info["avg_launch_us"],
           "launches_per_detection": per}
    if out["traffic"] is not None:
        tg = out["traffic"] / t / 1e9
        out["achieved_traffic"] = round(tg, 1)
        out["traffic_frac"] = round(tg / HBM_PEAK_GBPS, 4)
        out["traffic_over_algorithmic"] = round(out["traffic"] / alg, 3)
    return out


def other_config(name, steps, warmup, dev, stream, tune=True):
    """A smaller workload (the 64x64 or 1024x1024 image) timed like the
    headline step, with its kernel breakdown and the answer checked against
    the oracle."""
    import torch

    import oracle
    import synth
    from paper_1912_01884_amd import autotune, fhtp

    s = synth.make_config(name)
    h, w, k, B = s.h, s.w, s.k, s.bend
    img = torch.from_numpy(s.image).to(dev)
    dt = fhtp.FHTP_U8 if s.image.dtype.itemsize == 1 else fhtp.FHTP_U16
    ws = torch.empty(fhtp.detect_workspace_bytes(dt, h, w, k, fhtp.make_bend(B)), dtype=torch.uint8,
                     device=dev)
    score = torch.empty(1, dtype=torch.int32, device=dev)
    xs = torch.empty(k + 1, dtype=torch.int32, device=dev)

    def step():
        fhtp.detect_polyline(img, k, bend=B, ws=ws, score=score, xs=xs, stream=stream)

    previous = fhtp.tune_get()
    tuning = None
    if tune:
        tuning = autotune.tune([img], [k], bends=[B], reps=max(5, steps // 2), stream=stream)
    try:
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ms_eager = time_events(step, steps, stream)
        got = (int(score.cpu()[0]), xs.cpu().numpy().tolist())
        kernels = kernel_breakdown(step, max(5, steps // 2))
        # the same detection replayed as a recorded graph (one launch per step)
        plan = fhtp.Plan([img], [k], bends=[B], scores=[score], xss=[xs])
        for _ in range(warmup):
            plan.launch(stream)
        torch.cuda.synchronize()
        ms_graph = time_events(lambda: plan.launch(stream), steps, stream)
        got_graph = (int(score.cpu()[0]), xs.cpu().numpy().tolist())
        plan.destroy()
    finally:
        fhtp.tune_set(previous)
    ms = min(ms_eager, ms_graph)
    want = oracle.detect_polyline(s.image, k, bend=B)
    model = byte_model(h, w, k, s.image.dtype.itemsize)
    g = model["total"] / (ms * 1e-3) / 1e9
    return {"workload": f"{h}x{w} {s.image.dtype.name} image, k={k} bands of {h // k} rows, "
                        f"bend bound {B} shifts",
            "ms_per_detection": round(ms, 4), "eager_ms": round(ms_eager, 4),
            "graph_ms": round(ms_graph, 4), "mpix_per_s": round(h * w / (ms * 1e-3) / 1e6, 2),
            "images_per_s": round(1e3 / ms, 1), "kernels": kernels,
            "roofline_detection": {"achieved": round(g, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                   "frac": round(g / HBM_PEAK_GBPS, 4),
                                   "algorithmic_bytes": model["total"]},
            "tuned_rules": None if tuning is None else tuning.rules,
            "parity": got == got_graph == (int(want[0]), [int(v) for v in want[1]])}


def copy_bandwidth(dev, stream, reps=10):
    """Attainable HBM bandwidth: a 1 GiB device-to-device copy timed with events
    (bytes read + bytes written per second)."""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = time_events(lambda: b.copy_(a), reps, stream)
    del a, b
    return {"bytes": 2 << 30, "gbps": round((2 << 30) / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round((2 << 30) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def probe(dev):
    """A short program for hardware-counter runs: a 256 MiB fill and copy of known
    size (counter calibration), then one whole detection of the 4096x4096 image."""
    import torch

    import synth
    from paper_1912_01884_amd import fhtp

    s = synth.make_large()
    img = torch.from_numpy(s.image).to(dev)
    a = torch.empty(64 << 20, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    a.fill_(1)
    b.copy_(a)
    score, xs = fhtp.detect_polyline(img, s.k, bend=s.bend)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "fill + copy 268435456 bytes; detect_polyline 4096x4096 k=32",
                      "score": int(score.cpu()[0])}), flush=True)


# ---- rocprofv3 output summaries ------------------------------------------------

def _csv_rows(folder, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no *{suffix} under {folder}")
    return rows


def _short(name, width=90):
    name = name.replace("void ", "").replace("fhtp::(anonymous namespace)::", "")
    return name if len(name) <= width else name[:width - 3] + "..."


def summarize_trace(folder):
    """Markdown table of a `rocprofv3 --kernel-trace --stats` run: per kernel
    calls and durations, then the kernels of the last whole detection."""
    rows = _csv_rows(folder, "kernel_trace.csv")
    by = {}
    seq = []
    for r in rows:
        name = _short(r["Kernel_Name"])
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        by.setdefault(name, []).append(us)
        seq.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), name, us))
    total = sum(sum(v) for v in by.values())
    print("| kernel | calls | avg us | median us | min us | max us | share |")
    print("|---|---|---|---|---|---|---|")
    for name, v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:14]:
        v = sorted(v)
        print(f"| `{name}` | {len(v)} | {sum(v) / len(v):.2f} | {v[len(v) // 2]:.2f} | "
              f"{v[0]:.2f} | {v[-1]:.2f} | {100 * sum(v) / total:.1f}% |")
    seq.sort()
    starts = [q for q, e in enumerate(seq) if e[2].startswith("fht_reg_kernel")]
    for q0 in reversed(starts):
        q1 = next((q for q in range(q0, len(seq)) if seq[q][2].startswith("walk")), None)
        if q1 is None or any(", true" in e[2] for e in seq[q0:q1 + 1]):
            continue  # incomplete, or a through-point query (pinned kernels)
        print("\nOne detection (the last unpinned one traced; kernels in launch order):\n")
        run = {}
        order = []
        for e in seq[q0:q1 + 1]:
            if e[2] not in run:
                order.append(e[2])
            run.setdefault(e[2], []).append(e[3])
        for name in order:
            v = run[name]
            if len(v) == 1:
                print(f"- `{name}`: {v[0]:.2f}")
            else:
                print(f"- `{name}` x{len(v)}: total {sum(v):.1f}, mean {sum(v) / len(v):.2f}, "
                      f"min {min(v):.2f}, max {max(v):.2f}")
        print(f"- first kernel start to walk end: {(seq[q1][1] - seq[q0][0]) / 1e3:.1f}")
        break


def summarize_counters(fetch_dir, write_dir):
    """Markdown table of two `rocprofv3 --pmc` runs of `bench.py --probe`
    (FETCH_SIZE, then WRITE_SIZE): the counters per dispatch, scaled by what
    they read for the probe's 256 MiB copy (FETCH_SIZE) and fill (WRITE_SIZE)."""
    mib256 = 256 * 1024  # KiB

    def per_kernel(folder, counter):
        out = {}
        for r in _csv_rows(folder, "counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(_short(r["Kernel_Name"], 200), []).append(float(r["Counter_Value"]))
        return out

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    # the probe's 256 MiB device copy is the largest copyBuffer dispatch (the
    # image's upload from the host is another one), its fill the FillFunctor one
    copy_f = max(x for k, v in fetch.items() if "copyBuffer" in k for x in v)
    fill_w = max(x for k, v in write.items() if "FillFunctor" in k for x in v)
    sf = copy_f / mib256
    sw = fill_w / mib256
    print(f"Calibration: FETCH_SIZE reads {sf:.4f} x the bytes the copy fetched, "
          f"WRITE_SIZE {sw:.4f} x the bytes the fill wrote.\n")
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetched (scaled) | "
          "written (scaled) |")
    print("|---|---|---|---|---|---|")
    for name in fetch:
        if name not in write:
            continue
        f, w = fetch[name], write[name]
        mf, mw = sum(f) / len(f), sum(w) / len(w)
        print(f"| `{_short(name)}` | {len(f)} | {mf:.1f} | {mw:.1f} | "
              f"{mf / sf * 1024 / 1e6:.2f} MB | {mw / sw * 1024 / 1e6:.2f} MB |")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="4096x4096", choices=["64x64", "1024x1024", "4096x4096"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-images", type=int, default=256,
                    help="images of the mixed-size workload timed batched vs one at a time "
                         "(0 skips it)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per arrival rate in the serving run (0 skips it)")
    ap.add_argument("--serve-streams", type=int, default=4,
                    help="streams of the continuous-batching server (groups in flight at once)")
    ap.add_argument("--serve-rates", default="200,1000,5000,inf",
                    help="Poisson arrival rates (requests/s) of the serving run; inf = all at once")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the 64x64 and 1024x1024 workloads")
    ap.add_argument("--no-tune", action="store_true",
                    help="run with the library's default launch shapes (no autotuning)")
    ap.add_argument("--dp-steps", type=int, default=0, choices=[0, 1, 2, 3],
                    help="force this many DP steps per launch for fixed windows instead of "
                         "tuning (for profiling one kernel family; 0: tune)")
    ap.add_argument("--plan-out", default=None,
                    help="save the mixed workload's tuned rules to this JSON file")
    ap.add_argument("--probe", action="store_true",
                    help="run the short counter-calibration program instead of the benchmark")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print the kernel table of a rocprofv3 --kernel-trace run and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the traffic table of two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()

    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(independent images and requests would shard one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1912_01884_amd import fhtp

    from paper_1912_01884_amd import autotune
    if args.dp_steps:
        fhtp.tune_set([autotune.rule(window=0, dc=8, steps=args.dp_steps)])
    if args.probe:
        probe(torch.device("cuda:0"))
        return

    s = synth.make_config(args.config)
    h, w, k, B = s.h, s.w, s.k, s.bend
    bpp = s.image.dtype.itemsize
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    img = torch.from_numpy(s.image).to(dev)
    dt = fhtp.FHTP_U8 if bpp == 1 else fhtp.FHTP_U16
    bend = fhtp.make_bend(B)
    ws = torch.empty(fhtp.detect_workspace_bytes(dt, h, w, k, bend), dtype=torch.uint8, device=dev)
    score = torch.empty(1, dtype=torch.int32, device=dev)
    xs = torch.empty(k + 1, dtype=torch.int32, device=dev)

    def step():
        fhtp.detect_polyline(img, k, bend=B, ws=ws, score=score, xs=xs, stream=stream)

    # Launch shapes for this workload, picked by the autotuner before the
    # timed region (results are the same under every candidate).
    tuning = {"forced_dp_steps": args.dp_steps} if args.dp_steps else None
    if not args.no_tune and not args.dp_steps:
        tuning = autotune.tune([img], [k], bends=[B], reps=max(5, args.steps // 2),
                               stream=stream).as_dict()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_eager = time_events(step, args.steps, stream)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0
    result = (int(score.cpu()[0]), xs.cpu().numpy().tolist())

    # The same detection recorded once as a HIP graph by the library's plan
    # calls (fhtp_plan_create / _capture) and replayed with fhtp_plan_launch:
    # one graph launch per step instead of one launch per kernel.
    plan = fhtp.Plan([img], [k], bends=[B], scores=[score], xss=[xs])

    def replay():
        plan.launch(stream)

    for _ in range(args.warmup):
        replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_graph = time_events(replay, args.steps, stream)
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t0
    graph_result = (int(score.cpu()[0]), xs.cpu().numpy().tolist())
    # Both are full timed runs of the same detection; the step time is the
    # faster of the two submission paths (graph replays carry a fixed host
    # cost per launch that can exceed the GPU time of one detection).
    ms_per_step = max(min(ms_graph, ms_eager), 1e-9)
    launch = ("fhtp_plan_launch: hip graph replay of one detection" if ms_graph <= ms_eager
              else "fhtp_detect_polyline: one call per detection, kernels launched on the stream")

    # Per-kernel launch times of the same detection (event brackets on the
    # launch stream, outside the timed region above).
    kernels = kernel_breakdown(step, max(5, args.steps // 2))

    # Single detections timed one by one: warm (tables and planes of the
    # previous detection still in L2/MALL) and cold (a 1 GiB buffer written
    # between detections, outside the timed region, evicts L2 and MALL).
    single_warm = single_detections(step, stream, 20)
    flush_buf = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    single_cold = single_detections(step, stream, 10, flush=lambda: flush_buf.fill_(1))
    del flush_buf
    copy_bw = copy_bandwidth(dev, stream)

    # Phase timings on the same stream: the band FHT and the DP.
    tables = torch.empty(fhtp.table_shape(h, w, k), dtype=torch.int32, device=dev)
    fws_n = fhtp.fht_workspace_bytes(dt, h, w, k)
    fws = torch.empty(max(fws_n, 1), dtype=torch.uint8, device=dev)
    dws = torch.empty(fhtp.dp_workspace_bytes(h, w, k, bend), dtype=torch.uint8, device=dev)
    ms_fht = time_events(lambda: fhtp.fht_bands(img, k, tables=tables, ws=fws if fws_n else None,
                                                stream=stream), args.steps, stream)
    ms_dp = time_events(lambda: fhtp.polyline_dp(tables, h, w, k, bend=B, ws=dws, score=score,
                                                 xs=xs, stream=stream), args.steps, stream)

    model = byte_model(h, w, k, bpp)
    # The kernel with the most time per detection carries the roofline object.
    headline = (h, w, k, bpp) == (4096, 4096, 32, 2)
    roofs = {f: roofline_of(f, info, model, headline) for f, info in kernels.items()}
    ranked = sorted((f for f in roofs if roofs[f] is not None),
                    key=lambda f: -kernels[f]["us_per_detection"])
    dominant = ranked[0] if ranked else None

    def whole(ms):
        g = model["total"] / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": "whole detection", "achieved": round(g, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(g / HBM_PEAK_GBPS, 4),
                "ms": round(ms, 4), "algorithmic_bytes": model["total"]}

    # DP phase: the tables it reads and the back-pointers it writes (the byte
    # model's DP share); the value planes it passes between launches are
    # reported apart (each launch reads one plane and writes one).
    dp_launches = sum(v["launches_per_detection"] for f, v in kernels.items()
                      if f.startswith("dp_"))
    dp_bytes = model["tables_read"] + model["backptr"]
    dp_gbps = dp_bytes / (ms_dp * 1e-3) / 1e9
    line = {
        "metric": "FHT+DP Mpix/s & HBM GB/s @4096²,k=32; batched imgs/s vs plain; p99 ms",
        "value": round(h * w / (ms_per_step * 1e-3) / 1e6, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "wall_ms_per_step": round((wall_graph if ms_graph <= ms_eager else wall_eager) * 1e3
                                  / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{h}x{w} {s.image.dtype.name} image, k={k} "
                               f"bands of {h // k} rows, bend bound {B} shifts, one image per step",
                   "h": h, "w": w, "k": k, "bend": B, "pixel": s.image.dtype.name},
        "images_per_s": round(1e3 / ms_per_step, 2),
        "hbm_gbps_model": round(model["total"] / (ms_per_step * 1e-3) / 1e9, 1),
        "model_bytes": {q: model[q] for q in ("image", "tables_write", "tables_read", "backptr",
                                              "total")},
        "launch": launch,
        "tuning": tuning,
        "eager_ms_per_step": round(ms_eager, 4),
        "graph_ms_per_step": round(ms_graph, 4),
        "phase_ms": {"fht_bands": round(ms_fht, 4), "polyline_dp": round(ms_dp, 4)},
        "kernels": kernels,
        "single_detection_ms": {"warm": single_warm, "cold": single_cold},
        "roofline": roofs.get(dominant),
        "roofline_fht": roofs.get("fht_reg_kernel"),
        "roofline_detection": {"warm": whole(ms_per_step), "cold": whole(single_cold["median"])},
        "roofline_dp_phase": {"bound": "hbm", "kernel": "every DP launch + walk",
                              "achieved": round(dp_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                              "frac": round(dp_gbps / HBM_PEAK_GBPS, 4),
                              "algorithmic_bytes": dp_bytes, "ms": round(ms_dp, 4),
                              "dp_launches": round(dp_launches, 3),
                              "v_plane_bytes_per_launch": 2 * model["v_plane"]},
        "copy_bandwidth": copy_bw,
    }
    # The DP under the other bend forms on the same tables: the angle bound of
    # eqs. (6)-(7) and the unbounded case of Section 2.2 (scanned windows).
    forms = {}
    sc_f = torch.empty(1, dtype=torch.int32, device=dev)
    xs_f = torch.empty(k + 1, dtype=torch.int32, device=dev)
    for name, kw in [("shift_bound_8", dict(bend=B)), ("angle_10deg", dict(gamma=math.radians(10))),
                     ("angle_30deg", dict(gamma=math.radians(30))),
                     ("unbounded", dict(bend=2 * (h // k) - 2))]:
        bb = fhtp.make_bend(kw.get("bend"), kw.get("gamma"))
        wsf = torch.empty(fhtp.dp_workspace_bytes(h, w, k, bb), dtype=torch.uint8, device=dev)
        forms[name] = round(time_events(
            lambda: fhtp.polyline_dp(tables, h, w, k, ws=wsf, score=sc_f, xs=xs_f, stream=stream,
                                     **kw), max(3, args.steps // 5), stream), 4)
        del wsf
    line["dp_ms_by_bend_form"] = forms
    # A through-point query (Sections 2.2-2.3): the whole detection with the
    # polyline pinned at the middle band boundary, at the column the unpinned
    # answer passes there.
    if k >= 2:
        pj = k // 2
        pin = (pj, int(result[1][pj]))
        opt = fhtp.make_options(0, False, pin)
        wsp = torch.empty(fhtp.detect_ex_workspace_bytes(dt, h, w, k, bend, opt), dtype=torch.uint8,
                          device=dev)
        sc_p = torch.empty(1, dtype=torch.int32, device=dev)
        xs_p = torch.empty(k + 1, dtype=torch.int32, device=dev)
        line["through_point_ms"] = {
            "pin": list(pin),
            "detect_ms": round(time_events(
                lambda: fhtp.detect_polyline_ex(img, k, bend=B, pin=pin, ws=wsp, score=sc_p, xs=xs_p,
                                                stream=stream), max(3, args.steps // 5), stream), 4),
        }
        del wsp
    if args.config == "4096x4096" and not args.no_other_configs:
        line["other_configs"] = {c: other_config(c, max(20, args.steps), args.warmup, dev, stream,
                                                 tune=not args.no_tune)
                                 for c in ("64x64", "1024x1024")}
    if args.batch_images > 0:
        line["mixed_batch"] = mixed_batch(args.batch_images, max(3, args.steps // 10), dev, stream,
                                          tune=not args.no_tune, plan_out=args.plan_out)
    if args.serve_requests > 0:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        line["serving"] = serving(dev, rates, args.serve_requests, streams=args.serve_streams)
        k1000 = line["serving"].get("1000_per_s")
        if k1000:
            line["p99_ms"] = k1000["server"]["p99_ms"]
    if not args.no_cpu_baseline:
        base, want = cpu_baseline(s.image, k, B, args.cpu_seconds)
        base["single_thread"] = cpu_single_thread(3.0)
        line["cpu_baseline"] = base
    else:
        import oracle
        want = oracle.detect_polyline(s.image, k, bend=B)
        want = (int(want[0]), [int(v) for v in want[1]])
    # The timed detection's answer (eager calls and graph replays) against the oracle.
    line["parity"] = bool(result == want and graph_result == want and
                          all(o["parity"] for o in line.get("other_configs", {}).values()))
    line["result"] = {"score": result[0], "x0": result[1][0], "xk": result[1][-1]}
    print(json.dumps(line), flush=True)
    if not line["parity"]:
        print(f"parity failure: gpu {result} / {graph_result}, oracle {want}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
