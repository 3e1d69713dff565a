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

# HBM bytes per launch of the band FHT kernel on the 4096x4096 uint16 image
# (k = 32), from two rocprofv3 --pmc runs of `bench.py --probe` (FETCH_SIZE,
# then WRITE_SIZE), each scaled by what the same counter reads for a copy of a
# known size in the same run.  Valid only for the kernel source they were
# taken on (sha256 of csrc/fhtp_fht.hip); otherwise the traffic is unknown.
FHT_TRAFFIC = {"source_sha256": "7b1ac4b7416bda6e4842dd87714b9d40e083681e4821b0d889f36885ddba7dc4",
               "fetch_bytes": 46875988, "write_bytes": 151035200}


def byte_model(h, w, k, bpp):
    """Algorithmic HBM bytes of one detection with materialised band tables."""
    n = h // k
    D, W = 2 * n - 1, w + n
    image = h * w * bpp
    tables = 4 * k * D * W
    # back-pointer planes for bands 2..k-1 (the first successor is recorded by
    # the last step with its keys)
    backptr = max(k - 2, 0) * D * w * (1 if D <= 256 else 2)
    return {"image": image, "tables_write": tables, "tables_read": tables, "backptr": backptr,
            "total": image + 2 * tables + backptr, "fht_kernel": image + tables}


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
    import oracle
    h, w = img.shape
    runs = 0
    t0 = time.perf_counter()
    while True:
        oracle.detect_polyline(img, k, bend=bend)
        runs += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": round(h * w * runs / el / 1e6, 3), "unit": "Mpix/s",
            "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{runs} full detection(s) of the {h}x{w} image, {el:.1f} s"}


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


def mixed_batch(n_images, reps, dev, stream):
    """The mixed-size workload: images/s one detection at a time vs one batched call.

    Both paths get prebuilt arguments and preallocated workspaces, so the
    comparison is between the library's two entry points, not Python overhead.
    """
    import ctypes as C

    import torch

    import synth
    from paper_1912_01884_amd import fhtp

    batch = synth.make_mixed_batch(n_images)
    imgs = [torch.from_numpy(s.image).to(dev) for s in batch]
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
    mpix = sum(s.h * s.w for s in batch) / 1e6
    return {"images": n_images, "mpix_per_batch": round(mpix, 2),
            "plain_images_per_s": round(n_images / (ms_plain * 1e-3), 1),
            "batched_images_per_s": round(n_images / (ms_batch * 1e-3), 1),
            "plain_ms": round(ms_plain, 3), "batched_ms": round(ms_batch, 3),
            "speedup": round(ms_plain / ms_batch, 2),
            "batched_mpix_per_s": round(mpix / (ms_batch * 1e-3), 1)}


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


def fht_traffic():
    import hashlib
    if FHT_TRAFFIC is None:
        return None
    src = os.path.join(ROOT, "paper_1912_01884_amd", "csrc", "fhtp_fht.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != FHT_TRAFFIC["source_sha256"]:
        return None
    return FHT_TRAFFIC["fetch_bytes"] + FHT_TRAFFIC["write_bytes"]


def probe(dev):
    """A short program for hardware-counter runs: a 256 MiB fill and copy of known
    size (counter calibration), then one band FHT and one DP of the 4096x4096 image."""
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
    tables = fhtp.fht_bands(img, s.k)
    score, xs = fhtp.polyline_dp(tables, s.h, s.w, s.k, bend=s.bend)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy 268435456 bytes; fht_bands + polyline_dp 4096x4096 k=32",
                      "score": int(score.cpu()[0])}), flush=True)


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
    ap.add_argument("--serve-rates", default="200,1000,5000,inf",
                    help="Poisson arrival rates (requests/s) of the serving run; inf = all at once")
    ap.add_argument("--probe", action="store_true",
                    help="run the short counter-calibration program instead of the benchmark")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(independent images and requests would shard one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1912_01884_amd import fhtp

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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_eager = time_events(step, args.steps, stream)
    torch.cuda.synchronize()
    wall_eager = time.perf_counter() - t0

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
    # Both are full timed runs of the same detection; the step time is the
    # faster of the two submission paths (graph replays carry a fixed host
    # cost per launch that can exceed the GPU time of one detection).
    ms_per_step = max(min(ms_graph, ms_eager), 1e-9)
    launch = ("fhtp_plan_launch: hip graph replay of one detection" if ms_graph <= ms_eager
              else "fhtp_detect_polyline: one call per detection, kernels launched on the stream")

    # Single detections timed one by one: warm (tables and planes of the
    # previous detection still in L2/MALL) and cold (a 1 GiB buffer written
    # between detections, outside the timed region, evicts L2 and MALL).
    single_warm = single_detections(step, stream, 20)
    flush_buf = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    single_cold = single_detections(step, stream, 10, flush=lambda: flush_buf.fill_(1))
    del flush_buf

    # Phase timings on the same stream: the band FHT (one kernel) and the DP.
    tables = torch.empty(fhtp.table_shape(h, w, k), dtype=torch.int32, device=dev)
    fws_n = fhtp.fht_workspace_bytes(dt, h, w, k)
    fws = torch.empty(max(fws_n, 1), dtype=torch.uint8, device=dev)
    dws = torch.empty(fhtp.dp_workspace_bytes(h, w, k, bend), dtype=torch.uint8, device=dev)
    ms_fht = time_events(lambda: fhtp.fht_bands(img, k, tables=tables, ws=fws if fws_n else None,
                                                stream=stream), args.steps, stream)
    ms_dp = time_events(lambda: fhtp.polyline_dp(tables, h, w, k, bend=B, ws=dws, score=score,
                                                 xs=xs, stream=stream), args.steps, stream)

    model = byte_model(h, w, k, bpp)
    fht_gbps = model["fht_kernel"] / (ms_fht * 1e-3) / 1e9
    # Algorithmic bytes of the DP phase (columns < w, 4 bytes a value cell,
    # 1 or 2 bytes a back-pointer).  A single image with a fixed window of at
    # most 16 shifts on a grid that leaves the chip latency-bound (fewer than
    # 2^17 threads at 16 displacements each) takes bands k-2..1 two per launch
    # (reads V_{i+2}, H_{i+1}, H_i; writes V_i, A_{i+2}, A_{i+1}), one single
    # step first when their count is odd (reads H_i, V_{i+1}; writes V_i,
    # A_{i+1}); the last step reads H_0 and V_1 and writes keys.  The phase
    # time includes the backtrace walk, so the figure is a lower bound.
    D = 2 * (h // k) - 1
    ab = 1 if D <= 256 else 2
    cells = D * w
    paired = B <= 16 and k >= 4 and w * ((D + 15) // 16) < 1 << 17
    bands = max(k - 2, 0)
    pairs, singles = (bands // 2, bands % 2) if paired else (0, bands)
    dp_bytes = cells * (pairs * (16 + 2 * ab) + singles * (12 + ab) + (8 if k >= 2 else 4))
    launches = pairs + singles + 1
    dp_gbps = dp_bytes / (ms_dp * 1e-3) / 1e9
    dp_roofline = {"bound": "hbm",
                   "kernel": f"dp_pair_fixed x{pairs} + dp_step_fixed x{singles + 1} + walk",
                   "achieved": round(dp_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                   "frac": round(dp_gbps / HBM_PEAK_GBPS, 4), "traffic": None,
                   "algorithmic_bytes": dp_bytes, "launches": launches,
                   "us_per_launch_incl_walk": round(ms_dp * 1e3 / launches, 3)}
    line = {
        "metric": "FHT+DP Mpix/s & HBM GB/s @4096\u00b2,k=32; batched imgs/s vs plain; p99 ms",
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
        "model_bytes": model,
        "launch": launch,
        "eager_ms_per_step": round(ms_eager, 4),
        "graph_ms_per_step": round(ms_graph, 4),
        "phase_ms": {"fht_bands": round(ms_fht, 4), "polyline_dp": round(ms_dp, 4)},
        "single_detection_ms": {"warm": single_warm, "cold": single_cold},
        "roofline": {"bound": "hbm", "kernel": "fht_reg_kernel",
                     "achieved": round(fht_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(fht_gbps / HBM_PEAK_GBPS, 4),
                     "traffic": fht_traffic() if (h, w, k, bpp) == (4096, 4096, 32, 2) else None,
                     "algorithmic_bytes": model["fht_kernel"]},
        "roofline_dp_phase": dp_roofline,
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
        pin = (pj, int(xs.cpu()[pj]))
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
    if args.batch_images > 0:
        line["mixed_batch"] = mixed_batch(args.batch_images, max(3, args.steps // 10), dev, stream)
    if args.serve_requests > 0:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
        line["serving"] = serving(dev, rates, args.serve_requests)
        k1000 = line["serving"].get("1000_per_s")
        if k1000:
            line["p99_ms"] = k1000["server"]["p99_ms"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s.image, k, B, args.cpu_seconds)
    res = (int(score.cpu()[0]), xs.cpu().numpy().tolist())
    line["result"] = {"score": res[0], "x0": res[1][0], "xk": res[1][-1]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
