"""Autotuner: launch shapes for a workload, measured on the device.

The library cuts its work into launches and workgroups by rules that never
change a result (fhtp_tune_set, include/fhtp.h): the displacements per thread
of one-step DP launches, how many DP steps (one, two or three) share a
launch, the stripe width of the multi-step kernels' workgroup order, and whether the FHT runs a
resident grid or one workgroup per work item.  ``tune`` times the candidates
on the caller's own images through the batched entry point (the shapes a
workload really launches, packed as they really are), checks that every
candidate returns exactly the results of the library's defaults, and keeps
the fastest:

  1. the DP knobs, one choice for every fixed-window request of the workload
     (a shared choice keeps images of one window class in shared launches);
  2. then the FHT grid, separately for each (pixel type, band height) group
     (FHT launches are grouped that way anyway).

The result is a list of rules, one pair per group plus a catch-all, that can
be installed (``install``), saved as JSON keyed by the device name, its
architecture and the library version (``save``), and loaded again
(``load``, or ``load_from_env`` for the file named by FHTP_PLAN) only on a
device and library that match the key.
"""

from __future__ import annotations

import ctypes as C
import json
import os
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

from . import fhtp

W_ANY = (0, 1 << 20)

# Three and two steps per launch at four stripe widths each, one step per
# launch at 8 and 16 displacements per thread.
DP_CANDIDATES = ([dict(dc=8, steps=g, stripe=s) for g in (3, 2) for s in (4, 8, 16, 32)] +
                 [dict(dc=8, steps=1, stripe=0), dict(dc=16, steps=1, stripe=0)])
FHT_CANDIDATES = (0, 1)


def rule(dtype=-1, log2n=-1, window=-1, dc=0, steps=0, stripe=0, fht_grid=0, small=0,
         w_min=W_ANY[0], w_max=W_ANY[1]) -> dict:
    return dict(dtype=int(dtype), log2n=int(log2n), w_min=int(w_min), w_max=int(w_max),
                window=int(window), dc=int(dc), steps=int(steps), stripe=int(stripe),
                fht_grid=int(fht_grid), small=int(small))


def device_key() -> dict:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return {"device": p.name, "arch": getattr(p, "gcnArchName", ""), "library": fhtp.version()}


@dataclass
class TuneResult:
    rules: List[dict]
    default_ms: float
    tuned_ms: float
    dp_choice: dict
    fht_choice: Dict[str, int]
    timings: Dict[str, float] = field(default_factory=dict)
    seconds: float = 0.0

    def as_dict(self) -> dict:
        return {"rules": self.rules, "default_ms": round(self.default_ms, 4),
                "tuned_ms": round(self.tuned_ms, 4), "dp_choice": self.dp_choice,
                "fht_choice": self.fht_choice,
                "timings_ms": {k: round(v, 4) for k, v in self.timings.items()},
                "seconds": round(self.seconds, 2)}


class Workload:
    """A fixed set of device images run as one fhtp_detect_batch call."""

    def __init__(self, images, ks, bends=None, gammas=None, stream=None):
        import torch
        self.torch = torch
        self.images = list(images)
        self.ks = [int(k) for k in ks]
        self.jobs, self.keep = fhtp.make_jobs(self.images, self.ks, bends, gammas)
        self.arr = (fhtp.Job * len(self.jobs))(*self.jobs)
        self.nbytes = fhtp.batch_workspace_bytes(self.jobs)
        dev = self.images[0].device
        self.ws = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.groups = sorted({(fhtp._dtype_code(im), (im.shape[0] // k).bit_length() - 1)
                              for im, k in zip(self.images, self.ks)})

    def run(self) -> None:
        rc = fhtp.lib().fhtp_detect_batch(self.arr, len(self.jobs), C.c_void_p(self.ws.data_ptr()),
                                          self.nbytes, C.c_void_p(self.stream.cuda_stream))
        fhtp._check(rc, "detect_batch")

    def results(self):
        self.torch.cuda.synchronize()
        return [(int(s.cpu()[0]), x.cpu().tolist()) for s, x in self.keep]

    def time_ms(self, reps: int) -> float:
        torch = self.torch
        self.run()  # warm: caches, lazily built streams
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(self.stream)
        for _ in range(reps):
            self.run()
        b.record(self.stream)
        b.synchronize()
        return a.elapsed_time(b) / reps


def _rules_for(groups, dp: dict, fht: Dict[tuple, int]) -> List[dict]:
    """One rule per (pixel type, band height) group and window kind, then a
    catch-all for fixed windows."""
    out = []
    for g in groups:
        fg = fht.get(g, 0)
        out.append(rule(dtype=g[0], log2n=g[1], window=0, fht_grid=fg, **dp))
        out.append(rule(dtype=g[0], log2n=g[1], window=1, fht_grid=fg))
    out.append(rule(window=0, **dp))
    return out


def tune(images: Sequence, ks: Sequence[int], bends=None, gammas=None, reps: int = 5,
         stream=None, install_result: bool = True) -> TuneResult:
    """Time every candidate on these images (batched) and return the fastest rules.

    Raises if any candidate's results differ from the defaults' (they never
    should: the rules only change launch shapes).  The rules in force before
    the call are restored unless `install_result` (then the tuned ones are).
    """
    t0 = time.perf_counter()
    previous = fhtp.tune_get()
    wl = Workload(images, ks, bends, gammas, stream)
    timings: Dict[str, float] = {}
    try:
        fhtp.tune_set([])
        base_ms = wl.time_ms(reps)
        want = wl.results()
        timings["defaults"] = base_ms

        def trial(name, rules):
            fhtp.tune_set(rules)
            ms = wl.time_ms(reps)
            got = wl.results()
            if got != want:
                raise RuntimeError(f"tuning candidate {name} changed a result")
            timings[name] = ms
            return ms

        best_dp, best_ms = None, float("inf")
        for cand in DP_CANDIDATES:
            name = "dp dc{dc} steps{steps} stripe{stripe}".format(**cand)
            ms = trial(name, _rules_for(wl.groups, cand, {}))
            if ms < best_ms:
                best_dp, best_ms = cand, ms
        fht: Dict[tuple, int] = {}
        for g in wl.groups:
            best_fg, best_g = 0, float("inf")
            for fg in FHT_CANDIDATES:
                ms = trial(f"fht dtype{g[0]} log2n{g[1]} grid{fg}",
                           _rules_for(wl.groups, best_dp, {**fht, g: fg}))
                if ms < best_g:
                    best_fg, best_g = fg, ms
            fht[g] = best_fg
        rules = _rules_for(wl.groups, best_dp, fht)
        fhtp.tune_set(rules)
        tuned_ms = wl.time_ms(reps)
        if wl.results() != want:
            raise RuntimeError("tuned rules changed a result")
        if tuned_ms > base_ms:  # within noise of the defaults: keep the library's choices
            rules, tuned_ms = [], base_ms
    finally:
        fhtp.tune_set(previous)
    res = TuneResult(rules=rules, default_ms=base_ms, tuned_ms=tuned_ms, dp_choice=best_dp,
                     fht_choice={f"dtype{g[0]} log2n{g[1]}": v for g, v in fht.items()},
                     timings=timings, seconds=time.perf_counter() - t0)
    if install_result:
        install(res.rules)
    return res


def install(rules: List[dict]) -> None:
    fhtp.tune_set(rules)


def save(result: TuneResult, path: str, workload: str = "") -> None:
    doc = {"key": device_key(), "workload": workload, **result.as_dict()}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)


def load(path: str, install_rules: bool = True) -> Optional[List[dict]]:
    """The rules saved at `path` if they were tuned on this device and library
    version (installed unless install_rules is False), else None."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("key") != device_key():
        return None
    rules = [rule(**{k: r[k] for k in ("dtype", "log2n", "window", "dc", "steps", "stripe",
                                       "fht_grid", "small", "w_min", "w_max") if k in r})
             for r in doc["rules"]]
    if install_rules:
        install(rules)
    return rules


def load_from_env() -> Optional[List[dict]]:
    """Install the rules of the file named by FHTP_PLAN, when set and matching."""
    path = os.environ.get("FHTP_PLAN")
    if not path or not os.path.exists(path):
        return None
    return load(path)
