"""GPU tests of the tuning rules: every candidate launch shape gives the oracle's answer.

The tuner picks among launch shapes that must not change any result.  Each
candidate (the DP knobs for fixed windows, times both FHT grids) is applied
to every request of a mixed batch (8- and 16-bit pixels, band heights 8 to
512, k from 2 to 12, fixed and scanned windows, widths crossing tiles and
stripes), and every score and vertex list must equal the CPU oracle's.  Then
the tuner itself runs on a slice of the mixed-size workload.
"""

import dataclasses
import math

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


def _jobs():
    rng = np.random.default_rng([191201884, 131, 0])
    shapes = [(64, 300, 8, np.uint8, 3), (512, 700, 4, np.uint8, 4), (256, 1500, 2, np.uint16, 8),
              (1024, 400, 8, np.uint8, 1), (96, 129, 12, np.uint8, 2), (2048, 300, 4, np.uint8, 5),
              (384, 2100, 3, np.uint16, 16), (256, 260, 4, np.uint8, 25),
              (512, 333, 8, np.uint16, None)]
    jobs = []
    for h, w, k, dt, b in shapes:
        top = 255 if dt == np.uint8 else 4000
        img = rng.integers(0, top + 1, size=(h, w)).astype(dt)
        jobs.append((img, k, b, None if b is not None else 0.4))
    return jobs


@pytest.fixture(scope="module")
def case(orc):
    dev = require_gpu()
    jobs = _jobs()
    want = [orc.detect_polyline(img, k, bend=b, gamma=g) for img, k, b, g in jobs]
    return dev, jobs, want


def _cands():
    from paper_1912_01884_amd import autotune
    return [(dp, fg) for dp in autotune.DP_CANDIDATES for fg in autotune.FHT_CANDIDATES]


@pytest.mark.parametrize("dp,fg", _cands(),
                         ids=[f"dc{d['dc']}t{d['steps']}s{d['stripe']}g{g}" for d, g in _cands()])
def test_every_candidate_matches_the_oracle(case, dp, fg):
    from paper_1912_01884_amd import autotune, fhtp
    dev, jobs, want = case
    imgs = [to_device(img, dev) for img, _, _, _ in jobs]
    fhtp.tune_set([autotune.rule(window=0, fht_grid=fg, **dp), autotune.rule(window=1, fht_grid=fg)])
    try:
        announce(f"tuning candidate {dp} fht_grid={fg}: batch of {len(jobs)}, then singles")
        out = fhtp.detect_batch(imgs, [j[1] for j in jobs], bends=[j[2] for j in jobs],
                                gammas=[j[3] for j in jobs])
        single = [fhtp.detect_polyline(im, k, bend=b, gamma=g)
                  for im, (_, k, b, g) in zip(imgs, jobs)]
        torch.cuda.synchronize()
    finally:
        fhtp.tune_set([])
    for q, (s, x) in enumerate(want):
        assert int(host(out[q][0])[0]) == s and host(out[q][1]).tolist() == x.tolist(), q
        assert int(host(single[q][0])[0]) == s and host(single[q][1]).tolist() == x.tolist(), q


def test_tuner_on_mixed_workload_slice(tmp_path):
    from paper_1912_01884_amd import autotune, fhtp
    dev = require_gpu()
    batch = synth.make_mixed_batch(24)
    imgs = [to_device(s.image, dev) for s in batch]
    announce("autotune 24 mixed images")
    res = autotune.tune(imgs, [s.k for s in batch], bends=[s.bend for s in batch], reps=2,
                        install_result=False)
    assert fhtp.tune_get() == []  # restored
    assert 0 < res.tuned_ms <= res.default_ms
    if not res.rules:
        # No candidate beat the library's own choices within the timing noise:
        # the tuner then keeps them (no rules).  Persistence and the tuned batch
        # below are checked on rules that change every launch shape instead.
        assert res.tuned_ms == res.default_ms
        res = dataclasses.replace(res, rules=[autotune.rule(steps=1, dc=16, stripe=4, fht_grid=1)])
    assert len(res.timings) == 1 + len(autotune.DP_CANDIDATES) + 2 * len(
        {(0, (s.h // s.k).bit_length() - 1) for s in batch})
    path = str(tmp_path / "plan.json")
    autotune.save(res, path, workload="mixed 24")
    assert autotune.load(path) == res.rules
    try:
        out = fhtp.detect_batch(imgs, [s.k for s in batch], bends=[s.bend for s in batch])
        torch.cuda.synchronize()
        for q, s in enumerate(batch):
            s1, x1 = fhtp.detect_polyline(imgs[q], s.k, bend=s.bend)
            assert np.array_equal(host(out[q][0]), host(s1)) and \
                np.array_equal(host(out[q][1]), host(x1)), q
    finally:
        fhtp.tune_set([])
