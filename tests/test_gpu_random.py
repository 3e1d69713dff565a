"""Seeded random sweep: small detections of every shape class against the oracle.

Band heights 1 .. 256 (one and two FHT passes), band counts 1 .. 12 (single
steps, pairs of steps with odd and even counts), widths from 1 column to
several FHT tiles and DP column tiles, both pixel types (some saturated), the
fixed window from 0 to 20 shifts and the angle form; then batches of one window
class with mixed sizes and band counts.  Every result must equal the oracle's.
"""

import numpy as np
import pytest
import torch

from tests.gpu_util import announce, host, require_gpu, to_device

pytestmark = pytest.mark.gpu


def _cases(count, seed):
    rng = np.random.default_rng([191201884, 4242, seed])
    out = []
    for _ in range(count):
        n = 1 << int(rng.integers(0, 9))
        k = int(rng.integers(1, 13))
        w = int(rng.integers(1, 700))
        dt = np.uint8 if rng.random() < 0.6 else np.uint16
        top = 255 if dt == np.uint8 else 65535
        img = rng.integers(0, top + 1, size=(n * k, w)).astype(dt)
        if rng.random() < 0.15:
            img[:] = top
        if rng.random() < 0.2:
            kw = dict(gamma=float(rng.uniform(0.01, 1.6)))
        else:
            kw = dict(bend=int(rng.integers(0, 21)))
        out.append((img, k, kw))
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_random_single_detections(orc, seed, path):
    dev = require_gpu()
    for q, (img, k, kw) in enumerate(_cases(100, seed)):
        want_s, want_x = orc.detect_polyline(img, k, **kw)
        announce(f"random {seed}/{q} ({path}): {img.shape} {img.dtype} k={k} {kw}")
        from paper_1912_01884_amd import fhtp
        sc, xs = fhtp.detect_polyline(to_device(img, dev), k, **kw)
        assert int(host(sc)[0]) == want_s, (q, img.shape, k, kw)
        assert host(xs).tolist() == want_x.tolist(), (q, img.shape, k, kw)


def test_random_batches(orc, path):
    from paper_1912_01884_amd import fhtp
    dev = require_gpu()
    rng = np.random.default_rng([191201884, 4243])
    for b in range(8):
        bend = int(rng.integers(0, 17))
        jobs = []
        for _ in range(int(rng.integers(2, 12))):
            n = 1 << int(rng.integers(0, 8))
            k = int(rng.integers(1, 10))
            w = int(rng.integers(1, 300))
            jobs.append((rng.integers(0, 256, size=(n * k, w)).astype(np.uint8), k))
        announce(f"random batch {b}: {len(jobs)} images, bend {bend}, k = {[k for _, k in jobs]}")
        out = fhtp.detect_batch([to_device(a, dev) for a, _ in jobs], [k for _, k in jobs],
                                bends=[bend] * len(jobs))
        torch.cuda.synchronize()
        for q, (a, k) in enumerate(jobs):
            want_s, want_x = orc.detect_polyline(a, k, bend=bend)
            assert int(host(out[q][0])[0]) == want_s, (b, q, a.shape, k)
            assert host(out[q][1]).tolist() == want_x.tolist(), (b, q, a.shape, k)
