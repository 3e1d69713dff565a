"""Helpers for the GPU tests: device placement and case announcements."""

from __future__ import annotations

import contextlib
import sys

import numpy as np


def announce(msg: str) -> None:
    """Name the case on stderr (unbuffered) before it touches the GPU."""
    sys.__stderr__.write(f"[gpu case] {msg}\n")
    sys.__stderr__.flush()


def require_gpu():
    import torch
    from paper_1912_01884_amd import fhtp
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    fhtp.lib()  # raises if libfhtp.so was not built: no silent fallback
    return torch.device("cuda:0")


def to_device(img: np.ndarray, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(img)).to(dev)


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


@contextlib.contextmanager
def general_path():
    """Run with the general kernels only: small images do not take the
    one-workgroup path (a tuning rule; the rules in force are restored)."""
    from paper_1912_01884_amd import autotune, fhtp
    previous = fhtp.tune_get()
    fhtp.tune_set([autotune.rule(small=1)])
    try:
        yield
    finally:
        fhtp.tune_set(previous)
