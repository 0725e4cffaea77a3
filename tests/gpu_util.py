"""Helpers shared by the GPU tests (device transfer, case banners)."""

import sys

import numpy as np


def banner(msg):
    """Name the case on stdout before GPU work, so a failing run is attributable."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, ld=None):
    """FP32 device copy of a square matrix, optionally inside a wider buffer
    (leading dimension ``ld``); returns the n x n view."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.float32)
    n = a.shape[0]
    if ld is None or ld == n:
        return torch.from_numpy(a).to("cuda")
    buf = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :n] = torch.from_numpy(a).to("cuda")
    return buf[:, :n]


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)
