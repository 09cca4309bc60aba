"""Helpers shared by the GPU tests: move seeded synthetic graphs to the device
and compare results with the oracle."""
import sys

import numpy as np
import torch


def to_device(g, weights="keep", device="cuda"):
    """Graph -> (indptr int64, indices int32, data or None) on the device.
    weights: "keep" (float64 data as float64), "f32", "bf16", or "none"."""
    ip = torch.from_numpy(np.ascontiguousarray(g.indptr, dtype=np.int64)).to(device)
    ix = torch.from_numpy(np.ascontiguousarray(g.indices, dtype=np.int32)).to(device)
    if g.data is None or weights == "none":
        return ip, ix, None
    d = torch.from_numpy(np.ascontiguousarray(g.data, dtype=np.float64))
    if weights == "f32":
        d = d.to(torch.float32)
    elif weights == "bf16":
        d = d.to(torch.bfloat16)
    return ip, ix, d.to(device)


def host_weights(data):
    """The weights exactly as the device sees them, in float64."""
    if data is None:
        return None
    return data.detach().to("cpu", torch.float64).numpy()


def col_rel_err(got, want):
    """max over columns of ||got - want|| / ||want||."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    num = np.linalg.norm(got - want, axis=0)
    den = np.linalg.norm(want, axis=0)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
