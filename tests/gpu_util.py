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


def elem_rel_err(got, want, floor):
    """Element-wise error: max over elements of
    |got - want| / (|want| + floor * rms(want's column)), and the (row,
    column) where it is largest.  The column-norm error of col_rel_err can
    hide a few wrong rows of a large block; this bound cannot."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if want.ndim == 1:
        got, want = got[:, None], want[:, None]
    rms = np.sqrt(np.mean(want * want, axis=0))
    den = np.abs(want) + floor * np.where(rms > 0, rms, 1.0)[None, :]
    r = np.abs(got - want) / den
    i, j = np.unravel_index(int(np.argmax(r)), r.shape)
    return float(r[i, j]), (int(i), int(j))


# Element-wise bounds by storage precision, (floor, bound): an entry may be
# off by bound * (|want| + floor * rms of its column), i.e. by `bound`
# relative where it is large and by bound * floor * rms where it is near 0
# (rounding of the block leaves an absolute error of the order of the
# column's scale there).  Measured worst cases over the parity tests: FP64
# 2e-11, FP32 1.5e-4, BF16 about 0.03 of the rms near 0.
ELEM = {"f64": (1e-6, 1e-9), "f32": (1e-3, 1e-3), "bf16": (0.5, 0.05)}


def check_elems(got, want, dtype, what=""):
    """Asserts the element-wise bound of ELEM[dtype] and prints the worst
    entry."""
    floor, bound = ELEM[dtype]
    err, (i, j) = elem_rel_err(got, want, floor)
    say(f"  {what} element-wise err {err:.2e} at row {i} col {j} (bound {bound:.0e})")
    assert err <= bound, (err, i, j)
    return err


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
