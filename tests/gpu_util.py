"""Helpers for the GPU tests: numpy <-> device tensors, bit for bit."""
import numpy as np
import torch


def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def to_dev(x):
    x = np.ascontiguousarray(x)
    if x.dtype == np.uint32:
        x = x.view(np.int32)
    elif x.dtype == np.uint64:
        x = x.view(np.int64)
    return torch.from_numpy(x).to(dev())


def to_host(t, unsigned_dtype):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(unsigned_dtype)


def mismatch_report(got, want, limit=5):
    bad = np.argwhere(got != want)
    lines = [f"{len(bad)} of {got.size} differ"]
    for idx in bad[:limit]:
        idx = tuple(int(i) for i in idx)
        lines.append(f"  at {idx}: got {int(got[idx])} want {int(want[idx])}")
    return "\n".join(lines)
