"""Device-buffer helpers for the GPU tests (numpy uint64 <-> torch int64)."""
import numpy as np


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return torch


def to_dev(a: np.ndarray):
    torch = require_gpu()
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.copy()).to("cuda")


def to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def empty_words(n: int):
    torch = require_gpu()
    return torch.empty(int(n), dtype=torch.int64, device="cuda")
