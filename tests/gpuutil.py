"""Helpers for the GPU tests: moving uint64 words between numpy and torch."""
from __future__ import annotations

import numpy as np


def dev():
    import torch

    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).to(dev())


def masks_to_dev(m: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(m, dtype=np.uint16).view(np.int16).copy()).to(dev())


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def say(msg: str) -> None:
    print(msg, flush=True)
