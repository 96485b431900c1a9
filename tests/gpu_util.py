"""Helpers shared by the GPU tests (host <-> device copies, step logging)."""
import sys

import numpy as np
import torch


def log(msg: str):
    """Name the case before a GPU step, flushed, so a crash report says what ran."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def to_dev(a: np.ndarray, dtype=np.uint8, pitch: int = 0) -> torch.Tensor:
    """Copy an integer image to the GPU; with pitch > width, as a view into wider rows."""
    a = np.ascontiguousarray(a.astype(dtype))
    t = torch.from_numpy(a)
    if pitch and pitch > a.shape[1]:
        big = torch.zeros((a.shape[0], pitch), dtype=t.dtype, device="cuda")
        big[:, :a.shape[1]].copy_(t.cuda())
        return big[:, :a.shape[1]]
    return t.cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_available() -> bool:
    return torch.cuda.is_available()
