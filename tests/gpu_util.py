"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import sys

import numpy as np
import torch

from oracle import basis as OB
from oracle import model as OM


def say(*a):
    """Names the case before each GPU step, flushed, so a failing run shows where it was."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def to_dev(x: np.ndarray, dtype=torch.complex128) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def neel_row(L: int) -> int:
    st = OB.sector_states(L, L // 2)
    return int(OB.lookup(st, [OM.neel_state(L)])[0])


def max_rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
