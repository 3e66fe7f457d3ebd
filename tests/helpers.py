"""Shared helpers of the GPU parity tests: device upload and pyramid-level extraction."""
import sys

import numpy as np
import torch


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def level_of(pyr: torch.Tensor, layout, l: int) -> np.ndarray:
    """Level l >= 1 of a device pyramid buffer as a host array."""
    off, p, w, h = layout.offset[l], layout.pitch[l], layout.width[l], layout.height[l]
    return pyr[off:off + p * h].view(h, p)[:, :w].cpu().numpy()


def say(*a):
    """Names the case on stdout before GPU work starts (flushed)."""
    print(*a, flush=True)
    sys.stdout.flush()
