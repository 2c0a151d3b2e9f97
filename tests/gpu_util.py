"""Helpers shared by the GPU parity tests (not a test module)."""

import sys

import numpy as np
import pytest


def cuda_device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*msg):
    """Name the case before a GPU step, flushed, so a failed run shows it."""
    print("[gpu-case]", *msg, flush=True)
    sys.stdout.flush()


def to_complex(t) -> np.ndarray:
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def to_pairs(c: np.ndarray) -> np.ndarray:
    """complex [..., C] -> float32 [..., C, 2] (rounded to FP32)."""
    return np.stack([c.real, c.imag], axis=-1).astype(np.float32)


def as_fp32_complex(c: np.ndarray) -> np.ndarray:
    """The FP32-rounded version of complex coefficients, back in FP64."""
    p = to_pairs(c).astype(np.float64)
    return p[..., 0] + 1j * p[..., 1]


def normwise(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-row ||got - ref|| / ||ref||."""
    return np.linalg.norm(got - ref, axis=-1) / np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
