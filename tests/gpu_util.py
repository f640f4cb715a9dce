"""Helpers shared by the GPU tests (no method arithmetic)."""
import numpy as np
import pytest
import torch

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_np(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """max |a - b| / max |b| per (rhs, mode), eq. results:error."""
    num = np.abs(a - b).max(axis=-1)
    den = np.abs(b).max(axis=-1)
    return num / np.where(den > 0, den, 1.0)
