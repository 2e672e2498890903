"""Argument checks of the Python binding that run before anything reaches
the library (no GPU needed): rings the kernels write through must be
contiguous float64 tensors on the GPU or in pinned host memory, large
enough for the call."""
import os
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1211_0780_amd.sim import Sim  # noqa: E402


@pytest.mark.parametrize("t", [
    torch.zeros(10, dtype=torch.float64),           # pageable host memory
    torch.zeros(10, dtype=torch.float32),           # wrong dtype
    torch.zeros(10, 2, dtype=torch.float64).t(),    # strided view
], ids=["host", "float32", "strided"])
def test_ring_rejected(t):
    with pytest.raises(ValueError, match="float64 tensor on the GPU or in pinned host memory"):
        Sim._check_ring(None, "obs", t, 5)


def test_absent_ring_is_accepted():
    Sim._check_ring(None, "bonds", None, 5)
