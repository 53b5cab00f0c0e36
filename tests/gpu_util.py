"""Shared helpers of the GPU tests: skip when no GPU or no built library."""
import os

import pytest

from paper_2508_07610_amd import mpdo as M


def gpu_available() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


def require_gpu():
    if not os.path.exists(M.LIB_PATH):
        pytest.fail("libmpdo.so is not built (python -m paper_2508_07610_amd.build)")
    if not gpu_available():
        pytest.skip("no GPU")
