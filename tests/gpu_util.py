"""Helpers for GPU tests: skip cleanly without a GPU, fail loudly if the
library is missing on a GPU machine."""
import os

import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_02419_amd import _bbe
    if not os.path.exists(_bbe.LIB_PATH):
        raise RuntimeError("libbbe.so is not built; the GPU tests need the HIP library")
    _bbe.lib()
    return torch


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
