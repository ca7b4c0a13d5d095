"""Shared helpers of the GPU tests (no arithmetic of the method here)."""
import functools
import sys

import pytest


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=1)
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_01478_amd.api import Context
    return Context(0)
