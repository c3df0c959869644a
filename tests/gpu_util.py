"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np
import pytest


def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def to_dev(a, d):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


def to_np(t):
    return t.detach().cpu().numpy()


def say(*a):
    """Names the case before a GPU step, so a fault report says which one."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def assert_equal(got, exp, what):
    got = np.asarray(got)
    exp = np.asarray(exp)
    assert got.shape == exp.shape, (what, got.shape, exp.shape)
    if not np.array_equal(got, exp):
        bad = np.argwhere(got != exp)
        y, x = bad[0][:2]
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at (y={y}, x={x}): got {got[y, x]} "
                             f"expected {exp[y, x]}")
