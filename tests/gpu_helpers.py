"""Shared helpers for the GPU parity tests (loaded only by tests marked gpu)."""
import sys

import numpy as np
import torch

import oracle


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def clear_prefix(gaps, thr):
    """Number of leading pivots whose best-vs-runner-up gap exceeds thr."""
    n = 0
    for g in gaps:
        if g < thr:
            break
        n += 1
    return n


def rel_err_id(A, J, T):
    return oracle.e_id(A, np.asarray(J, dtype=np.int64), np.asarray(T, dtype=np.float64))


def check_perm(J, n):
    J = np.asarray(J)
    assert J.shape == (n,)
    assert np.array_equal(np.sort(J), np.arange(n)), "J is not a permutation"
