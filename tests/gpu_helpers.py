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


U32 = 2.0 ** -24


def check_t_fp32(Y, J, k, T, tag=""):
    """FP32 interpolation matrix against the FP64 least-squares T of the same
    skeleton (Section 4.1, eq. (lsqr_for_T)): S11 T = S12 with S = Q^T Y P is
    T = Y(:, J1)^+ Y(:, J2). The FP32 QR and triangular solve leave a relative
    error of about cond(S11) u32 (times a modest constant), so the bar is
    max(1e-3, 50 cond(S11) u32) in the Frobenius norm."""
    J = np.asarray(J)
    Y = np.asarray(Y, dtype=np.float64)
    Y1, Y2 = Y[:, J[:k]], Y[:, J[k:]]
    T_ref = np.linalg.lstsq(Y1, Y2, rcond=None)[0]
    s = np.linalg.svd(Y1, compute_uv=False)
    cond = s[0] / s[-1]
    dT = np.linalg.norm(np.asarray(T, dtype=np.float64)[:, : Y2.shape[1]] - T_ref) / max(np.linalg.norm(T_ref), 1e-300)
    bound = max(1e-3, 50.0 * cond * U32)
    say(f"  {tag} |dT|_F/|T|_F = {dT:.3e}, cond(S11) = {cond:.3e}, bound {bound:.3e}")
    assert dT <= bound, (tag, dT, bound)
