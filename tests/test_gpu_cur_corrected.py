"""GPU parity of the CUR with the error-corrected U (U R = V* + C^+ E, Section 4.3,
eq. (cur_ur_sys2)) against the FP64 oracle: same C and R (pivots identical on
clear gaps), U within tolerance (FP64) and the CUR error within 1.05x of the
oracle's (FP32), and never above the plain U's error."""
import numpy as np
import pytest

import synth
import oracle
import oracle.decomp as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev  # noqa: E402


def _e(A, C, U, R):
    return oracle.e_cur(A, C.astype(np.float64), U.astype(np.float64), R.astype(np.float64))


def test_corrected_u_fp64_matches_oracle():
    m, n, k = 600, 400, 25
    say(f"cur corrected fp64 {m}x{n} k={k}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 6.0), seed=77)
    ref = D.cur(A, k, u_correct=True)
    got = P.cur(to_dev(A, torch.float64), k, u_correct=True)
    assert np.array_equal(got.J.cpu().numpy()[:k], ref.ts.col.J[:k])
    assert np.array_equal(got.I.cpu().numpy()[:k], ref.ts.row.J[:k])
    U = got.U.cpu().numpy()
    assert np.abs(U - ref.U).max() <= 1e-7 * np.abs(ref.U).max()
    e_g, e_o = _e(A, got.C.cpu().numpy(), U, got.R.cpu().numpy()), oracle.e_cur(A, ref.C, ref.U, ref.R)
    assert abs(e_g / e_o - 1) <= 1e-8


def test_corrected_u_fp32_sketched_error():
    m, n, k, p = 4000, 2000, 60, 10
    say(f"cur corrected fp32 {m}x{n} k={k} p={p} q=1")
    A = synth.lowrank(m, n, synth.sigma_pow(min(m, n), 2.0), seed=5).astype(np.float32)
    A64 = A.astype(np.float64)
    om = P.gaussian(k + p, m, seed=9, dtype=torch.float32)
    ref = D.cur(A64, k, omega=om.double().cpu().numpy(), q=1, u_correct=True)
    got = P.cur(to_dev(A, torch.float32), k, p=p, q=1, omega=om, u_correct=True)
    plain = P.cur(to_dev(A, torch.float32), k, p=p, q=1, omega=om)
    e_g = _e(A64, got.C.cpu().numpy(), got.U.cpu().numpy(), got.R.cpu().numpy())
    e_p = _e(A64, plain.C.cpu().numpy(), plain.U.cpu().numpy(), plain.R.cpu().numpy())
    e_o = oracle.e_cur(A64, ref.C, ref.U, ref.R)
    say(f"  e_cur corrected gpu {e_g:.4e} oracle {e_o:.4e}; plain gpu {e_p:.4e}")
    assert e_g <= 1.05 * e_o
    assert e_g <= e_p * (1 + 1e-6)
