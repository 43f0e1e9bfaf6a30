"""GPU parity of the FP32 sketch Y = Omega A (Section 5.1), q = 0, against the
FP64 product, entry by entry: every entry must lie within (K + 2) u32
(|Omega| |A|) of it (K terms summed in FP32 by the matrix cores, the split-K
partial sums added in FP64, one final FP32 rounding; u32 = 2^-24).

The shapes cover both operand layouts of the thin-output kernel (column sketch:
A read along its rows, M = n; row sketch: A read along K), column counts l that
select 8, 14 and 16 column tiles, a ragged last 64-row stripe, K not a multiple
of the 16-deep stage, a long K split over many workgroups, and shapes whose
extents are not multiples of 4 (served by the general kernel).
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev  # noqa: E402

U32 = 2.0**-24


@pytest.mark.parametrize("row", [False, True])
@pytest.mark.parametrize("m,n,l", [(1004, 700, 30), (2000, 1500, 210), (900, 1204, 250), (1003, 701, 30),
                                   (20000, 1024, 210)])
def test_fp32_sketch_within_summation_bound(row, m, n, l):
    p = 5
    k = l - p
    rows = n if row else m
    say(f"fp32 sketch row={row} {m}x{n} l={l}")
    A = synth.gaussian(m, n, seed=m + 7 * n + l).astype(np.float32)
    om = synth.gaussian(l, rows, seed=l + 3).astype(np.float32)
    Yt = P.sketch(to_dev(A, torch.float32), k, p=p, q=0, omega=to_dev(om, torch.float32), row=row)
    got = Yt.cpu().numpy().T.astype(np.float64)
    B = (A.T if row else A).astype(np.float64)
    om64 = om.astype(np.float64)
    want = om64 @ B
    K = B.shape[0]
    bound = (K + 2) * U32 * (np.abs(om64) @ np.abs(B))
    err = np.abs(got - want)
    say(f"  worst |err|/bound = {float(np.max(err / bound)):.3f}")
    assert np.all(err <= bound)
