"""GPU parity of the subsampled randomized Hadamard sketch (the real counterpart
of Section 5.2's structured sketch) against the FP64 oracle (oracle/srht.py).

The random signs and sampled rows are drawn by ``synth.srht_draws`` and handed to
both sides. The sketch itself is checked entry by entry against the summation
bound of the fast transform: every entry is l^(-1/2) times a signed sum of the
column's entries, formed by 7 butterfly levels per 128-row block, a sum over at
most ``bps`` blocks, the split sums and two roundings, so it lies within
(bps + 10) u |column|_1 / sqrt(l) of the exact value (u of the dtype). IDs on the
sketch must give the oracle's pivots wherever its gap is clear of the
arithmetic's noise and the same error (FP64: to 1e-8 relative; FP32: within 1.05x).
"""
import math

import numpy as np
import pytest

import synth
import oracle
from oracle import srht

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, rel_err_id, check_perm  # noqa: E402


def _draws(M, l, seed):
    rows, signs = synth.srht_draws(M, l, seed)
    return (rows, signs, torch.as_tensor(rows, device="cuda").contiguous(),
            torch.as_tensor(signs, device="cuda").contiguous())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("row", [False, True])
@pytest.mark.parametrize("m,n,l", [(1000, 300, 40), (130, 50, 16), (4096, 257, 100), (20000, 1000, 210),
                                   (777, 2049, 255), (3000, 700, 257), (20000, 600, 400), (1100, 1300, 512)])
def test_structured_sketch_within_summation_bound(dtype, row, m, n, l):
    say(f"srht sketch {dtype} row={row} {m}x{n} l={l}")
    M = n if row else m
    A = synth.gaussian(m, n, seed=m + 3 * n + l)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A = A.astype(npdt)
    rows, signs, rows_d, signs_d = _draws(M, l, seed=l + 17)
    Yt = P.sketch(to_dev(A, dtype), l - 5, p=5, q=0, srht=(rows_d, signs_d), row=row)
    P.sync_status(Yt.device)
    got = Yt.cpu().numpy().T.astype(np.float64)
    B = (A.T if row else A).astype(np.float64)
    want = srht.srht_sketch(B, rows, signs)
    u = 2.0**-24 if dtype == torch.float32 else 2.0**-53
    nblk = math.ceil(M / 128)
    bound = (nblk + 10) * u * np.abs(B).sum(axis=0)[None, :] / math.sqrt(l)
    err = np.abs(got - want)
    say(f"  worst |err|/bound = {float(np.max(err / bound)):.3f}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_id_col_on_structured_sketch_matches_oracle(dtype):
    m, n, k = 3000, 800, 40
    l = 2 * k   # l = 2k, as Section 5.2 suggests for the structured sketch
    say(f"id_col srht {dtype} {m}x{n} k={k} l={l}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 6.0), seed=41)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A_in = A.astype(npdt)
    A64 = A_in.astype(np.float64)
    rows, signs, rows_d, signs_d = _draws(m, l, seed=3)
    ref = oracle.id_col(A64, k, omega=srht.srht_omega(m, rows, signs))
    got = P.id_col(to_dev(A_in, dtype), k, p=l - k, q=0, srht=(rows_d, signs_d))
    J = got.J.cpu().numpy()
    check_perm(J, n)
    c = clear_prefix(ref.qr.gaps, 1e-9 if dtype == torch.float64 else 1e-4)
    assert c >= 5
    assert np.array_equal(J[:c], ref.J[:c])
    e_g, e_o = rel_err_id(A64, J, got.T.cpu().numpy()), rel_err_id(A64, ref.J, ref.T)
    if dtype == torch.float64:
        assert c == k
        assert abs(e_g / e_o - 1) <= 1e-8
    assert e_g <= 1.05 * e_o


def test_cur_on_structured_sketch_matches_oracle_error():
    m, n, k = 4000, 2000, 50
    l = 2 * k
    say(f"cur srht fp32 {m}x{n} k={k} l={l}")
    A = synth.lowrank(m, n, synth.sigma_pow(min(m, n), 2.0), seed=8).astype(np.float32)
    A64 = A.astype(np.float64)
    rows, signs, rows_d, signs_d = _draws(m, l, seed=21)
    ref = oracle.cur(A64, k, omega=srht.srht_omega(m, rows, signs))
    got = P.cur(to_dev(A, torch.float32), k, p=l - k, q=0, srht=(rows_d, signs_d))
    e_o = oracle.e_cur(A64, ref.C, ref.U, ref.R)
    e_g = oracle.e_cur(A64, got.C.cpu().numpy().astype(np.float64), got.U.cpu().numpy().astype(np.float64),
                       got.R.cpu().numpy().astype(np.float64))
    say(f"  e_cur gpu {e_g:.4e} oracle {e_o:.4e}")
    assert e_g <= 1.05 * e_o


def test_structured_sketch_argument_checks():
    m, n, k, l = 300, 200, 10, 20
    A = to_dev(synth.gaussian(m, n, seed=1), torch.float32)
    rows, signs, rows_d, signs_d = _draws(m, l, seed=2)
    with pytest.raises(P.IDCurError):   # no power steps with the structured sketch
        P.id_col(A, k, p=l - k, q=1, srht=(rows_d, signs_d))
    with pytest.raises(P.IDCurError):   # native precision only
        P.id_col(A, k, p=l - k, q=0, srht=(rows_d, signs_d), prec="bf16")
    bad = rows_d.clone()
    bad[3] = 512   # beyond the padded order 512 of 300 rows: clamped and reported
    with pytest.raises(P.IDCurError):
        P.id_col(A, k, p=l - k, q=0, srht=(bad, signs_d))
        P.sync_status(A.device)
