"""GPU parity at ranks and sketch widths above 256, where every k x k (and l x l)
Cholesky factor and triangular inverse runs in the blocked form (diagonal blocks
on the one-workgroup kernel, the rest as FP64 matrix-core products), against the
FP64 oracle: orders just above 256 (two blocks) up to 520 (three). FP64 data, so
pivots, T and U are compared tightly."""
import numpy as np
import pytest

import synth
import oracle
from oracle import adjoint

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, rel_err_id, check_perm  # noqa: E402


def _case(m, n, seed, decay):
    return synth.lowrank(m, n, synth.sigma_exp(min(m, n), decay), seed=seed)


@pytest.mark.parametrize("m,n,k", [(700, 600, 300), (900, 1100, 520), (700, 600, 280), (650, 700, 288)])
def test_id_col_det_fp64_large_k(m, n, k):
    say(f"id_col det fp64 {m}x{n} k={k}")
    A = _case(m, n, seed=k, decay=0.4 * k)
    ref = oracle.id_col(A, k)
    got = P.id_col(to_dev(A, torch.float64), k)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    assert got.k == k
    c = clear_prefix(ref.qr.gaps, 1e-10)
    say(f"  clear pivots {c} of {k}")
    assert c >= k // 2
    assert np.array_equal(J[:c], ref.J[:c])
    e_g, e_o = rel_err_id(A, J, got.T.cpu().numpy()), rel_err_id(A, ref.J, ref.T)
    say(f"  e_ID device {e_g:.6e} oracle {e_o:.6e}")
    if c == k:
        assert np.abs(got.T.cpu().numpy() - ref.T).max() <= 1e-8 * max(1.0, np.abs(ref.T).max())
        assert abs(e_g / e_o - 1) <= 1e-9
    else:
        assert e_g <= (1 + 1e-6) * e_o


@pytest.mark.parametrize("k,p", [(300, 20), (260, 20), (250, 38)])
def test_sketch_wide_orth_q1_fp64(k, p):
    # l = k + p: Gram matrices of order 320, 280 and 288
    m, n, q = 1500, 1000, 1
    say(f"id_col sketch fp64 {m}x{n} k={k} p={p} q={q}")
    A = _case(m, n, seed=7, decay=120.0)
    om = synth.gaussian(k + p, m, seed=8)
    ref = oracle.id_col(A, k, omega=om, q=q)
    got = P.id_col(to_dev(A, torch.float64), k, p=p, q=q, omega=to_dev(om, torch.float64))
    J = got.J.cpu().numpy()
    c = clear_prefix(ref.qr.gaps, 1e-9)
    say(f"  clear pivots {c} of {k}")
    assert c >= 50
    assert np.array_equal(J[:c], ref.J[:c])
    e_g, e_o = rel_err_id(A, J, got.T.cpu().numpy()), rel_err_id(A, ref.J, ref.T)
    say(f"  e_ID device {e_g:.6e} oracle {e_o:.6e}")
    assert e_g <= (1 + 1e-6) * e_o


@pytest.mark.parametrize("k", [300, 288, 270])
def test_cur_fp64_k300(k):
    m, n = 800, 650
    say(f"cur det fp64 {m}x{n} k={k}")
    A = _case(m, n, seed=12, decay=120.0)
    ref = oracle.cur(A, k)
    cu = P.cur(to_dev(A, torch.float64), k)
    assert cu.k == k and cu.k_row == k
    Cg, Ug, Rg = (x.cpu().numpy() for x in (cu.C, cu.U, cu.R))
    J, I = cu.J.cpu().numpy(), cu.I.cpu().numpy()
    assert np.array_equal(Cg, A[:, J[:k]])
    assert np.array_equal(Rg, A[I[:k]])
    e_g = oracle.e_cur(A, Cg, Ug, Rg)
    e_o = oracle.e_cur(A, ref.C, ref.U, ref.R)
    say(f"  e_CUR device {e_g:.6e} oracle {e_o:.6e}")
    cj = clear_prefix(ref.ts.col.qr.gaps, 1e-10)
    same = cj == k and np.array_equal(J[:k], ref.ts.col.J[:k]) and np.array_equal(I[:k], ref.ts.row.J[:k])
    say(f"  clear column pivots {cj}, identical index sets: {same}")
    if same:
        assert abs(e_g / e_o - 1) <= 1e-7
        assert np.abs(Ug - ref.U).max() <= 1e-6 * np.abs(ref.U).max()
    else:
        assert e_g <= 1.05 * e_o


def test_rank_deficient_above_256():
    # exact rank 280 with k = 300: the k x k inverses run on a device order of 280
    # inside 300 x 300 buffers (identity padding in the blocked form)
    m, n, r = 600, 500, 280
    say(f"rank deficiency r={r}, k=300")
    A = synth.lowrank(m, n, synth.sigma_pow(r, 0.5), seed=5, rank=r)
    got = P.id_col(to_dev(A, torch.float64), 300)
    assert got.k == r
    assert rel_err_id(A, got.J.cpu().numpy(), got.T.cpu().numpy()) <= 1e-11
    cu = P.cur(to_dev(A, torch.float64), 300)
    assert cu.k == r
    e_c = oracle.e_cur(A, cu.C.cpu().numpy(), cu.U.cpu().numpy(), cu.R.cpu().numpy())
    assert e_c <= 1e-10


def test_backward_k300_fp64():
    m, n, k, p = 700, 500, 300, 10
    say(f"adjoint fp64 {m}x{n} k={k}")
    A = _case(m, n, seed=3, decay=120.0) + 1e-3 * synth.rng(4).standard_normal((m, n))
    dA = to_dev(A, torch.float64)
    om = P.gaussian(k + p, m, seed=5, dtype=torch.float64)
    r = P.id_col(dA, k, p=p, q=0, omega=om)
    J = r.J.cpu().numpy().astype(np.int64)
    g = P.id_col_backward(dA, r.J, r.T, k, omega=om).cpu().numpy()
    want = adjoint.recon_grad(A, J, k, om.cpu().numpy())
    e = float(np.linalg.norm(g - want) / np.linalg.norm(want))
    say(f"  |dA - oracle| / |oracle| = {e:.3e}")
    assert e <= 1e-8
