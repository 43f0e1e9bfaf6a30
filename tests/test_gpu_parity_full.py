"""Full-size parity of the CUR path against the FP64 oracle, on the same Omega
(Algorithm 3 with the randomized front end of Algorithm 4 and the power scheme
of Section 5.3), plus invariances of the device path.

* The FP32 randomized workload (20000 x 10000, sigma_j = (j+1)^-2, k = 200,
  p = 10, q = 1): skeleton columns J and rows I identical wherever the oracle's
  pivot gap is clear of FP32 noise (1e-4); T against the FP64 least-squares
  interpolation matrix of the device's own skeleton (T is unique given J,
  Section 4.1) within a bound from cond(S11); C and R bitwise; CUR error within
  1.05x of the oracle's.
* Bitwise determinism of the CUR path (two calls, same inputs).
* Norm-downdate cancellation (the recompute of Section 2.2's norms): an input
  whose trailing columns lie within 1e-9 (FP64) / 3e-3 (FP32) of the span of
  the first pivots, so every downdate cancels; J must equal the exact-norm
  oracle's with downdating, with exact norms and with every slab kernel.
"""
import contextlib
import os

import numpy as np
import pytest

import synth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, check_perm  # noqa: E402

U32 = 2.0**-24


@contextlib.contextmanager
def kernel(which):
    old = os.environ.get("IDCUR_CPQR_SLAB")
    if which is None:
        os.environ.pop("IDCUR_CPQR_SLAB", None)
    else:
        os.environ["IDCUR_CPQR_SLAB"] = which
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("IDCUR_CPQR_SLAB", None)
        else:
            os.environ["IDCUR_CPQR_SLAB"] = old


@pytest.fixture(scope="module")
def c2():
    cfg = synth.CONFIGS["rand_fp32_20000x10000_k200"]
    say(f"generating A {cfg.m}x{cfg.n} (FP32 randomized workload)")
    A = synth.lowrank_torch(cfg.m, cfg.n, cfg.spectrum(), seed=4242, device=torch.device("cuda", 0))
    A = A.to(torch.float32).contiguous()
    om = P.gaussian(cfg.k + cfg.p, cfg.m, seed=4243, dtype=torch.float32)
    torch.cuda.synchronize()
    A64 = A.cpu().numpy().astype(np.float64)
    om64 = om.cpu().numpy().astype(np.float64)
    say("oracle CUR (FP64) on the same Omega")
    ref = oracle.cur(A64, cfg.k, omega=om64, q=cfg.q)
    Y64 = oracle.sketch(A64, om64, cfg.q)
    return cfg, A, om, A64, ref, Y64


def test_c2_full_cur_against_oracle(c2):
    cfg, A, om, A64, ref, Y64 = c2
    k = cfg.k
    got = P.cur(A, k, p=cfg.p, q=cfg.q, omega=om)
    assert got.k == k and got.k_row == k
    J, I = got.J.cpu().numpy(), got.I.cpu().numpy()
    check_perm(J, cfg.n)
    check_perm(I, cfg.m)
    cj = clear_prefix(ref.ts.col.qr.gaps, 1e-4)
    nj = k if np.array_equal(J[:k], ref.ts.col.J[:k]) else int(np.argmax(J[:k] != ref.ts.col.J[:k]))
    say(f"  J: clear prefix {cj}, identical prefix {nj} of {k}")
    assert cj >= 20
    assert np.array_equal(J[:cj], ref.ts.col.J[:cj])
    # C and R are bitwise copies of A's columns and rows
    Cg, Ug, Rg = (x.cpu().numpy().astype(np.float64) for x in (got.C, got.U, got.R))
    assert np.array_equal(Cg, A64[:, J[:k]])
    assert np.array_equal(Rg, A64[I[:k]])
    # T against the FP64 interpolation matrix of the device's skeleton on the
    # oracle's sketch: S11 T = S12 with S = Q^T Y P, i.e. T = Y(:,J1)^+ Y(:,J2)
    Y1, Y2 = Y64[:, J[:k]], Y64[:, J[k:]]
    T_ref = np.linalg.lstsq(Y1, Y2, rcond=None)[0]
    # the device T of the column ID (id_col on the same inputs gives the same J)
    cid = P.id_col(A, k, p=cfg.p, q=cfg.q, omega=om)
    assert np.array_equal(cid.J.cpu().numpy(), J)
    Tg = cid.T.cpu().numpy().astype(np.float64)
    s = np.linalg.svd(Y1, compute_uv=False)
    cond = s[0] / s[-1]
    dT = np.linalg.norm(Tg - T_ref) / np.linalg.norm(T_ref)
    bound = max(1e-3, 50.0 * cond * U32)
    say(f"  |dT|_F/|T|_F = {dT:.3e}, cond(S11) = {cond:.3e}, bound {bound:.3e}")
    assert dT <= bound
    # the row ID of C: where J agrees with the oracle's, C is the same matrix
    if nj == k:
        ci = clear_prefix(ref.ts.row.qr.gaps, 1e-4)
        say(f"  I: clear prefix {ci}")
        assert ci >= 10
        assert np.array_equal(I[:ci], ref.ts.row.J[:ci])
    e_g = oracle.e_cur(A64, Cg, Ug, Rg)
    e_o = oracle.e_cur(A64, ref.C, ref.U, ref.R)
    say(f"  e_CUR device {e_g:.5e} oracle {e_o:.5e} ratio {e_g / e_o:.4f}")
    assert e_g <= 1.05 * e_o
    assert e_o >= cfg.frobenius_floor()


def test_cur_bitwise_deterministic(c2):
    cfg, A, om, *_ = c2
    k = cfg.k
    a = P.cur(A, k, p=cfg.p, q=cfg.q, seed=99)
    b = P.cur(A, k, p=cfg.p, q=cfg.q, seed=99)
    for name in ("J", "I", "C", "U", "R"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name


def _cancel_case(m, n, nb, eps_lo, eps_hi, seed):
    """Columns 0..nb-1 span B (orthonormal, distinct scales); every other column
    is a combination of B plus a tiny component eps_c z_c outside it, with eps_c
    log-spaced and distinct, so that after nb steps every downdated norm has
    cancelled to rounding noise and only a recompute finds the next pivots."""
    rng = synth.rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    B, Z = Q[:, :nb], Q[:, nb:]
    A = np.empty((m, n))
    A[:, :nb] = B * (2.0 ** np.arange(nb, 0, -1))
    coef = rng.standard_normal((nb, n - nb))
    eps = np.exp(rng.permutation(np.linspace(np.log(eps_lo), np.log(eps_hi), n - nb)))
    zc = Z @ rng.standard_normal((m - nb, n - nb))
    zc /= np.linalg.norm(zc, axis=0)
    A[:, nb:] = B @ coef + zc * eps
    return A


@pytest.mark.parametrize("which", [None, "1", "2", "3"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_downdate_cancellation_recomputes(which, dtype):
    m, n, nb, k = 240, 65, 5, 25
    # FP32: residuals 3e-3..3e-2 of unit-size columns, so the update's own
    # rounding (~1e-7) stays far below the pivot gaps while the downdate's
    # (~2e-7 on squared norms of 1e-5..1e-3) does not
    lo, hi = (1e-9, 1e-8) if dtype == torch.float64 else (3e-3, 3e-2)
    A = _cancel_case(m, n, nb, lo, hi, seed=8)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A_in = A.astype(npdt)
    ref = oracle.id_col(A_in.astype(np.float64), k)
    c = clear_prefix(ref.qr.gaps, 1e-9 if dtype == torch.float64 else 2e-3)
    say(f"downdate cancellation {dtype} kernel={which}: oracle clear prefix {c} of {k}")
    assert c >= 15
    with kernel(which):
        dd = P.id_col(to_dev(A_in, dtype), k, norms="downdate")
        ex = P.id_col(to_dev(A_in, dtype), k, norms="exact")
    Jd, Je = dd.J.cpu().numpy(), ex.J.cpu().numpy()
    assert np.array_equal(Jd[:c], ref.J[:c])
    assert np.array_equal(Je[:c], ref.J[:c])
