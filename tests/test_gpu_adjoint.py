"""GPU parity of the column-ID reconstruction-loss gradient (skeleton frozen)
against the FP64 oracle (oracle/adjoint.py), through the C ABI and through the
torch.autograd.Function.

The skeleton J comes from the GPU forward pass and is handed to the oracle, as
is the sketch matrix Omega (generated on the device from its Philox
definition), so both sides differentiate the same function. Tolerances:
FP64 normwise 1e-9; FP32 normwise 2e-4 (FP32 storage of A, T and the m x n
products, FP64 for the k x k factorisation).
"""
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
from gpu_helpers import say, to_dev, check_perm  # noqa: E402


def _case(m, n, seed, noise):
    A = synth.lowrank(m, n, synth.sigma_pow(min(m, n), 1.5), seed=seed)
    A = A + noise * synth.rng(seed + 7).standard_normal((m, n))
    return A


def _relnorm(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 2e-4)])
@pytest.mark.parametrize("sketched", [True, False])
def test_gradient_matches_oracle(dtype, tol, sketched):
    m, n, k, p = 300, 200, 20, 10
    say(f"adjoint {m}x{n} k={k} sketched={sketched} {dtype}")
    A = _case(m, n, seed=31, noise=1e-3)
    dA = to_dev(A, dtype)
    om = P.gaussian(k + p, m, seed=77, dtype=dtype) if sketched else None
    r = P.id_col(dA, k, p=p if sketched else -1, q=0, omega=om)
    assert r.k == k
    J = r.J.cpu().numpy().astype(np.int64)
    check_perm(J, n)
    g = P.id_col_backward(dA, r.J, r.T, k, omega=om).cpu().numpy()
    A64 = dA.double().cpu().numpy()
    om64 = om.double().cpu().numpy() if sketched else None
    want = adjoint.recon_grad(A64, J, k, om64)
    e = _relnorm(g, want)
    say(f"  |dA - oracle| / |oracle| = {e:.3e}")
    assert e <= tol


def test_deterministic_t_path_vanishes():
    # Y = A: at the least-squares T the path through T is zero up to rounding,
    # so the gradient is 2E on J2 and -2 E T^T on J1 (closed form)
    m, n, k = 300, 200, 20
    A = _case(m, n, seed=5, noise=1e-3)
    dA = to_dev(A, torch.float64)
    r = P.id_col(dA, k)
    J = r.J.cpu().numpy().astype(np.int64)
    g = P.id_col_backward(dA, r.J, r.T, k).cpu().numpy()
    C = A[:, J[:k]]
    T = np.linalg.lstsq(C, A[:, J[k:]], rcond=None)[0]
    E = A[:, J[k:]] - C @ T
    ref = np.zeros_like(A)
    ref[:, J[k:]] = 2 * E
    ref[:, J[:k]] = -2 * E @ T.T
    assert _relnorm(g, ref) <= 1e-9


def test_scale_and_ragged_shapes():
    # a shape that is not a multiple of any tile, and the scale argument
    m, n, k, p = 131, 97, 7, 5
    A = _case(m, n, seed=9, noise=1e-2)
    dA = to_dev(A, torch.float64)
    om = P.gaussian(k + p, m, seed=3, dtype=torch.float64)
    r = P.id_col(dA, k, p=p, q=0, omega=om)
    J = r.J.cpu().numpy().astype(np.int64)
    g = P.id_col_backward(dA, r.J, r.T, k, omega=om, scale=-0.25).cpu().numpy()
    want = -0.25 * adjoint.recon_grad(A, J, k, om.cpu().numpy())
    assert _relnorm(g, want) <= 1e-9


def test_autograd_function_matches_direct_call():
    m, n, k, p = 256, 160, 16, 10
    A = _case(m, n, seed=12, noise=1e-3)
    dA = to_dev(A, torch.float64).requires_grad_(True)
    om = P.gaussian(k + p, m, seed=5, dtype=torch.float64)
    L = P.recon_loss(dA, k, om)
    L.backward()
    r = P.id_col(dA.detach(), k, p=p, q=0, omega=om)
    J = r.J.cpu().numpy().astype(np.int64)
    # the loss value: (e_ID |A|_F)^2 of the same ID
    Lref = adjoint.recon_loss(A, J, k, om.cpu().numpy())
    assert abs(float(L.detach()) - Lref) <= 1e-9 * Lref
    want = adjoint.recon_grad(A, J, k, om.cpu().numpy())
    assert _relnorm(dA.grad.cpu().numpy(), want) <= 1e-9


def test_out_of_range_index_is_reported():
    # an index outside [0, n) is clamped on the device and reported, never read
    m, n, k = 64, 40, 4
    A = _case(m, n, seed=1, noise=1e-2)
    dA = to_dev(A, torch.float64)
    r = P.id_col(dA, k)
    Jbad = r.J.clone()
    Jbad[5] = n + 1000
    with pytest.raises(P.IDCurError):
        P.id_col_backward(dA, Jbad, r.T, k)
        P.sync_status(dA.device)


def test_full_size_differentiable_id_workload():
    # the differentiable-ID workload at its full size: FP32 8192 x 4096, spectrum
    # (j+1)^-1.5 under N(0, 1e-3^2) noise, k = 128, p = 10, q = 0
    cfg = synth.CONFIGS["diff_fp32_8192x4096_k128"]
    m, n, k, p = cfg.m, cfg.n, cfg.k, cfg.p
    say(f"adjoint full size {m}x{n} k={k} p={p}")
    dev = torch.device("cuda")
    A = synth.noisy_lowrank_torch(m, n, cfg.spectrum(), 1e-3, seed=2024, device=dev).to(torch.float32).contiguous()
    om = P.gaussian(k + p, m, seed=11, dtype=torch.float32)
    r = P.id_col(A, k, p=p, q=0, omega=om)
    assert r.k == k
    J = r.J.cpu().numpy().astype(np.int64)
    check_perm(J, n)
    g = P.id_col_backward(A, r.J, r.T, k, omega=om).cpu().numpy().astype(np.float64)
    want = adjoint.recon_grad(A.double().cpu().numpy(), J, k, om.double().cpu().numpy())
    e = _relnorm(g, want)
    say(f"  |dA - oracle| / |oracle| = {e:.3e}")
    assert e <= 2e-4
