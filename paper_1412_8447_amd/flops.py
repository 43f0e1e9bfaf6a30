"""Algorithmic operation counts of the ID / CUR path (host-side accounting).

Counts follow the cost statements of the paper: a k-step column-pivoted QR of an
l x n matrix costs sum_{j<k} 4 (l-j)(n-j) flops (Section 4.4: O(mnk) dominated by
the first k QR steps), the sketch Y = Omega A costs 2 l m n per product with A or
A^T and the power scheme repeats it 2q times (Section 5.3: O((2q+1) mnk)), a
triangular solve with k x k factor and r right-hand sides costs k^2 r. The
Cholesky-QR orthonormalisation of an N x l block costs 2 N l^2 (Gram) +
l^3 / 3 (factor) + N l^2 (triangular solve).
"""
from __future__ import annotations


def cpqr_flops(l: int, n: int, k: int) -> float:
    return float(sum(4.0 * (l - j) * (n - j) for j in range(min(k, l, n))))


def orth_flops(N: int, l: int, passes: int = 1) -> float:
    return passes * (2.0 * N * l * l + l ** 3 / 3.0 + 1.0 * N * l * l)


def flop_model(op: str, m: int, n: int, k: int, p: int = -1, q: int = 0, orth_passes: int = 1,
               u_passes: int = 2) -> dict:
    """Per-stage and total algorithmic flops for op in {"id_col", "id_row",
    "two_sided", "cur"} on an m x n matrix with rank k, oversampling p (p < 0:
    deterministic) and q orthonormalised power steps."""
    if op == "id_row":
        m, n = n, m
    out = {}
    sketched = p >= 0 and k + p < m
    l = k + p if sketched else m
    if sketched:
        out["sketch"] = 2.0 * l * m * n * (2 * q + 1)
        out["orth"] = q * (orth_flops(n, l, orth_passes) + orth_flops(m, l, orth_passes))
    out["cpqr"] = cpqr_flops(l, n, k)
    out["trsm"] = float(k) * k * (n - k)
    if op in ("two_sided", "cur"):
        out["row_cpqr"] = cpqr_flops(k, m, k)
        out["row_trsm"] = float(k) * k * (m - k)
    if op == "cur":
        # CholeskyQR (u_passes) of R^T (n x k), Q^T V (k x n x k), two k x k solves
        out["u"] = u_passes * (2.0 * n * k * k + k ** 3 / 3.0 + n * k * k) + 2.0 * n * k * k + 2.0 * k ** 3
    out["total"] = float(sum(out.values()))
    return out


def batched_flops(ms, ns, ks, l: int) -> float:
    """Batched column IDs (one sketch width l per block): sketch 2 l m n, the
    k-step pivoted QR of the l x n sketch, and the k x k triangular solve with
    n - k right-hand sides, summed over blocks."""
    tot = 0.0
    for m, n, k in zip(ms, ns, ks):
        k = max(int(k), 0)
        tot += 2.0 * l * m * n + cpqr_flops(l, n, k) + float(k) * k * (n - k)
    return tot


def adjoint_flops(m: int, n: int, k: int, l: int = 0) -> float:
    """Gradient of the column-ID reconstruction loss (skeleton frozen), sketched
    with l rows (l = 0: Y = A): E = A(:,J2) - C T, Tbar = -2 C^T E and -2 E T^T
    (2 m (n-k) k each), Y = Omega A(:,J) and Omega^T Ybar (2 l m n each), the Gram
    matrix (2 k^2 l, or 2 k^2 m), its Cholesky factor (k^3 / 3), M (2 k^2 (n-k)),
    T M^T (2 k^2 (n-k)), Y2 - Y1 T, Y1 M and (Y2 - Y1 T) M^T (2 l k (n-k) each),
    Y1 (T M^T) (2 l k^2); without a sketch the last group works on m rows and
    Y2 - Y1 T is E itself."""
    n2 = n - k
    rows = l if l > 0 else m
    f = 3 * 2.0 * m * n2 * k
    if l > 0:
        f += 2 * 2.0 * l * m * n
    f += 2.0 * k * k * rows + k ** 3 / 3.0 + 2 * 2.0 * k * k * n2
    f += (3 if l > 0 else 2) * 2.0 * rows * k * n2 + 2.0 * rows * k * k
    return f
