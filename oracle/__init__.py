"""Oracle: a plain, slow, FP64 CPU implementation of the CUR / interpolative
decomposition path (Voronin & Martinsson, "Efficient Algorithms for CUR and
Interpolative Matrix Decompositions").

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or run it. The product
path (``paper_1412_8447_amd``) never imports it and shares no code, constants or
helpers with it; the two meet only through the seeded inputs of ``synth``.

Layout of the oracle:

* ``cpqr``     -- truncated column-pivoted Householder QR (Section 2.2, eq. (trunc)),
                  with exact column norms recomputed at every step.
* ``backsub``  -- back-substitution for upper-triangular systems (Section 4.1).
* ``decomp``   -- column ID (Algorithm 1), row ID (remark in Section 2.3), two-sided
                  ID (Algorithm 2), CUR-ID (Algorithm 3), the Gaussian sketch and
                  the orthonormalised power scheme (Algorithm 4 and Section 5.3).
* ``errors``   -- the reported error measures (Frobenius; spectral at small sizes).
* ``philox``   -- Philox4x32-10 (Salmon et al., SC'11) and a Box-Muller transform,
                  the counter-based generator used for the sketch matrix.
* ``srht``     -- the subsampled randomized Hadamard sketch (the real counterpart
                  of the structured sketch of Section 5.2).

Every function here is pinned by a ``-m "not gpu"`` test against something other
than itself (brute force, closed forms, library routines, identities from the
paper). A function without such a pin says "parity unpinned" in its docstring.
"""
from .cpqr import cpqr, CPQRResult, default_rank_tol
from .backsub import back_substitute
from .decomp import (
    orth,
    sketch,
    id_col,
    id_row,
    two_sided,
    cur,
    vstar_from,
    w_from,
    IDResult,
    TwoSidedResult,
    CURResult,
)
from .errors import (
    rel_fro,
    e_id,
    e_two_sided,
    e_cur,
)
from .stabilized import interp_tikhonov, interp_tsvd, tikhonov_weight
from . import philox

__all__ = [
    "cpqr", "CPQRResult", "default_rank_tol", "back_substitute", "orth", "sketch",
    "id_col", "id_row", "two_sided", "cur", "vstar_from", "w_from",
    "IDResult", "TwoSidedResult", "CURResult", "rel_fro", "e_id", "e_two_sided",
    "e_cur", "philox", "interp_tikhonov", "interp_tsvd", "tikhonov_weight",
]
