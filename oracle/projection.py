"""Per-element projection of Hessians onto the PSD cone (oracle).

TEST INFRASTRUCTURE ONLY.  Sec. 5.2 (projection to positive semi-definiteness)
and Alg. 1 (ProjectToPD before the block loop): each element Hessian is
replaced, before assembly, by the nearest positive semi-definite matrix in the
Frobenius norm, V max(Lambda, 0) V^T.  Negative eigenvalues are clamped to
zero (not to a small positive value); this projection is unique, so any
correct eigensolver gives the same result.
"""
from __future__ import annotations

import numpy as np


def project_psd(H):
    """Batched nearest-PSD projection of symmetric matrices H (..., n, n)."""
    Hs = 0.5 * (H + np.swapaxes(H, -1, -2))
    lam, V = np.linalg.eigh(Hs)
    lam = np.maximum(lam, 0.0)
    return np.einsum("...ij,...j,...kj->...ik", V, lam, V)
