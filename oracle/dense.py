"""Dense matrices of linear field operators on small lattices (oracle checks).

The column j of the matrix is the operator applied to the j-th unit field in
the canonical layout, so the dense matrix acts on flattened canonical fields.
"""
from __future__ import annotations

import numpy as np


def dense_matrix(op, shape):
    """Dense matrix of the linear map ``op`` on fields of ``shape``."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = op(e.reshape(shape)).ravel()
        e[j] = 0.0
    return M


def site_diag(values, inner):
    """Block-diagonal matrix of a per-site scalar times the identity on ``inner``
    components (e.g. epsilon(x) on a staggered field)."""
    return np.diag(np.repeat(np.asarray(values, dtype=np.complex128).ravel(), inner))
