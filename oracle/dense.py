"""Dense eigenvalues of an explicit matrix: the plain definition of what the
eigensolver must reach on tiny grids (the k eigenvalues of smallest real part)."""
from __future__ import annotations

import numpy as np


def lowest_eigenvalues(A, k):
    """The k eigenvalues of A with smallest real part, ascending by real part."""
    ev = np.linalg.eigvals(np.asarray(A, dtype=np.float64))
    order = np.argsort(ev.real, kind="stable")
    return ev[order[:k]]
