"""Non-linear approximation: keep the k coefficients of largest magnitude.

Test infrastructure only (see the package docstring).

Sec. III (Haar-domain methods) and Sec. VI (number of coefficients used per
material): only the largest wavelet coefficients of a signal are kept.  Ranks
are by |value| over all positions (scaling coefficients compete with the
wavelets), ties go to the lower flat index, and the kept positions are
returned in ascending order.
"""
import numpy as np


def topk_abs(x, k):
    """Indices (ascending, int64) of the k largest |x| of a 1-D array."""
    x = np.asarray(x, dtype=np.float64).ravel()
    k = int(k)
    assert 0 <= k <= x.size
    order = np.lexsort((np.arange(x.size), -np.abs(x)))   # |x| desc, index asc
    return np.sort(order[:k])


def topk_rows(X, k):
    """Row-wise topk_abs of a 2-D array -> (idx [rows, k], values [rows, k])."""
    X = np.asarray(X, dtype=np.float64)
    idx = np.stack([topk_abs(row, k) for row in X]) if X.shape[0] else np.zeros((0, k), np.int64)
    vals = np.take_along_axis(X, idx, axis=1) if X.shape[0] else np.zeros((0, k))
    return idx, vals
