"""Orthonormal non-standard 2-D Haar transform of each cube face (FP64).

Test infrastructure only (see the package docstring).

Follows Sec. V.B: at every scale the horizontal, vertical and diagonal
coefficients are first-order finite differences of the signal along the
columns, the rows and both, and the next coarser scale is obtained from 2x2
averages.  For one 2x2 block [[a, b], [c, d]] (row-major, a top-left):

    S = (a + b + c + d) / 2      scaling (block average, orthonormal weight)
    H = (a - b + c - d) / 2      left minus right   (derivative along phi)
    V = (a + b - c - d) / 2      top minus bottom   (derivative along theta)
    D = (a - b - c + d) / 2      mixed difference

The non-standard (quadtree) decomposition repeats this on the S values.
Output layout per face is the Mallat quadrant layout: S/H/V/D of the current
level go to the top-left/top-right/bottom-left/bottom-right quadrants of the
current s x s corner, and the recursion continues in the top-left quadrant.
With this normalisation the transform is orthonormal and a constant face of
value c has a single non-zero coefficient N*c at (0, 0).
"""
import numpy as np


def haar_forward(x):
    """Forward transform of the last two axes (n x n, n a power of two)."""
    c = np.array(x, dtype=np.float64, copy=True)
    n = c.shape[-1]
    assert c.shape[-2] == n and n >= 1 and (n & (n - 1)) == 0
    s = n
    while s > 1:
        blk = c[..., :s, :s]
        a = blk[..., 0::2, 0::2]
        b = blk[..., 0::2, 1::2]
        cc = blk[..., 1::2, 0::2]
        d = blk[..., 1::2, 1::2]
        h = s // 2
        out = np.empty_like(blk)
        out[..., :h, :h] = (a + b + cc + d) / 2.0
        out[..., :h, h:] = (a - b + cc - d) / 2.0
        out[..., h:, :h] = (a + b - cc - d) / 2.0
        out[..., h:, h:] = (a - b - cc + d) / 2.0
        c[..., :s, :s] = out
        s = h
    return c


def haar_inverse(coef):
    """Inverse (= transpose) of haar_forward."""
    x = np.array(coef, dtype=np.float64, copy=True)
    n = x.shape[-1]
    s = 2
    while s <= n:
        h = s // 2
        S = x[..., :h, :h]
        H = x[..., :h, h:s]
        V = x[..., h:s, :h]
        D = x[..., h:s, h:s]
        blk = np.empty(x.shape[:-2] + (s, s), dtype=np.float64)
        blk[..., 0::2, 0::2] = (S + H + V + D) / 2.0
        blk[..., 0::2, 1::2] = (S - H + V - D) / 2.0
        blk[..., 1::2, 0::2] = (S + H - V - D) / 2.0
        blk[..., 1::2, 1::2] = (S - H - V + D) / 2.0
        x[..., :s, :s] = blk
        s *= 2
    return x


def coefficient_block(r, c, n):
    """Which basis function sits at Mallat position (r, c) of an n x n face.

    Returns (kind, size, br, bc): kind in 'S', 'H', 'V', 'D'; the function is
    supported on the size x size texel block whose top-left texel is
    (br*size, bc*size).
    """
    if r == 0 and c == 0:
        return "S", n, 0, 0
    m = max(r, c)
    q = 1 << (m.bit_length() - 1)         # quadrant side at this level
    size = n // q
    if r < q:
        return "H", size, r, c - q
    if c < q:
        return "V", size, r - q, c
    return "D", size, r - q, c - q
