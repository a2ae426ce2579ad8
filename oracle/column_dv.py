"""Column systems of the paper's section 2.3 ("Matrix-free solvers"), solved
densely: the oracle of the library's matrix-free column scans.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 2.3 prints, for a 3-layer column, the two block matrices

    D_vu  (horizontal pressure gradient system, D_vu r = F)
    D_vd  (vertical velocity system,           D_vd w = F)

in units of M_h / 2, with M_h = J_h/24 [2 1 1; 1 2 1; 1 1 2] the 2D mass
matrix, and says the pattern continues with more layers.  Unknowns of a layer
are ordered top-face nodes then bottom-face nodes (3 each), layers from the
surface down.  The oracle writes the pattern out for N layers, assembles each
column's 6N x 6N matrix with dense Kronecker products and calls
``numpy.linalg.solve``: no recursion, no reordering.
"""

from __future__ import annotations

import numpy as np

# block patterns per layer l (0-based), in units of M_h / 2; columns index
# (layer, face) with face 0 = top nodes, 1 = bottom nodes
#   D_vu, top rows of l:    +2 (l-1, bottom)  -1 (l, top)  -1 (l, bottom)
#   D_vu, bottom rows of l: +1 (l, top)       -1 (l, bottom)
#   D_vd, top rows of l:    +1 (l, top)       -1 (l, bottom)
#   D_vd, bottom rows of l: +1 (l, top)       +1 (l, bottom)  -2 (l+1, top)


def pattern(kind: str, n_layers: int) -> np.ndarray:
    """(2N, 2N) coefficient grid of D_vu or D_vd in units of M_h / 2."""
    n = 2 * n_layers
    P = np.zeros((n, n))
    for l in range(n_layers):
        t, b = 2 * l, 2 * l + 1
        if kind == "vu":
            if l > 0:
                P[t, 2 * (l - 1) + 1] = 2.0
            P[t, t] = -1.0
            P[t, b] = -1.0
            P[b, t] = 1.0
            P[b, b] = -1.0
        elif kind == "vd":
            P[t, t] = 1.0
            P[t, b] = -1.0
            P[b, t] = 1.0
            P[b, b] = 1.0
            if l + 1 < n_layers:
                P[b, 2 * (l + 1)] = -2.0
        else:
            raise ValueError(kind)
    return P


def mass_2d(jh: float) -> np.ndarray:
    """M_h = J_h/24 [2 1 1; 1 2 1; 1 1 2] (section 2.3)."""
    return jh / 24.0 * np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]])


def column_matrix(kind: str, n_layers: int, jh: float) -> np.ndarray:
    """The 6N x 6N matrix (1/2) pattern (x) M_h of one column."""
    return 0.5 * np.kron(pattern(kind, n_layers), mass_2d(jh))


def column_jh(vxy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """J_h = (x1-x0)(y2-y0) - (x2-x0)(y1-y0) per triangle (twice its area)."""
    p = vxy[tri]
    return (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])


def dv_solve(kind: str, vxy, tri, nlayers, F: np.ndarray) -> np.ndarray:
    """Solve D x = F in every column.  F: (K, 6, P) in natural prism order
    (column by column, layers top to bottom); returns x of the same shape."""
    F = np.asarray(F, dtype=np.float64)
    K = F.shape[0]
    jh = column_jh(np.asarray(vxy, np.float64), np.asarray(tri))
    nl = np.asarray(nlayers)
    off = np.concatenate([[0], np.cumsum(nl)])
    x = np.empty_like(F)
    for c in range(len(nl)):
        N = int(nl[c])
        A = column_matrix(kind, N, float(jh[c]))
        # unknown vector of a column: layer by layer, 6 nodes each
        rhs = F[:, :, off[c]:off[c] + N].transpose(2, 1, 0).reshape(6 * N, K)
        sol = np.linalg.solve(A, rhs)
        x[:, :, off[c]:off[c] + N] = sol.reshape(N, 6, K).transpose(2, 1, 0)
    return x
