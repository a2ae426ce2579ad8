"""Pins of the dense column-system oracle (section 2.3, matrix-free solvers).

Routes other than the oracle's own assembly:
* the 3-layer matrices as printed in the paper (golden fixtures);
* the solution against the system assembled directly from those printed
  3-layer matrices and the printed M_h (residual);
* the continuous problems behind the two systems (dx/dz = f with x = 0 at the
  surface for D_vu and at the seabed for D_vd): right-hand sides computed by
  quadrature of the weak form, and the exact integrals of f, which the
  discrete solution reproduces at every outflow face and, for sources
  constant in depth, at every node.
"""

import os

import numpy as np
import pytest

import oracle as O
import workloads as W

CD = O.column_dv
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    rows = [l.split() for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=np.float64)


def _jh(p):
    """Twice the signed area of each triangle p (C, 3, 2)."""
    e1, e2 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]
    return e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]


def _ragged():
    w = W.ragged(seed=3, n=6, n_fields=1)
    return w.vxy, w.tri, w.nlayers


@pytest.mark.parametrize("kind", ["vu", "vd"])
def test_printed_three_layer_pattern(kind):
    assert np.array_equal(CD.pattern(kind, 3), _load(f"column_dv_{kind}_3layer.txt"))


def test_printed_mass_matrix():
    jh = 7.25
    assert np.allclose(CD.mass_2d(jh), _load("mass_2d.txt") * jh / 24.0, rtol=0, atol=1e-15)
    # the (layer 0 top, layer 0 top) block of the assembled matrix is -M_h / 2 for D_vu
    A = CD.column_matrix("vu", 2, jh)
    assert np.allclose(A[:3, :3], -0.5 * _load("mass_2d.txt") * jh / 24.0, atol=1e-15)


def test_solution_satisfies_printed_system():
    """On 3-layer columns the solution satisfies the system assembled from the
    printed matrices themselves: (1/2) pattern (x) M_h, both from the golden
    fixtures, with no use of the oracle's own pattern or assembly."""
    w = W.tiny(seed=4, n=3, n_layers=3)
    nl = w.nlayers
    assert np.all(nl == 3)
    rng = np.random.default_rng(11)
    F = rng.standard_normal((2, 6, int(nl.sum())))
    jh = _jh(w.vxy[w.tri])
    mh = _load("mass_2d.txt") / 24.0
    for kind in ("vu", "vd"):
        x = CD.dv_solve(kind, w.vxy, w.tri, nl, F)
        printed = _load(f"column_dv_{kind}_3layer.txt")
        for c in range(len(nl)):
            D = 0.5 * np.kron(printed, jh[c] * mh)
            for k in range(2):
                xs = x[k, :, 3 * c:3 * c + 3].T.ravel()      # (layer, node)
                fs = F[k, :, 3 * c:3 * c + 3].T.ravel()
                assert np.max(np.abs(D @ xs - fs)) <= 1e-12 * np.max(np.abs(fs)), (kind, c, k)


# -- the continuous problems -------------------------------------------------
# reference triangle rule exact to degree 2 (edge midpoints, weight 1/6 each)
_TRI_Q = np.array([[0.5, 0.0], [0.5, 0.5], [0.0, 0.5]])
_TRI_QW = np.full(3, 1.0 / 6.0)
# 2-point Gauss on [-1, 1] (exact to degree 3)
_GZ = np.array([-1.0, 1.0]) / np.sqrt(3.0)


def _weak_rhs(jh, a, b):
    """F of one column for the source q = sum_j lambda_j (a_j + b_j zhat) per
    layer (zhat = +1 on the layer's top face): F_i = int phi_i q J_h, with the
    nodal basis lambda_i (1 + zhat)/2 (top) and lambda_i (1 - zhat)/2 (bottom)."""
    N = a.shape[0]
    F = np.zeros((N, 6))
    for (xi, et), wq in zip(_TRI_Q, _TRI_QW):
        lam = np.array([1.0 - xi - et, xi, et])
        for zh in _GZ:
            q = (a + b * zh) @ lam           # (N,)
            F[:, :3] += wq * jh * np.outer(q * (1.0 + zh) / 2.0, lam)
            F[:, 3:] += wq * jh * np.outer(q * (1.0 - zh) / 2.0, lam)
    return F


def _column_sources(rng, nl, linear):
    a = rng.uniform(-1.0, 1.0, size=(nl, 3))
    b = rng.uniform(-1.0, 1.0, size=(nl, 3)) if linear else np.zeros((nl, 3))
    return a, b


@pytest.mark.parametrize("linear", [False, True])
@pytest.mark.parametrize("kind", ["vu", "vd"])
def test_weak_form_exactness(kind, linear):
    vxy, tri, nl = _ragged()
    rng = np.random.default_rng(5 + int(linear))
    p = vxy[tri]
    jh = _jh(p)
    off = np.concatenate([[0], np.cumsum(nl)])
    P = int(nl.sum())
    F = np.zeros((1, 6, P))
    srcs = []
    for c in range(len(nl)):
        a, b = _column_sources(rng, int(nl[c]), linear)
        srcs.append((a, b))
        F[0, :, off[c]:off[c + 1]] = _weak_rhs(jh[c], a, b).T
    x = CD.dv_solve(kind, vxy, tri, nl, F)[0]
    for c in range(len(nl)):
        a, b = srcs[c]
        X = x[:, off[c]:off[c + 1]].T           # (N, 6)
        inc = 2.0 * a                            # integral of q over a layer, per node
        if kind == "vu":
            # x(surface) = 0, x decreases downwards by the layer integral
            bot = -np.cumsum(inc, axis=0)
            top = bot + inc
            out_face, in_face, exact_out, exact_in = X[:, 3:], X[:, :3], bot, top
        else:
            # x(seabed) = 0, x increases upwards by the layer integral
            top = np.cumsum(inc[::-1], axis=0)[::-1]
            bot = top - inc
            out_face, in_face, exact_out, exact_in = X[:, :3], X[:, 3:], top, bot
        scale = np.max(np.abs(exact_out)) + 1.0
        assert np.max(np.abs(out_face - exact_out)) <= 1e-12 * scale, c
        if not linear:
            assert np.max(np.abs(in_face - exact_in)) <= 1e-12 * scale, c
        else:
            # a source linear in depth is not reproduced at the inflow face
            assert np.max(np.abs(in_face - exact_in)) > 1e-6


def test_single_layer_closed_form():
    # one prism, D_vu: -(r_t + r_b)/2 M = F_t, (r_t - r_b)/2 M = F_b
    jh = 3.0
    M = CD.mass_2d(jh)
    rt, rb = np.array([1.0, -2.0, 0.5]), np.array([0.25, 4.0, -1.0])
    Ft, Fb = -0.5 * M @ (rt + rb), 0.5 * M @ (rt - rb)
    vxy = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 1.0]])
    F = np.concatenate([Ft, Fb])[None, :, None]
    x = CD.dv_solve("vu", vxy, np.array([[0, 1, 2]]), np.array([1]), F)
    assert np.allclose(x[0, :, 0], np.concatenate([rt, rb]), rtol=0, atol=1e-13)
