"""Pins of the horizontal (along-layer) diffusion term of the oracle.

Routes other than the oracle's own quadrature:
* constants are annihilated and the sum over all test functions vanishes
  (zero-flux boundaries conserve the tracer);
* the symmetric interior penalty form gives a symmetric, negative
  semi-definite matrix;
* a field linear in x and y is reproduced exactly on every prism whose three
  lateral faces are interior: zero on flat layers, and on sloped layers the
  closed form kh (a, b) . grad(z_zeta) J_h / 6 of the along-layer operator;
* on a closed square with flat layers the smallest nonzero generalised
  eigenvalue of (D, M) converges to -kh (pi/L)^2 (the first Neumann mode)
  at second order;
* Okubo's relation in metres agrees with its centimetre form.
"""

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from oracle.horizontal_diffusion import OKUBO_COEF, horizontal_diffusion_term, okubo_diffusivity

L_DOM = W.prism_mesh.DOMAIN_L


def _mesh(w):
    return O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)


def _flat(n, n_layers=1, jitter=0.2, seed=0, dz=2.0):
    vxy, tri, nbr = W.prism_mesh.square_mesh(n, jitter=jitter, seed=seed)
    nl = np.full(len(tri), n_layers)
    zl = np.concatenate([np.repeat((-np.arange(n_layers + 1) * dz)[:, None], 3, 1) for _ in nl])
    return O.PrismMesh(vxy, tri, nbr, nl, zl)


def _matrix(m, kh, eta=4.0, chunk=256):
    n = 6 * m.P
    D = np.zeros((n, n))
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        E = np.zeros((j1 - j0, 6 * m.P))
        E[np.arange(j1 - j0), np.arange(j0, j1)] = 1.0
        D[:, j0:j1] = horizontal_diffusion_term(m, kh, E.reshape(j1 - j0, 6, m.P), eta).reshape(j1 - j0, -1).T
    return D


def test_okubo_units():
    l_m = 250.0
    k_cgs = 0.0103 * (l_m * 100.0) ** 1.15      # cm^2/s with l in cm
    assert abs(OKUBO_COEF * l_m ** 1.15 - k_cgs * 1e-4) < 1e-12 * k_cgs * 1e-4


@pytest.mark.parametrize("mesh", ["ragged", "sigma"])
def test_constants_and_conservation(mesh):
    w = W.ragged(seed=2, n=5, n_fields=1) if mesh == "ragged" else W.rotating_blob(n=5, n_layers=3)
    m = _mesh(w)
    kh = okubo_diffusivity(m, 50.0)
    D1 = horizontal_diffusion_term(m, kh, np.full((1, 6, m.P), 3.0))
    T = np.random.default_rng(4).standard_normal((2, 6, m.P))
    D = horizontal_diffusion_term(m, kh, T)
    scale = np.abs(D).max()
    assert np.abs(D1).max() < 1e-13 * scale
    assert np.abs(D.sum(axis=(1, 2))).max() < 1e-12 * scale * m.P


@pytest.mark.parametrize("mesh", ["ragged", "sigma"])
def test_symmetric_negative_semidefinite(mesh):
    w = W.ragged(seed=5, n=3, n_fields=1, n_max=4) if mesh == "ragged" else W.rotating_blob(n=3, n_layers=2)
    m = _mesh(w)
    kh = okubo_diffusivity(m, 10.0) * np.linspace(0.5, 2.0, m.C)       # varying kh per column
    D = _matrix(m, kh)
    assert np.abs(D - D.T).max() < 1e-12 * np.abs(D).max()
    ev = np.linalg.eigvalsh(0.5 * (D + D.T))
    assert ev.max() < 1e-10 * np.abs(ev).max(), ev.max()


def _interior_prisms(m):
    ok = np.ones(m.P, dtype=bool)
    for k in range(3):
        c2 = m.nbr[m.col, k]
        ok &= (c2 >= 0) & (m.lay < m.nl[np.where(c2 >= 0, c2, 0)])
    return ok


def test_linear_field_flat_layers():
    m = _flat(6, n_layers=2)
    kh = np.full(m.C, 3.5)
    a, b = 0.7, -1.3
    T = (a * m.X + b * m.Y)
    T = np.concatenate([T, T], axis=1).T[None]          # (1, 6, P): top and bottom nodes
    D = horizontal_diffusion_term(m, kh, T)
    inner = _interior_prisms(m)
    assert inner.sum() > 10
    scale = np.abs(horizontal_diffusion_term(m, kh, np.random.default_rng(1).standard_normal(T.shape))).max()
    assert np.abs(D[:, :, inner]).max() < 1e-12 * scale


def test_linear_field_sloped_layers_closed_form():
    w = W.rotating_blob(n=6, n_layers=3)
    m = _mesh(w)
    kh = np.full(m.C, 2.0)
    a, b = 0.4, 0.9
    T = np.concatenate([a * m.X + b * m.Y, a * m.X + b * m.Y], axis=1).T[None]
    D = horizontal_diffusion_term(m, kh, T)[0]
    # grad of z_zeta = (z_top - z_bottom)/2, linear on the triangle
    x1, x2 = m.X[:, 1] - m.X[:, 0], m.X[:, 2] - m.X[:, 0]
    y1, y2 = m.Y[:, 1] - m.Y[:, 0], m.Y[:, 2] - m.Y[:, 0]
    Jh = x1 * y2 - x2 * y1
    zz = 0.5 * (m.ZT - m.ZB)
    d1, d2 = zz[:, 1] - zz[:, 0], zz[:, 2] - zz[:, 0]
    gx = (d1 * y2 - d2 * y1) / Jh
    gy = (x1 * d2 - x2 * d1) / Jh
    ref = 2.0 * (a * gx + b * gy) * Jh / 6.0
    inner = _interior_prisms(m)
    assert inner.sum() > 10 and np.abs(ref[inner]).max() > 1e-3
    err = np.abs(D[:, inner] - ref[None, inner]).max()
    assert err < 1e-11 * np.abs(ref[inner]).max(), err


def test_first_neumann_eigenvalue_second_order():
    kappa = 5.0
    exact = kappa * (np.pi / L_DOM) ** 2
    errs = []
    for n in (4, 8, 16):
        m = _flat(n, jitter=0.0)
        D = _matrix(m, np.full(m.C, kappa))
        M = scipy.linalg.block_diag(*O.mass_matrix(m))
        # unknowns are (node, prism) in D; reorder M accordingly
        perm = (np.arange(6)[:, None] * m.P + np.arange(m.P)[None, :]).T.ravel()
        Mn = np.zeros_like(M)
        Mn[np.ix_(perm, perm)] = M
        ev = scipy.linalg.eigh(-0.5 * (D + D.T), Mn, eigvals_only=True)
        lam = np.sort(ev)[np.sort(ev) > 1e-9 * exact][0]
        errs.append(abs(lam - exact) / exact)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("eigenvalue errors", errs, "orders", orders)
    assert errs[-1] < 0.02 and np.all(orders > 1.8), (errs, orders)
