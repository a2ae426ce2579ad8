"""Pins of the split-IMEX step of the oracle (two steps: vertically implicit
over dt/2, then explicit over dt).

Routes other than the oracle's own code:
* pure vertical diffusion: the two steps compose to the trapezoidal
  (Crank-Nicolson) rule, computed here directly as (M - dt/2 A)^-1 (M + dt/2 A);
* pure advection: the explicit midpoint rule T0 + dt L(T0 + dt/2 L(T0));
* the mass budget: the change of mass over a step is minus dt times the
  boundary flux of the step-1 field (A conserves, R only exchanges through
  open boundaries); a closed flow conserves mass and keeps constants;
* second order in time against the exact solution of the semi-discrete
  linear system (matrix exponential).
"""

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from oracle.split_imex import imex_step, vertical_diffusion_apply


def _mesh(w):
    return O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)


def test_pure_diffusion_is_crank_nicolson():
    w = W.ragged(seed=2, n=5, n_fields=2)
    m = _mesh(w)
    U0 = np.zeros_like(w.U)
    kappa = np.full(int(w.nlayers.max()), 0.5)           # stiff: dt kappa / dz^2 >> 1
    dt = 200.0
    T1 = imex_step(m, U0, kappa, w.T0, dt, w.t_ext)
    for c in range(m.C):
        K, Mc = O.column_system(m, kappa, 0.5 * dt, c)   # K = M - dt/2 A
        ps = m.off[c] + np.arange(m.nl[c])
        x0 = w.T0[:, :, ps].transpose(2, 1, 0).reshape(-1, w.n_fields)
        ref = np.linalg.solve(K, (2.0 * Mc - K) @ x0)    # (M - dt/2 A)^-1 (M + dt/2 A) x0
        got = T1[:, :, ps].transpose(2, 1, 0).reshape(-1, w.n_fields)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), c


def test_pure_advection_is_explicit_midpoint():
    w = W.rotating_blob(n=5, n_layers=3)
    m = _mesh(w)
    rng = np.random.default_rng(3)
    T0 = w.T0 + 0.1 * rng.standard_normal(w.T0.shape)
    kappa = np.zeros(3)
    T1 = imex_step(m, w.U, kappa, T0, w.dt, [0.7])
    L = lambda X: O.explicit_operator(m, w.U, X, [0.7])
    ref = T0 + w.dt * L(T0 + 0.5 * w.dt * L(T0))
    assert np.max(np.abs(T1 - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_mass_budget_identity():
    w = W.rotating_blob(n=6, n_layers=4)
    m = _mesh(w)
    kappa = np.geomspace(1e-1, 1e-3, 4)
    T1, Th = imex_step(m, w.U, kappa, w.T0, w.dt, w.t_ext, return_half=True)
    dm = O.mass(m, T1) - O.mass(m, w.T0)
    pred = -w.dt * O.boundary_flux(m, w.U, Th, w.t_ext)
    assert np.abs(dm - pred).max() < 1e-12 * np.abs(O.mass(m, w.T0)).max()
    # the step-1 budget: half a step of the boundary flux of the initial field
    dmh = O.mass(m, Th) - O.mass(m, w.T0)
    assert np.abs(dmh + 0.5 * w.dt * O.boundary_flux(m, w.U, w.T0, w.t_ext)).max() < \
        1e-12 * np.abs(O.mass(m, w.T0)).max()


def test_closed_flow_conserves_and_keeps_constants():
    from tests.test_oracle_pins import _closed_flow
    w, U = _closed_flow()
    m = _mesh(w)
    kappa = np.full(w.nlayers.max(), 1e-2)
    T = w.T0 + 0.3 * np.random.default_rng(1).standard_normal(w.T0.shape)
    m0 = O.mass(m, T)
    X = T
    for _ in range(3):
        X = imex_step(m, U, kappa, X, w.dt, [5.0])
    assert abs(O.mass(m, X)[0] - m0[0]) < 1e-13 * abs(m0[0])
    C = imex_step(m, U, kappa, np.full_like(T, 2.5), w.dt, [9.0])
    assert np.abs(C - 2.5).max() < 1e-12


def test_second_order_in_time():
    w = W.tiny(n_fields=1)
    m = _mesh(w)
    n = 6 * m.P
    kappa = np.geomspace(5e-3, 5e-4, 3)
    t_ext = [0.0]                                   # linear operator
    Mp = O.mass_matrix(m)                           # (P, 6, 6), block-diagonal M
    G = np.zeros((n, n))                            # M^-1 (R + A) as a matrix
    for j in range(n):
        e = np.zeros((1, 6, m.P))
        e.reshape(-1)[j] = 1.0
        Ae = vertical_diffusion_apply(m, kappa, e)[0]                       # (6, P)
        MinvAe = np.linalg.solve(Mp, Ae.T[:, :, None])[:, :, 0].T           # (6, P)
        G[:, j] = O.explicit_operator(m, w.U, e, t_ext).reshape(-1) + MinvAe.reshape(-1)
    T0 = w.T0.reshape(-1)
    t_end = 4 * w.dt
    exact = scipy.linalg.expm(t_end * G) @ T0
    errs = []
    for k in (16, 32, 64):
        dt = t_end / k
        X = w.T0
        for _ in range(k):
            X = imex_step(m, w.U, kappa, X, dt, t_ext)
        errs.append(np.max(np.abs(X.reshape(-1) - exact)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("errors", errs, "orders", orders)
    assert np.all(np.abs(orders - 2.0) < 0.15), (errs, orders)
