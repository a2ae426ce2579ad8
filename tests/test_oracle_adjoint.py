"""Pins of the oracle adjoint: the assembled linear operator equals the
matrix-free residual, A is linear in the per-layer diffusivity, and the
reverse-mode gradient matches central finite differences of the forward
objective (a route that does not use the adjoint at all)."""

import numpy as np
import pytest

import oracle as O
import oracle.adjoint as OA
import workloads as W


def _mesh(w):
    return O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)


@pytest.mark.parametrize("name", ["ragged", "wnonzero"])
def test_assembled_advection_matches_matrix_free(name):
    if name == "ragged":
        w = W.ragged(n=6, n_fields=2)
    else:
        w = W.config1(n=5, n_layers=3)
        rng = np.random.default_rng([5, 7])
        w.U = w.U + 0.05 * rng.standard_normal(w.U.shape)
        w.U[2] = 1e-3 * rng.standard_normal(w.U[2].shape)
    m = _mesh(w)
    R = OA.advection_matrix(m, w.U)
    T = np.random.default_rng(2).standard_normal((2, 6, m.P))
    got = OA._unflat(R @ OA._flat(T), 2)
    ref = O.advective_residual(m, w.U, T, [0.0, 0.0])
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_vertical_operator_is_linear_in_kappa():
    w = W.ragged(n=5)
    m = _mesh(w)
    kap = np.geomspace(1e-2, 1e-4, len(w.kappa))
    A = OA.vertical_matrix_global(m, kap)
    S = None
    for l in range(len(kap)):
        e = np.zeros_like(kap)
        e[l] = 1.0
        term = kap[l] * OA.vertical_matrix_global(m, e)
        S = term if S is None else S + term
    assert abs(A - S).max() <= 1e-13 * abs(A).max()


def _fd_check(m, w, n_steps, seed):
    J, gT, gk = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n_steps, w.penalty)
    rng = np.random.default_rng(seed)
    for trial in range(3):
        d = rng.standard_normal(w.T0.shape)
        d /= np.abs(d).max()
        eps = 1e-6
        jp = OA.objective_after_steps(m, w.U, w.kappa, w.T0 + eps * d, w.dt, w.t_ext, n_steps, w.penalty)
        jm = OA.objective_after_steps(m, w.U, w.kappa, w.T0 - eps * d, w.dt, w.t_ext, n_steps, w.penalty)
        fd = (jp - jm) / (2 * eps)
        ad = float(np.sum(gT * d))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("T0", trial, fd, ad)
        dk = rng.standard_normal(w.kappa.shape) * w.kappa
        jp = OA.objective_after_steps(m, w.U, w.kappa + eps * dk, w.T0, w.dt, w.t_ext, n_steps, w.penalty)
        jm = OA.objective_after_steps(m, w.U, w.kappa - eps * dk, w.T0, w.dt, w.t_ext, n_steps, w.penalty)
        fd = (jp - jm) / (2 * eps)
        ad = float(np.sum(gk * dk))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("kappa", trial, fd, ad)


def test_gradient_matches_finite_differences_tiny():
    w = W.tiny(n_fields=2)
    w.dt *= 20.0          # makes the vertical solve matter
    _fd_check(_mesh(w), w, 3, 1)


def test_gradient_matches_finite_differences_ragged():
    w = W.ragged(n=5, n_fields=1)
    w.dt *= 10.0
    _fd_check(_mesh(w), w, 2, 2)
