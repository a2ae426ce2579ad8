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
        w = W.rotating_blob(n=5, n_layers=3)
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


def _final(m, w, kappa, T0, n_steps, kappa_h):
    return OA.forward(m, w.U, kappa, T0, w.dt, w.t_ext, n_steps, w.penalty, kappa_h)[-1]


def _central_difference(m, xp, xm, eps):
    """(J(+) - J(-)) / (2 eps) without subtracting the two objectives:
    J+^2 - J-^2 = sum_f (x+ - x-)^T M (x+ + x-), so the difference of the
    final states carries the O(eps) signal instead of two nearly equal J."""
    Mp = O.mass_matrix(m)
    dq = np.einsum("fin,nij,fjn->", xp - xm, Mp, xp + xm)
    jp, jm = OA.objective(m, xp), OA.objective(m, xm)
    return dq / (jp + jm) / (2 * eps)


def _fd_check(m, w, n_steps, seed, kappa_h=None):
    J, gT, gk = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n_steps, w.penalty, kappa_h)
    rng = np.random.default_rng(seed)
    for trial in range(3):
        d = rng.standard_normal(w.T0.shape)
        d /= np.abs(d).max()
        eps = 1e-6
        fd = _central_difference(m, _final(m, w, w.kappa, w.T0 + eps * d, n_steps, kappa_h),
                                 _final(m, w, w.kappa, w.T0 - eps * d, n_steps, kappa_h), eps)
        ad = float(np.sum(gT * d))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("T0", trial, fd, ad)
        # J moves by ~1e-5 of itself per unit relative change of kappa, so a
        # step of 1e-6 would drown in the round-off of a stiff column solve
        dk = rng.standard_normal(w.kappa.shape) * w.kappa
        ek = 1e-4
        fd = _central_difference(m, _final(m, w, w.kappa + ek * dk, w.T0, n_steps, kappa_h),
                                 _final(m, w, w.kappa - ek * dk, w.T0, n_steps, kappa_h), ek)
        ad = float(np.sum(gk * dk))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("kappa", trial, fd, ad)


def test_gradient_matches_finite_differences_tiny():
    w = W.tiny(n_fields=2)
    w.kappa = w.kappa * 100.0     # kappa dt / dz^2 up to ~28: the solve matters
    _fd_check(_mesh(w), w, 3, 1)


def test_gradient_matches_finite_differences_ragged():
    w = W.ragged(n=5, n_fields=1)
    w.kappa = w.kappa * 100.0
    _fd_check(_mesh(w), w, 2, 2)


def test_gradient_with_horizontal_diffusion_matches_finite_differences():
    from oracle.horizontal_diffusion import okubo_diffusivity
    w = W.ragged(n=5, n_fields=1)
    w.kappa = w.kappa * 100.0
    m = _mesh(w)
    _fd_check(m, w, 2, 3, kappa_h=okubo_diffusivity(m, 50.0))


def _imex_objective(m, w, kappa, T0, n_steps, kappa_h):
    from oracle.split_imex import imex_step
    x = T0
    for _ in range(n_steps):
        x = imex_step(m, w.U, kappa, x, w.dt, w.t_ext, w.penalty, kappa_h=kappa_h)
    return x


@pytest.mark.parametrize("with_hdiff", [False, True])
def test_imex_gradient_matches_finite_differences(with_hdiff):
    from oracle.horizontal_diffusion import okubo_diffusivity
    w = W.ragged(n=5, n_fields=1)
    w.kappa = w.kappa * 100.0
    m = _mesh(w)
    kh = okubo_diffusivity(m, 50.0) if with_hdiff else None
    n_steps = 2
    J, gT, gk = OA.gradient_imex(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n_steps, w.penalty, kh)
    assert abs(J - OA.objective(m, _imex_objective(m, w, w.kappa, w.T0, n_steps, kh))) <= 1e-13 * J
    rng = np.random.default_rng(7)
    for trial in range(3):
        d = rng.standard_normal(w.T0.shape)
        d /= np.abs(d).max()
        eps = 1e-6
        fd = _central_difference(m, _imex_objective(m, w, w.kappa, w.T0 + eps * d, n_steps, kh),
                                 _imex_objective(m, w, w.kappa, w.T0 - eps * d, n_steps, kh), eps)
        ad = float(np.sum(gT * d))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("T0", trial, fd, ad)
        dk = rng.standard_normal(w.kappa.shape) * w.kappa
        ek = 1e-4
        fd = _central_difference(m, _imex_objective(m, w, w.kappa + ek * dk, w.T0, n_steps, kh),
                                 _imex_objective(m, w, w.kappa - ek * dk, w.T0, n_steps, kh), ek)
        ad = float(np.sum(gk * dk))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("kappa", trial, fd, ad)
