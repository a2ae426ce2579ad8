"""The process-parallel evaluation of the oracle's steps (used for the
full-size comparisons) gives the sequential oracle's result: the work splits
over prisms and columns without changing any prism's or column's arithmetic.
NumPy's vectorised loops may round differently on arrays of other lengths
(fused or unfused multiply-adds in their tails), so agreement is to 1e-14 of
each field's maximum rather than bitwise."""

import numpy as np
import pytest

import oracle as O
import oracle.parallel as OP
import workloads as W
from oracle.split_imex import imex_step


@pytest.mark.parametrize("scheme", ["lie", "imex"])
def test_parallel_steps_equal_sequential(scheme, monkeypatch):
    monkeypatch.setattr(OP, "_PRISM_CHUNK", 37)       # many uneven ranges
    monkeypatch.setattr(OP, "_COLUMN_CHUNK", 5)
    w = W.ragged(n=5, n_fields=2)
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    got = OP.run_steps(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, 2, scheme, w.penalty, workers=3)
    ref = w.T0
    for _ in range(2):
        ref = (O.step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty) if scheme == "lie"
               else imex_step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty))
    err = np.abs(got - ref).reshape(2, -1).max(axis=1) / np.abs(ref).reshape(2, -1).max(axis=1)
    assert np.all(err <= 1e-14), err


def test_parallel_states_feed_the_adjoint(monkeypatch):
    """run_steps(states=True) returns every state x^0 .. x^N, and the
    oracle's gradient computed from them equals the one that runs its own
    forward steps (to 1e-13: the stiff column systems, kappa dt / dz^2 up to
    ~80, magnify the different rounding of the vectorised loops)."""
    import oracle.adjoint as OA
    monkeypatch.setattr(OP, "_PRISM_CHUNK", 41)
    monkeypatch.setattr(OP, "_COLUMN_CHUNK", 4)
    w = W.ragged(n=4, n_fields=1)
    w.kappa = w.kappa * 300.0
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    xs = OP.run_steps(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, 3, "lie", w.penalty, workers=2, states=True)
    assert len(xs) == 4 and np.array_equal(xs[0], w.T0)
    seq = OA.forward(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, 3, w.penalty)
    for a, b in zip(xs, seq):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    J, gT, gk, ga = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, 3, w.penalty, return_scale=True, xs=xs)
    J2, gT2, gk2, ga2 = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, 3, w.penalty, return_scale=True)
    assert abs(J - J2) <= 1e-14 * J
    assert np.abs(gT - gT2).max() <= 1e-13 * np.abs(gT2).max()
    assert np.all(np.abs(gk - gk2) <= 1e-13 * ga2)
    with pytest.raises(ValueError):
        OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, 3, w.penalty, xs=xs[:3])
