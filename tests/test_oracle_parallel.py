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
