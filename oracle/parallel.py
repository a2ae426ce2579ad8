"""Process-parallel evaluation of the oracle's time steps on large meshes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The explicit operator is element-local given the stage input, and the
implicit solves are independent per column, so a step's work splits over
prism ranges (the three SSP-RK3 stages, the split-IMEX residuals) and over
column ranges (the vertical solves) without changing what any prism or column
computes: each worker calls the oracle's own functions (``rk_stage``,
``implicit_solve``, the split-IMEX steps) on its range and writes the result
into shared memory.  Workers are forked after the mesh and inputs exist, so
they share them without copies; no worker may touch a GPU.
"""

from __future__ import annotations

import mmap
import multiprocessing as mp
import time

import numpy as np

from .prism_dg import PrismMesh, implicit_solve, rk_stage
from .split_imex import _residual, imex_full_step, imex_half_step

_G: dict = {}
_PRISM_CHUNK = 1 << 15
_COLUMN_CHUNK = 1 << 12


def shared_array(shape) -> np.ndarray:
    """A float64 array in anonymous shared memory (visible to forked workers)."""
    n = int(np.prod(shape))
    buf = mmap.mmap(-1, max(8 * n, 8))
    return np.frombuffer(buf, dtype=np.float64, count=n).reshape(shape)


def _stage_job(job):
    stage, tn, ts, dst, lo, hi = job
    g = _G
    sel = np.arange(lo, hi)
    g[dst][:, :, lo:hi] = rk_stage(g["mesh"], g["U"], stage, g[tn], g[ts], g["dt"], g["t_ext"], prisms=sel,
                                   kappa_h=g["kappa_h"], eta=g["eta"])
    return hi - lo


def _solve_job(job):
    src, dst, h, cols = job
    g = _G
    implicit_solve(g["mesh"], g["kappa"], h, g[src], g["eta"], columns=cols, out=g[dst])
    return len(cols)


def _residual_job(job):
    src, dst, lo, hi = job
    g = _G
    sel = np.arange(lo, hi)
    g[dst][:, :, lo:hi] = _residual(g["mesh"], g["U"], g[src], g["t_ext"], g["kappa_h"], g["eta"], sel)
    return hi - lo


def _imex_half_job(job):
    cols = job
    g = _G
    imex_half_step(g["mesh"], g["kappa"], g["X"], g["R"], g["dt"], g["eta"], g["H"], columns=cols)
    return len(cols)


def _imex_full_job(job):
    cols = job
    g = _G
    imex_full_step(g["mesh"], g["kappa"], g["X"], g["H"], g["R"], g["dt"], g["eta"], g["Y"], columns=cols)
    return len(cols)


def _prism_ranges(P):
    return [(lo, min(lo + _PRISM_CHUNK, P)) for lo in range(0, P, _PRISM_CHUNK)]


def _column_ranges(mesh):
    return [np.arange(lo, min(lo + _COLUMN_CHUNK, mesh.C)) for lo in range(0, mesh.C, _COLUMN_CHUNK)]


def run_steps(mesh: PrismMesh, U, kappa, T0, dt, t_ext, n_steps, scheme="lie", eta=4.0, kappa_h=None,
              workers=8, log=None, states=False):
    """n_steps of the oracle step ('lie': SSP-RK3 then the vertical solve,
    as ``prism_dg.step``; 'imex': ``split_imex.imex_step``) from T0 (F, 6, P),
    evaluated by ``workers`` forked processes; returns the final state, or
    with states=True the list of every state x^0 .. x^N."""
    F = T0.shape[0]
    shape = (F, 6, mesh.P)
    _G.clear()
    _G.update(mesh=mesh, U=U, kappa=np.asarray(kappa, dtype=np.float64), dt=float(dt),
              t_ext=np.asarray(t_ext, dtype=np.float64), eta=float(eta), kappa_h=kappa_h)
    names = ("X", "A", "B", "C") if scheme == "lie" else ("X", "R", "H", "Y")
    for k in names:
        _G[k] = shared_array(shape)
    _G["X"][:] = T0
    prisms = _prism_ranges(mesh.P)
    columns = _column_ranges(mesh)
    ctx = mp.get_context("fork")
    t0 = time.time()
    kept = [np.array(T0, dtype=np.float64)] if states else None
    with ctx.Pool(workers) as pool:
        for n in range(n_steps):
            if scheme == "lie":
                for stage, tn, ts, dst in ((0, "X", "X", "A"), (1, "X", "A", "B"), (2, "X", "B", "C")):
                    pool.map(_stage_job, [(stage, tn, ts, dst, lo, hi) for lo, hi in prisms], chunksize=1)
                    if log:
                        log(f"oracle step {n + 1}/{n_steps}: stage {stage} done ({time.time() - t0:.0f} s)")
                pool.map(_solve_job, [("C", "X", float(dt), c) for c in columns], chunksize=1)
            elif scheme == "imex":
                pool.map(_residual_job, [("X", "R", lo, hi) for lo, hi in prisms], chunksize=1)
                pool.map(_imex_half_job, columns, chunksize=1)
                if log:
                    log(f"oracle step {n + 1}/{n_steps}: half step done ({time.time() - t0:.0f} s)")
                pool.map(_residual_job, [("H", "R", lo, hi) for lo, hi in prisms], chunksize=1)
                pool.map(_imex_full_job, columns, chunksize=1)
                _G["X"][:] = _G["Y"]
            else:
                raise ValueError(scheme)
            if states:
                kept.append(np.array(_G["X"]))
            if log:
                log(f"oracle step {n + 1}/{n_steps} done ({time.time() - t0:.0f} s)")
    out = kept if states else np.array(_G["X"])
    _G.clear()
    return out
