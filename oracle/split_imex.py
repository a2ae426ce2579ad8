"""Two-step split-IMEX tracer step (the paper's time integration of the
internal mode: section 2, mode splitting and vertical/horizontal separation;
section 3, the two-step scheme whose first step is vertically implicit over
half a time step and whose second step is explicit; section 3.2, the step
equation M_1 x_1 = M_0 x_0 + dt (horizontal fluxes of the current Runge-Kutta
field + vertical fluxes)), dense FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

With R the advective residual and A the vertical diffusion operator of the
rest of the oracle, and a static mesh (M_0 = M_1 = M):

    step 1, vertically implicit over dt/2, from x_0 with the horizontal
            fluxes of x_0:   M x_h = M x_0 + dt/2 (R(x_0) + A x_h)
    step 2, explicit over dt, from x_0 with every flux at the step-1 field:
                             M x_1 = M x_0 + dt (R(x_h) + A x_h)

Each column system is assembled densely and solved with numpy; the explicit
step uses the block-diagonal M column by column.
"""

from __future__ import annotations

import numpy as np

from .horizontal_diffusion import horizontal_diffusion_term
from .prism_dg import PrismMesh, _column_masses, advective_residual, vertical_diffusion_matrices


def _column_groups(mesh: PrismMesh, chunk_bytes: int = 1 << 25, columns=None):
    """Columns (all, or the given ones) grouped by layer count, in chunks of
    bounded dense size."""
    cols = np.arange(mesh.C) if columns is None else np.asarray(columns, dtype=np.int64)
    for N in np.unique(mesh.nl[cols]):
        group = cols[mesh.nl[cols] == N]
        step_c = max(1, chunk_bytes // (8 * 36 * int(N) * int(N)))
        for i in range(0, len(group), step_c):
            g = group[i:i + step_c]
            yield int(N), g, mesh.off[g][:, None] + np.arange(N)[None, :]


def _to_columns(T, ps):
    """(F, 6, P) values of the prisms ps (nc, N) -> (nc, 6N, F)."""
    nc, N = ps.shape
    return T[:, :, ps].transpose(2, 3, 1, 0).reshape(nc, 6 * N, T.shape[0])


def _from_columns(x, ps, out):
    nc, N = ps.shape
    out[:, :, ps] = x.reshape(nc, N, 6, -1).transpose(3, 2, 0, 1)


def vertical_diffusion_apply(mesh: PrismMesh, kappa, T, eta=4.0):
    """A T column by column, (F, 6, P)."""
    out = np.zeros_like(np.asarray(T, dtype=np.float64))
    for _, g, ps in _column_groups(mesh):
        A = vertical_diffusion_matrices(mesh, kappa, g, eta)
        _from_columns(A @ _to_columns(T, ps), ps, out)
    return out


def _residual(mesh, U, T, t_ext, kappa_h, eta, prisms=None):
    R = advective_residual(mesh, U, T, t_ext, prisms)
    if kappa_h is not None:
        R = R + horizontal_diffusion_term(mesh, kappa_h, T, eta, prisms)
    return R


def imex_half_step(mesh: PrismMesh, kappa, T0, R0, dt, eta, out, columns=None):
    """Step 1 on the selected columns: (M - dt/2 A) x_h = M x_0 + dt/2 R(x_0),
    with R0 = R(x_0) given; x_h written into out."""
    for _, g, ps in _column_groups(mesh, columns=columns):
        Mc = _column_masses(mesh, g)
        A = vertical_diffusion_matrices(mesh, kappa, g, eta)
        rhs = Mc @ _to_columns(T0, ps) + 0.5 * dt * _to_columns(R0, ps)
        _from_columns(np.linalg.solve(Mc - 0.5 * dt * A, rhs), ps, out)
    return out


def imex_full_step(mesh: PrismMesh, kappa, T0, Th, Rh, dt, eta, out, columns=None):
    """Step 2 on the selected columns: M x_1 = M x_0 + dt (R(x_h) + A x_h),
    with Rh = R(x_h) given; x_1 written into out."""
    for _, g, ps in _column_groups(mesh, columns=columns):
        Mc = _column_masses(mesh, g)
        A = vertical_diffusion_matrices(mesh, kappa, g, eta)
        incr = np.linalg.solve(Mc, _to_columns(Rh, ps) + A @ _to_columns(Th, ps))
        _from_columns(_to_columns(T0, ps) + dt * incr, ps, out)
    return out


def imex_step(mesh: PrismMesh, U, kappa, T0, dt, t_ext, eta=4.0, return_half=False, kappa_h=None):
    """One split-IMEX step from T0 (F, 6, P); returns T1 (and x_h).  With
    per-column kappa_h, R also holds the (explicit) horizontal diffusion."""
    T0 = np.asarray(T0, dtype=np.float64)
    R0 = _residual(mesh, U, T0, t_ext, kappa_h, eta)
    Th = imex_half_step(mesh, kappa, T0, R0, dt, eta, np.empty_like(T0))
    Rh = _residual(mesh, U, Th, t_ext, kappa_h, eta)
    T1 = imex_full_step(mesh, kappa, T0, Th, Rh, dt, eta, np.empty_like(T0))
    if return_half:
        return T1, Th
    return T1
