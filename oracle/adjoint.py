"""Oracle of the discrete adjoint of the tracer step.

TEST INFRASTRUCTURE ONLY (tests, smoke, bench baseline), like the rest of
``oracle/``.

The step is x^{n+1} = S P(x^n) + c: P the SSP-RK3 stages of the explicit
operator L = M^-1 R (affine in x through the exterior values), S the
implicit vertical-diffusion solve (M - dt A)^-1 M.  For

    J = sqrt(sum_f x_N,f^T M x_N,f)

reverse-mode differentiation gives (the operator is linear in T apart from
the constant inflow term, and A is linear in the per-layer diffusivity):

    lambda_N = M x_N / J
    mu_n     = (M - dt A)^-T lambda_{n+1}
    lambda_n = P'^T M mu_n,   P' = I + dt L + (dt L)^2/2 + (dt L)^3/6
    dJ/dkappa_l += dt mu_n^T A_l x^{n+1},   A_l = dA/dkappa_l = A(kappa = e_l)

and dJ/dx_0 = lambda_0.  Here every operator is assembled as a sparse
matrix from the same element definitions as the matrix-free oracle (the
transposes are then library transposes), which is only practical on small
meshes.  Degrees of freedom are numbered 6 p + i (prism p, node i).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .prism_dg import (
    GL2_PTS, GL2_W, GL3_PTS, GL3_W, TRI_PTS, TRI_W, PrismMesh, _column_masses, _horizontal_map,
    mass_matrix, reference_basis, step, vertical_diffusion_matrices,
)


def _coo_add(rows, cols, vals, pr, pc, blk):
    """Add (n, 6, 6) blocks coupling prisms pr (rows) to prisms pc (columns)."""
    n = len(pr)
    i = np.arange(6)
    r = (6 * pr[:, None, None] + i[None, :, None]) + 0 * i[None, None, :]
    c = (6 * pc[:, None, None] + i[None, None, :]) + 0 * i[None, :, None]
    rows.append(r.ravel())
    cols.append(c.ravel())
    vals.append(blk.reshape(n * 36))


def advection_matrix(mesh: PrismMesh, U) -> sp.csr_matrix:
    """R_lin (6P x 6P): the advective residual with zero exterior values,
    R_lin T = R(T) - R(0), assembled element by element."""
    P = mesh.P
    sel = np.arange(P)
    X, Y, ZT, ZB = mesh.X, mesh.Y, mesh.ZT, mesh.ZB
    zn = np.concatenate([ZT, ZB], axis=1)
    Jh, xi_x, xi_y, eta_x, eta_y = _horizontal_map(X, Y)
    rows, cols, vals = [], [], []
    # volume: R_ij += int phi_j U . grad(phi_i)
    blk = np.zeros((P, 6, 6))
    for (xi, eta), wt in zip(TRI_PTS, TRI_W):
        for zeta, wz in zip(GL2_PTS, GL2_W):
            phi, dxi, deta, dzeta = reference_basis(xi, eta, zeta)
            z_xi, z_eta, z_zeta = zn @ dxi, zn @ deta, zn @ dzeta
            detJ = Jh * z_zeta
            zeta_x = -(z_xi * xi_x + z_eta * eta_x) / z_zeta
            zeta_y = -(z_xi * xi_y + z_eta * eta_y) / z_zeta
            gx = np.outer(xi_x, dxi) + np.outer(eta_x, deta) + np.outer(zeta_x, dzeta)
            gy = np.outer(xi_y, dxi) + np.outer(eta_y, deta) + np.outer(zeta_y, dzeta)
            gz = np.outer(1.0 / z_zeta, dzeta)
            Uq = np.einsum("cin,i->cn", U, phi)
            adv = Uq[0][:, None] * gx + Uq[1][:, None] * gy + Uq[2][:, None] * gz   # (P, 6) over i
            blk += (wt * wz * detJ)[:, None, None] * adv[:, :, None] * phi[None, None, :]
    _coo_add(rows, cols, vals, sel, sel, blk)
    # lateral faces: Fhat = a T_in + b T_out, a = (u_n + |u_n|)/2, b = (u_n - |u_n|)/2
    rws = np.arange(P)
    for k in range(3):
        a_, b_ = k, (k + 1) % 3
        dx = X[:, b_] - X[:, a_]
        dy = Y[:, b_] - Y[:, a_]
        Le = np.hypot(dx, dy)
        nx, ny = dy / Le, -dx / Le
        dz_a = ZT[:, a_] - ZB[:, a_]
        dz_b = ZT[:, b_] - ZB[:, b_]
        c2 = mesh.nbr[mesh.col, k]
        interior = c2 >= 0
        c2s = np.where(interior, c2, 0)
        k2 = np.where(interior, mesh.nbr_edge[mesh.col, k], 0)
        wall = interior & (mesh.lay >= mesh.nl[c2s])
        live = interior & ~wall
        p2 = np.where(live, mesh.off[c2s] + mesh.lay, 0)
        own = np.zeros((P, 6, 6))
        nbr = np.zeros((P, 6, 6))
        for s, ws in zip(GL3_PTS, GL3_W):
            lam = np.zeros(3)
            lam[a_], lam[b_] = 1.0 - s, s
            lam2 = np.zeros((P, 3))
            lam2[rws, k2] = s
            lam2[rws, (k2 + 1) % 3] = 1.0 - s
            for zeta, wz in zip(GL2_PTS, GL2_W):
                phi_in = reference_basis(lam[1], lam[2], zeta)[0]
                phi_out = np.concatenate([lam2 * 0.5 * (1 + zeta), lam2 * 0.5 * (1 - zeta)], axis=1)
                uin = np.einsum("cin,i->cn", U, phi_in)
                uout = np.where(live[None], np.einsum("cin,ni->cn", U[:, :, p2], phi_out), uin)
                un = 0.5 * ((uin[0] + uout[0]) * nx + (uin[1] + uout[1]) * ny)
                dS = ws * wz * Le * 0.5 * ((1.0 - s) * dz_a + s * dz_b)
                a = np.where(wall, 0.0, 0.5 * (un + np.abs(un)) * dS)
                b = np.where(live, 0.5 * (un - np.abs(un)) * dS, 0.0)
                own -= a[:, None, None] * phi_in[None, :, None] * phi_in[None, None, :]
                nbr -= b[:, None, None] * phi_in[None, :, None] * phi_out[:, None, :]
        _coo_add(rows, cols, vals, sel, sel, own)
        _coo_add(rows, cols, vals, sel[live], p2[live], nbr[live])
    # horizontal faces
    zt_x = (ZT[:, 1] - ZT[:, 0]) * xi_x + (ZT[:, 2] - ZT[:, 0]) * eta_x
    zt_y = (ZT[:, 1] - ZT[:, 0]) * xi_y + (ZT[:, 2] - ZT[:, 0]) * eta_y
    zb_x = (ZB[:, 1] - ZB[:, 0]) * xi_x + (ZB[:, 2] - ZB[:, 0]) * eta_x
    zb_y = (ZB[:, 1] - ZB[:, 0]) * xi_y + (ZB[:, 2] - ZB[:, 0]) * eta_y
    has_above = mesh.lay > 0
    has_below = mesh.lay < mesh.nl[mesh.col] - 1
    pa = np.where(has_above, sel - 1, 0)
    pb = np.where(has_below, sel + 1, 0)
    for zeta_in, zeta_out, gx_, gy_, sgn, has, pn in ((1.0, -1.0, zt_x, zt_y, 1.0, has_above, pa),
                                                      (-1.0, 1.0, zb_x, zb_y, -1.0, has_below, pb)):
        own = np.zeros((P, 6, 6))
        nbr = np.zeros((P, 6, 6))
        for (xi, eta), wt in zip(TRI_PTS, TRI_W):
            phi_in = reference_basis(xi, eta, zeta_in)[0]
            phi_out = reference_basis(xi, eta, zeta_out)[0]
            uin = np.einsum("cin,i->cn", U, phi_in)
            uout = np.where(has[None], np.einsum("cin,i->cn", U[:, :, pn], phi_out), uin)
            ub = 0.5 * (uin + uout)
            un = sgn * (ub[2] - ub[0] * gx_ - ub[1] * gy_) * Jh * wt
            a = 0.5 * (un + np.abs(un))
            b = np.where(has, 0.5 * (un - np.abs(un)), 0.0)
            own -= a[:, None, None] * np.outer(phi_in, phi_in)[None]
            nbr -= b[:, None, None] * np.outer(phi_in, phi_out)[None]
        _coo_add(rows, cols, vals, sel, sel, own)
        _coo_add(rows, cols, vals, sel[has], pn[has], nbr[has])
    R = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(6 * P, 6 * P))
    return R.tocsr()


def mass_matrix_global(mesh: PrismMesh) -> sp.csr_matrix:
    """Block-diagonal M (6P x 6P)."""
    Mp = mass_matrix(mesh)
    return sp.block_diag(list(Mp), format="csr")


def mass_inverse_global(mesh: PrismMesh) -> sp.csr_matrix:
    """Block-diagonal M^-1 (6P x 6P): each prism's 6x6 mass block inverted."""
    return sp.block_diag(list(np.linalg.inv(mass_matrix(mesh))), format="csr")


def vertical_matrix_global(mesh: PrismMesh, kappa, eta=4.0) -> sp.csr_matrix:
    """Vertical diffusion A (6P x 6P) assembled column by column."""
    P = mesh.P
    A = sp.lil_matrix((6 * P, 6 * P))
    for N in np.unique(mesh.nl):
        cols = np.nonzero(mesh.nl == N)[0]
        blocks = vertical_diffusion_matrices(mesh, kappa, cols, eta)
        for c, B in zip(cols, blocks):
            d0 = 6 * mesh.off[c]
            A[d0:d0 + 6 * N, d0:d0 + 6 * N] = B
    return A.tocsr()


def _flat(T):
    """(F, 6, P) -> (6P, F) with DOF 6 p + i."""
    return T.transpose(2, 1, 0).reshape(-1, T.shape[0])


def _unflat(x, F):
    return x.reshape(-1, 6, F).transpose(2, 1, 0)


def objective(mesh: PrismMesh, T) -> float:
    """J = sqrt(sum_f T_f^T M T_f)."""
    M = mass_matrix_global(mesh)
    x = _flat(T)
    return float(np.sqrt(np.sum(x * (M @ x))))


def forward(mesh, U, kappa, T0, dt, t_ext, n_steps, eta=4.0, kappa_h=None):
    """States x^0 .. x^N of the matrix-free oracle step."""
    xs = [np.array(T0, dtype=np.float64)]
    for _ in range(n_steps):
        xs.append(step(mesh, U, kappa, xs[-1], dt, t_ext, eta, kappa_h=kappa_h))
    return xs


def gradient(mesh: PrismMesh, U, kappa, T0, dt, t_ext, n_steps, eta=4.0, kappa_h=None, return_scale=False,
             xs=None):
    """(J, dJ/dT0 of shape (F, 6, P), dJ/dkappa of shape (len(kappa),)).
    With per-column kappa_h the explicit operator also holds the horizontal
    diffusion matrix D (linear, so it adds D to R_lin).

    With return_scale, also the size of the sum behind each dJ/dkappa_l:
    sum_n dt |mu_n|^T |A_l| |x^{n+1}|, the sum of its terms' magnitudes, which
    bounds how far rounding in the terms can move the (cancelling) total.

    xs: the forward states x^0 .. x^N when the caller has them already (from
    ``forward`` or from ``parallel.run_steps(..., states=True)``, which
    evaluates the same step); otherwise ``forward`` computes them."""
    kappa = np.asarray(kappa, dtype=np.float64)
    F = T0.shape[0]
    if xs is None:
        xs = forward(mesh, U, kappa, T0, dt, t_ext, n_steps, eta, kappa_h)
    if len(xs) != n_steps + 1:
        raise ValueError("xs must hold the n_steps + 1 states x^0 .. x^N")
    M = mass_matrix_global(mesh)
    R = advection_matrix(mesh, U)
    if kappa_h is not None:
        from .horizontal_diffusion import horizontal_diffusion_matrix
        R = (R + horizontal_diffusion_matrix(mesh, kappa_h, eta)).tocsr()
    Minv_R = (mass_inverse_global(mesh) @ R).tocsr()     # L = M^-1 R, M block-diagonal
    Lt = Minv_R.T.tocsr()                                   # L^T
    A = vertical_matrix_global(mesh, kappa, eta)
    K_T = spla.splu((M - dt * A).T.tocsc())               # factored once, solved every step
    A_l = []
    for l in range(len(kappa)):
        e = np.zeros_like(kappa)
        e[l] = 1.0
        A_l.append(vertical_matrix_global(mesh, e, eta))
    absA_l = [abs(a) for a in A_l] if return_scale else None
    xN = _flat(xs[-1])
    J = float(np.sqrt(np.sum(xN * (M @ xN))))
    lam = (M @ xN) / J
    dk = np.zeros_like(kappa)
    dk_abs = np.zeros_like(kappa)
    for n in range(n_steps - 1, -1, -1):
        mu = K_T.solve(lam).reshape(lam.shape)
        x1 = _flat(xs[n + 1])
        for l in range(len(kappa)):
            dk[l] += dt * np.sum(mu * (A_l[l] @ x1))
            if return_scale:
                dk_abs[l] += dt * np.sum(np.abs(mu) * (absA_l[l] @ np.abs(x1)))
        y = M @ mu
        # P'^T y = y + dt L^T y + (dt L^T)^2 y / 2 + (dt L^T)^3 y / 6
        t1 = dt * (Lt @ y)
        t2 = dt * (Lt @ t1) / 2.0
        t3 = dt * (Lt @ t2) / 3.0
        lam = y + t1 + t2 + t3
    if return_scale:
        return J, _unflat(lam, F), dk, dk_abs
    return J, _unflat(lam, F), dk


def objective_after_steps(mesh, U, kappa, T0, dt, t_ext, n_steps, eta=4.0) -> float:
    return objective(mesh, forward(mesh, U, kappa, T0, dt, t_ext, n_steps, eta)[-1])


def gradient_imex(mesh: PrismMesh, U, kappa, T0, dt, t_ext, n_steps, eta=4.0, kappa_h=None, return_scale=False):
    """(J, dJ/dT0, dJ/dkappa) for n_steps of the split-IMEX step
    (``split_imex.imex_step``), by reverse-mode differentiation of its two
    steps with h = dt/2 and G = M^-1 (R + A):

        x_h = (M - h A)^-1 (M x + h R x + h c),   x' = x + dt G x_h

        mu      = (M - h A)^-T dt (R + A)^T M^-1 lambda'
        lambda  = lambda' + (M + h R)^T mu
        dJ/dkappa_l += dt lambda'^T M^-1 A_l x_h + h mu^T A_l x_h

    with the same assembled operators as ``gradient`` (R includes the
    horizontal diffusion matrix when kappa_h is given).  return_scale adds the
    sums of the kappa terms' magnitudes, as in ``gradient``."""
    from .split_imex import imex_step
    kappa = np.asarray(kappa, dtype=np.float64)
    F = T0.shape[0]
    h = 0.5 * dt
    xs, xh = [np.array(T0, dtype=np.float64)], []
    for _ in range(n_steps):
        x1, th = imex_step(mesh, U, kappa, xs[-1], dt, t_ext, eta, return_half=True, kappa_h=kappa_h)
        xs.append(x1)
        xh.append(th)
    M = mass_matrix_global(mesh).tocsc()
    R = advection_matrix(mesh, U)
    if kappa_h is not None:
        from .horizontal_diffusion import horizontal_diffusion_matrix
        R = (R + horizontal_diffusion_matrix(mesh, kappa_h, eta)).tocsr()
    A = vertical_matrix_global(mesh, kappa, eta)
    Kh_T = (M - h * A).T.tocsc()
    RA_T = (R + A).T.tocsr()
    MhR_T = (M + h * R).T.tocsr()
    A_l = []
    for l in range(len(kappa)):
        e = np.zeros_like(kappa)
        e[l] = 1.0
        A_l.append(vertical_matrix_global(mesh, e, eta))
    xN = _flat(xs[-1])
    J = float(np.sqrt(np.sum(xN * (M @ xN))))
    lam = (M @ xN) / J
    dk = np.zeros_like(kappa)
    dk_abs = np.zeros_like(kappa)
    for n in range(n_steps - 1, -1, -1):
        Minv_lam = spla.spsolve(M, lam).reshape(lam.shape)
        mu = spla.spsolve(Kh_T, dt * (RA_T @ Minv_lam)).reshape(lam.shape)
        x_h = _flat(xh[n])
        for l in range(len(kappa)):
            Ax = A_l[l] @ x_h
            dk[l] += dt * np.sum(Minv_lam * Ax) + h * np.sum(mu * Ax)
            if return_scale:
                aAx = abs(A_l[l]) @ np.abs(x_h)
                dk_abs[l] += dt * np.sum(np.abs(Minv_lam) * aAx) + h * np.sum(np.abs(mu) * aAx)
        lam = lam + MhR_T @ mu
    if return_scale:
        return J, _unflat(lam, F), dk, dk_abs
    return J, _unflat(lam, F), dk
