"""Horizontal tracer diffusion with the Okubo diffusivity (the paper's section
1.1: the diffusivity tensor is split into horizontal and vertical parts, the
horizontal diffusivity follows Okubo's model; section 2: horizontal terms are
explicit), dense FP64 quadrature.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper leaves the discretisation to its supporting document; the reading
taken here:

* the operator acts along the layers: derivatives at constant zeta (grad_z,
  the horizontal map's chain rule without the zeta term), i.e.
  (1/z_zeta) div_z (z_zeta kappa_h grad_z T); on flat layers this is
  div_h(kappa_h grad_h T);
* symmetric interior penalty on the lateral faces, for the own test function
  phi_i of a prism K:

    D_i = - int_K kh grad_z T . grad_z phi_i dV
          + sum_faces int ( {kh grad_z T}.n phi_i
                            + 1/2 kh_K (grad_z phi_i . n) [T]
                            - sigma [T] phi_i ) dS

  (D = -a(T, phi) for the symmetric bilinear form a);

  with [T] = T_K - T_neighbour, {v} the mean of both sides,
  sigma = eta (kh_K + kh_K')/2 / min(J_h,K / |e|, J_h,K' / |e|);
* zero diffusive flux through open lateral boundaries and z-level walls;
* kh per column from Okubo's relation K = 0.0103 l^1.15 (cm^2/s, l in cm),
  i.e. 2.055e-4 l^1.15 m^2/s with l in metres, l = sqrt(J_h) (the leg of the
  right isosceles triangle of the same area), times a scale.

Volume integrals use the 12-point prism rule, face integrals 3 x 2 Gauss
points; both are exact for these polynomial integrands.
"""

from __future__ import annotations

import numpy as np

from .prism_dg import GL2_PTS, GL2_W, GL3_PTS, GL3_W, TRI_PTS, TRI_W, PrismMesh, _horizontal_map, reference_basis

OKUBO_COEF = 0.0103 * 100.0 ** 1.15 / 1.0e4    # m^0.85 / s


def okubo_diffusivity(mesh: PrismMesh, scale: float = 1.0):
    """kh per column = scale * OKUBO_COEF * sqrt(J_h)^1.15 [m^2/s]."""
    p = mesh.vxy[mesh.tri]
    Jh = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    return scale * OKUBO_COEF * np.sqrt(Jh) ** 1.15


def _along_layer_grad(xi_x, xi_y, eta_x, eta_y, dxi, deta):
    """(n, 6) x- and y-derivatives at constant zeta of the 6 basis functions."""
    gx = np.outer(xi_x, dxi) + np.outer(eta_x, deta)
    gy = np.outer(xi_y, dxi) + np.outer(eta_y, deta)
    return gx, gy


def horizontal_diffusion_term(mesh: PrismMesh, kappa_h, T, eta=4.0, prisms=None):
    """D(T) of shape (F, 6, n) for the selected prisms (all by default)."""
    sel = mesh.all_prisms() if prisms is None else np.asarray(prisms)
    T = np.asarray(T, dtype=np.float64)
    kh_col = np.asarray(kappa_h, dtype=np.float64)
    n = len(sel)
    col, lay = mesh.col[sel], mesh.lay[sel]
    X, Y, ZT, ZB = mesh.X[sel], mesh.Y[sel], mesh.ZT[sel], mesh.ZB[sel]
    zn = np.concatenate([ZT, ZB], axis=1)
    Jh, xi_x, xi_y, eta_x, eta_y = _horizontal_map(X, Y)
    kh = kh_col[col]
    Ts = T[:, :, sel]
    out = np.zeros((T.shape[0], 6, n))

    # volume: - int kh grad_z T . grad_z phi_i  J_h z_zeta
    for (xi, et), wt in zip(TRI_PTS, TRI_W):
        for zeta, wz in zip(GL2_PTS, GL2_W):
            _, dxi, deta, dzeta = reference_basis(xi, et, zeta)
            z_zeta = zn @ dzeta
            gx, gy = _along_layer_grad(xi_x, xi_y, eta_x, eta_y, dxi, deta)       # (n, 6)
            Tx = np.einsum("fin,ni->fn", Ts, gx)
            Ty = np.einsum("fin,ni->fn", Ts, gy)
            w = wt * wz * Jh * z_zeta * kh                                         # (n,)
            out -= w[None, None, :] * (Tx[:, None, :] * gx.T[None] + Ty[:, None, :] * gy.T[None])

    # lateral faces
    rows = np.arange(n)
    for k in range(3):
        a, b = k, (k + 1) % 3
        dx, dy = X[:, b] - X[:, a], Y[:, b] - Y[:, a]
        Le = np.hypot(dx, dy)
        nx, ny = dy / Le, -dx / Le
        dz_a, dz_b = ZT[:, a] - ZB[:, a], ZT[:, b] - ZB[:, b]
        c2 = mesh.nbr[col, k]
        interior = c2 >= 0
        c2s = np.where(interior, c2, 0)
        live = interior & (lay < mesh.nl[c2s])
        if not live.any():
            continue
        k2 = np.where(interior, mesh.nbr_edge[col, k], 0)
        p2 = np.where(live, mesh.off[c2s] + lay, 0)
        X2, Y2 = mesh.X[p2], mesh.Y[p2]
        Jh2, xi_x2, xi_y2, eta_x2, eta_y2 = _horizontal_map(X2, Y2)
        kh2 = kh_col[c2s]
        T2 = T[:, :, p2]
        sigma = eta * 0.5 * (kh + kh2) / np.minimum(Jh / Le, Jh2 / Le)
        for s, ws in zip(GL3_PTS, GL3_W):
            lam = np.zeros(3)
            lam[a], lam[b] = 1.0 - s, s
            lam2 = np.zeros((n, 3))
            lam2[rows, k2] = s
            lam2[rows, (k2 + 1) % 3] = 1.0 - s
            for zeta, wz in zip(GL2_PTS, GL2_W):
                phi_in, dxi, deta, _ = reference_basis(lam[1], lam[2], zeta)
                gx, gy = _along_layer_grad(xi_x, xi_y, eta_x, eta_y, dxi, deta)     # own basis gradients
                phi_out = np.concatenate([lam2 * 0.5 * (1 + zeta), lam2 * 0.5 * (1 - zeta)], axis=1)
                _, dxi2, deta2, _ = reference_basis(lam2[0, 1], lam2[0, 2], zeta)   # gradients are constant in (xi, eta)
                gx2, gy2 = _along_layer_grad(xi_x2, xi_y2, eta_x2, eta_y2, dxi2, deta2)
                tin = np.einsum("fin,i->fn", Ts, phi_in)
                tout = np.einsum("fin,ni->fn", T2, phi_out)
                gn_in = np.einsum("fin,ni->fn", Ts, gx * nx[:, None] + gy * ny[:, None])
                gn_out = np.einsum("fin,ni->fn", T2, gx2 * nx[:, None] + gy2 * ny[:, None])
                jump = tin - tout
                avg = 0.5 * (kh * gn_in + kh2 * gn_out)
                dS = ws * wz * Le * 0.5 * ((1.0 - s) * dz_a + s * dz_b)
                dS = np.where(live, dS, 0.0)
                dphin = (gx * nx[:, None] + gy * ny[:, None])                      # (n, 6)
                out += dS[None, None, :] * (
                    phi_in[None, :, None] * (avg - sigma[None, :] * jump)[:, None, :]
                    + 0.5 * kh[None, None, :] * dphin.T[None] * jump[:, None, :])
    return out


def horizontal_diffusion_matrix(mesh: PrismMesh, kappa_h, eta=4.0, chunk=512):
    """D (6P x 6P), degrees of freedom numbered 6 p + i (prism p, node i),
    assembled column by column from the matrix-free term applied to unit
    vectors; practical on small meshes only."""
    import scipy.sparse as sp
    n = 6 * mesh.P
    cols = []
    for d0 in range(0, n, chunk):
        d = np.arange(d0, min(n, d0 + chunk))
        E = np.zeros((len(d), 6, mesh.P))
        E[np.arange(len(d)), d % 6, d // 6] = 1.0
        out = horizontal_diffusion_term(mesh, kappa_h, E, eta)       # (k, 6, P)
        cols.append(sp.csr_matrix(out.transpose(0, 2, 1).reshape(len(d), n)))
    return sp.vstack(cols).T.tocsr()
