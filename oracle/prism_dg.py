"""Plain FP64 oracle of the nodal-P1 DG tracer operator on extruded prisms.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s ``cpu_baseline`` leg, never by the product path.  It is
written for a reader checking it against the paper by eye: straightforward
NumPy over prisms, loops over quadrature points, faces and layers, dense
per-column solves.  Nothing is blocked, fused or reordered.

What it computes (paper: section 1.1, tracer equation; section 2.2, the
stage equations and their explicit variant; section 2.4, the vertically
implicit column systems):

    dT/dt + div_h(u T) + d(wT)/dz = d/dz(kappa dT/dz)

discretised with linear Lagrange prisms obtained by extruding a triangle mesh
(section 1, mesh figure).  The supporting information that spells out the
discretisation is not part of the paper text, so the oracle fixes a textbook
nodal-P1 DG scheme that reproduces every formula the paper does print:

* nodes: three on the top face then three on the bottom face (the r_i /
  r_{i+3} split of Algorithm 1);
* the 2D mass matrix M_h = J_h/24 [2 1 1; 1 2 1; 1 1 2] (section 2.3) -- a
  flat prism's mass matrix is M_h (x) (dz/6)[2 1; 1 2];
* the column matrix M - dt A has the sparsity drawn in section 2.4 (top three
  nodes of a prism couple to the six nodes of the prism above, bottom three
  to the six below), which is the incomplete interior-penalty (IIPG) form of
  the vertical diffusion flux;
* the explicit update is element-local through the block-diagonal M
  (section 2.2, explicit variant).

Readings where the paper is silent (listed in the design notes): upwind flux
per quadrature point with u_n the average of the two velocity traces; open
boundaries with a per-field exterior value; z-level steps are walls; SSP-RK3
for the explicit stages followed by one backward-Euler vertical diffusion
solve (Lie splitting); IIPG penalty sigma = eta * mean(kappa) / min(hbar);
kappa constant per layer; quadrature rules below.
"""

from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Quadrature rules (part of the operator definition)
# ---------------------------------------------------------------------------
# Symmetric 6-point degree-4 triangle rule (Dunavant 1985) on the reference
# triangle {xi, eta >= 0, xi + eta <= 1}; weights sum to the area 1/2.
_DA1 = 0.44594849091596488631832925388305199
_DW1 = 0.22338158967801146569500700843312280
_DA2 = 0.091576213509770743459571463402201508
_DW2 = 0.10995174365532186763832632490021053


def _orbit(a):
    b = 1.0 - 2.0 * a
    return [(a, a), (a, b), (b, a)]


TRI_PTS = np.array(_orbit(_DA1) + _orbit(_DA2), dtype=np.float64)
TRI_W = 0.5 * np.array([_DW1] * 3 + [_DW2] * 3, dtype=np.float64)

# 2-point Gauss-Legendre on [-1, 1] (vertical reference coordinate zeta).
GL2_PTS = np.array([-1.0 / math.sqrt(3.0), 1.0 / math.sqrt(3.0)])
GL2_W = np.array([1.0, 1.0])

# 3-point Gauss-Legendre on [0, 1] (edge parameter s).
GL3_PTS = np.array([0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)])
GL3_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])

_CHUNK = 1 << 16


# ---------------------------------------------------------------------------
# Reference prism
# ---------------------------------------------------------------------------

def reference_basis(xi, eta, zeta):
    """Values and reference derivatives of the six P1 prism basis functions.

    lambda = (1 - xi - eta, xi, eta); zeta = +1 on the top face.
    phi_a = lambda_a (1+zeta)/2 (top nodes a = 0,1,2),
    phi_{a+3} = lambda_a (1-zeta)/2 (bottom nodes), the node order of
    Algorithm 1.  Returns phi, dphi/dxi, dphi/deta, dphi/dzeta, each (6,).
    """
    lam = np.array([1.0 - xi - eta, xi, eta])
    dlam_dxi = np.array([-1.0, 1.0, 0.0])
    dlam_deta = np.array([-1.0, 0.0, 1.0])
    top = 0.5 * (1.0 + zeta)
    bot = 0.5 * (1.0 - zeta)
    phi = np.concatenate([lam * top, lam * bot])
    dxi = np.concatenate([dlam_dxi * top, dlam_dxi * bot])
    deta = np.concatenate([dlam_deta * top, dlam_deta * bot])
    dzeta = np.concatenate([0.5 * lam, -0.5 * lam])
    return phi, dxi, deta, dzeta


# ---------------------------------------------------------------------------
# Mesh view (natural prism order: column by column, layers top to bottom)
# ---------------------------------------------------------------------------

class PrismMesh:
    """The oracle's own view of an extruded mesh.

    vxy (n_vert, 2); tri (C, 3) CCW; nbr (C, 3) with edge k = (v_k, v_{k+1})
    and -1 on the boundary; nlayers (C,); zlev (sum(nlayers+1), 3) levels per
    column, top first.  Prism q = off[c] + l.
    """

    def __init__(self, vxy, tri, nbr, nlayers, zlev):
        self.vxy = np.asarray(vxy, dtype=np.float64)
        self.tri = np.asarray(tri, dtype=np.int64)
        self.nbr = np.asarray(nbr, dtype=np.int64)
        self.nl = np.asarray(nlayers, dtype=np.int64)
        zlev = np.asarray(zlev, dtype=np.float64)
        C = self.tri.shape[0]
        self.C = C
        self.off = np.concatenate([[0], np.cumsum(self.nl)]).astype(np.int64)
        self.P = int(self.off[-1])
        self.col = np.repeat(np.arange(C), self.nl)
        self.lay = np.arange(self.P) - self.off[self.col]
        loff = self.off[:-1] + np.arange(C)
        self.X = self.vxy[self.tri[self.col], 0]                # (P, 3)
        self.Y = self.vxy[self.tri[self.col], 1]
        self.ZT = zlev[loff[self.col] + self.lay]               # (P, 3)
        self.ZB = zlev[loff[self.col] + self.lay + 1]
        # local index of the shared edge inside the neighbour
        self.nbr_edge = np.full((C, 3), -1, dtype=np.int64)
        for c in range(C):
            for k in range(3):
                c2 = self.nbr[c, k]
                if c2 < 0:
                    continue
                a, b = self.tri[c, k], self.tri[c, (k + 1) % 3]
                for k2 in range(3):
                    if self.tri[c2, k2] == b and self.tri[c2, (k2 + 1) % 3] == a:
                        self.nbr_edge[c, k] = k2
                if self.nbr_edge[c, k] < 0:
                    raise ValueError(f"neighbour {c2} of column {c} does not share edge {k}")

    def prism(self, c, l):
        return self.off[c] + l

    def all_prisms(self):
        return np.arange(self.P)


# ---------------------------------------------------------------------------
# Geometry helpers (chain rule of the prism map)
# ---------------------------------------------------------------------------

def _horizontal_map(X, Y):
    x_xi = X[:, 1] - X[:, 0]
    x_eta = X[:, 2] - X[:, 0]
    y_xi = Y[:, 1] - Y[:, 0]
    y_eta = Y[:, 2] - Y[:, 0]
    Jh = x_xi * y_eta - x_eta * y_xi
    return Jh, y_eta / Jh, -x_eta / Jh, -y_xi / Jh, x_xi / Jh   # Jh, xi_x, xi_y, eta_x, eta_y


def _nodes(A, sel):
    return A[:, :, sel]


# ---------------------------------------------------------------------------
# Mass matrix
# ---------------------------------------------------------------------------

def mass_matrix(mesh: PrismMesh, prisms=None):
    """M_ij = int_K phi_i phi_j dV with the 12-point prism rule (exact)."""
    sel = mesh.all_prisms() if prisms is None else np.asarray(prisms)
    X, Y = mesh.X[sel], mesh.Y[sel]
    zn = np.concatenate([mesh.ZT[sel], mesh.ZB[sel]], axis=1)   # (n, 6)
    Jh = _horizontal_map(X, Y)[0]
    M = np.zeros((len(sel), 6, 6))
    for (xi, eta), wt in zip(TRI_PTS, TRI_W):
        for zeta, wz in zip(GL2_PTS, GL2_W):
            phi, _, _, dzeta = reference_basis(xi, eta, zeta)
            detJ = Jh * (zn @ dzeta)
            M += (wt * wz * detJ)[:, None, None] * np.outer(phi, phi)[None]
    return M


# ---------------------------------------------------------------------------
# Advective residual R_i(T) = int_K T U.grad(phi_i) - sum_faces int phi_i Fhat
# ---------------------------------------------------------------------------

def _upwind(un, tin, tout):
    """Fhat = 1/2 u_n (T_in + T_out) + 1/2 |u_n| (T_in - T_out), at one
    quadrature point: the upwind side is chosen point by point."""
    return 0.5 * un * (tin + tout) + 0.5 * np.abs(un) * (tin - tout)


def _mean_trace(uin, uout):
    """{U} = (U_in + U_out) / 2, the velocity whose normal component u_n the
    upwind flux uses on a face (U_out = U_in on an open boundary)."""
    return 0.5 * (uin + uout)


class _Chunk:
    """Per-prism geometry of a selection of prisms."""

    def __init__(self, mesh, U, T, sel):
        self.sel = sel
        self.X, self.Y = mesh.X[sel], mesh.Y[sel]
        self.ZT, self.ZB = mesh.ZT[sel], mesh.ZB[sel]
        self.zn = np.concatenate([self.ZT, self.ZB], axis=1)
        self.Jh, self.xi_x, self.xi_y, self.eta_x, self.eta_y = _horizontal_map(self.X, self.Y)
        self.Ts = T[:, :, sel]
        self.Us = U[:, :, sel]
        self.col = mesh.col[sel]
        self.lay = mesh.lay[sel]


def volume_term(mesh, U, T, prisms):
    """int_K T U . grad(phi_i) dV with the 12-point prism rule, (F, 6, n)."""
    g = _Chunk(mesh, U, T, np.asarray(prisms))
    R = np.zeros((T.shape[0], 6, len(g.sel)))
    for (xi, eta), wt in zip(TRI_PTS, TRI_W):
        for zeta, wz in zip(GL2_PTS, GL2_W):
            phi, dxi, deta, dzeta = reference_basis(xi, eta, zeta)
            z_xi, z_eta, z_zeta = g.zn @ dxi, g.zn @ deta, g.zn @ dzeta
            detJ = g.Jh * z_zeta
            # d(zeta)/dx at fixed (y, z): z(xi, eta, zeta) held constant
            zeta_x = -(z_xi * g.xi_x + z_eta * g.eta_x) / z_zeta
            zeta_y = -(z_xi * g.xi_y + z_eta * g.eta_y) / z_zeta
            zeta_z = 1.0 / z_zeta
            gx = np.outer(g.xi_x, dxi) + np.outer(g.eta_x, deta) + np.outer(zeta_x, dzeta)
            gy = np.outer(g.xi_y, dxi) + np.outer(g.eta_y, deta) + np.outer(zeta_y, dzeta)
            gz = np.outer(zeta_z, dzeta)
            Uq = np.einsum("cin,i->cn", g.Us, phi)                 # (3, n)
            Tq = np.einsum("fin,i->fn", g.Ts, phi)                 # (F, n)
            adv = Uq[0][:, None] * gx + Uq[1][:, None] * gy + Uq[2][:, None] * gz  # (n, 6)
            R += wt * wz * Tq[:, None, :] * (detJ[:, None] * adv).T[None]
    return R


def lateral_flux_term(mesh, U, T, t_ext, prisms):
    """sum over the 3 vertical faces of int phi_i Fhat dS, (F, 6, n).

    Face k spans edge (v_k -> v_{k+1}); outward normal (dy, -dx)/|e|;
    dS = |e| dz(s)/2 ds dzeta; the neighbour column at the same layer runs
    the edge the other way (s' = 1 - s).  No neighbour: open boundary with
    T_out = t_ext.  Neighbour with fewer layers: wall, no flux.
    """
    g = _Chunk(mesh, U, T, np.asarray(prisms))
    X, Y, ZT, ZB = g.X, g.Y, g.ZT, g.ZB
    n = len(g.sel)
    text = np.asarray(t_ext, dtype=np.float64)[:, None]
    out = np.zeros((T.shape[0], 6, n))
    rows = np.arange(n)
    for k in range(3):
        a, b = k, (k + 1) % 3
        dx = X[:, b] - X[:, a]
        dy = Y[:, b] - Y[:, a]
        Le = np.hypot(dx, dy)
        nx, ny = dy / Le, -dx / Le            # outward for a CCW triangle
        dz_a = ZT[:, a] - ZB[:, a]
        dz_b = ZT[:, b] - ZB[:, b]
        c2 = mesh.nbr[g.col, k]
        interior = c2 >= 0
        c2s = np.where(interior, c2, 0)
        k2 = np.where(interior, mesh.nbr_edge[g.col, k], 0)
        wall = interior & (g.lay >= mesh.nl[c2s])
        live = interior & ~wall
        p2 = np.where(live, mesh.off[c2s] + g.lay, 0)
        To_nodes = T[:, :, p2]
        Uo_nodes = U[:, :, p2]
        for s, ws in zip(GL3_PTS, GL3_W):
            lam = np.zeros(3)
            lam[a], lam[b] = 1.0 - s, s
            lam2 = np.zeros((n, 3))
            lam2[rows, k2] = s
            lam2[rows, (k2 + 1) % 3] = 1.0 - s
            for zeta, wz in zip(GL2_PTS, GL2_W):
                phi_in = reference_basis(lam[1], lam[2], zeta)[0]
                phi_out = np.concatenate([lam2 * 0.5 * (1 + zeta), lam2 * 0.5 * (1 - zeta)], axis=1)
                tin = np.einsum("fin,i->fn", g.Ts, phi_in)
                uin = np.einsum("cin,i->cn", g.Us, phi_in)
                tout = np.where(live[None], np.einsum("fin,ni->fn", To_nodes, phi_out), text)
                uout = np.where(live[None], np.einsum("cin,ni->cn", Uo_nodes, phi_out), uin)
                ub = _mean_trace(uin, uout)
                un = ub[0] * nx + ub[1] * ny
                dS = ws * wz * Le * 0.5 * ((1.0 - s) * dz_a + s * dz_b)
                fl = _upwind(un, tin, tout) * dS
                fl[:, wall] = 0.0
                out += phi_in[None, :, None] * fl[:, None, :]
    return out


def horizontal_flux_term(mesh, U, T, t_ext, prisms):
    """int phi_i Fhat over the top and bottom faces, (F, 6, n).

    Top face: outward normal * dS = (-dz/dx, -dz/dy, 1) J_h dxi deta, the
    neighbour is the prism above; bottom face: (dz/dx, dz/dy, -1) J_h dxi deta,
    the neighbour below.  Surface and bottom are open (T_out = t_ext).
    """
    g = _Chunk(mesh, U, T, np.asarray(prisms))
    ZT, ZB = g.ZT, g.ZB
    text = np.asarray(t_ext, dtype=np.float64)[:, None]
    out = np.zeros((T.shape[0], 6, len(g.sel)))
    zt_x = (ZT[:, 1] - ZT[:, 0]) * g.xi_x + (ZT[:, 2] - ZT[:, 0]) * g.eta_x
    zt_y = (ZT[:, 1] - ZT[:, 0]) * g.xi_y + (ZT[:, 2] - ZT[:, 0]) * g.eta_y
    zb_x = (ZB[:, 1] - ZB[:, 0]) * g.xi_x + (ZB[:, 2] - ZB[:, 0]) * g.eta_x
    zb_y = (ZB[:, 1] - ZB[:, 0]) * g.xi_y + (ZB[:, 2] - ZB[:, 0]) * g.eta_y
    has_above = g.lay > 0
    has_below = g.lay < mesh.nl[g.col] - 1
    pa = np.where(has_above, g.sel - 1, 0)
    pb = np.where(has_below, g.sel + 1, 0)
    for (xi, eta), wt in zip(TRI_PTS, TRI_W):
        phi_top = reference_basis(xi, eta, 1.0)[0]
        phi_bot = reference_basis(xi, eta, -1.0)[0]
        tin = np.einsum("fin,i->fn", g.Ts, phi_top)
        uin = np.einsum("cin,i->cn", g.Us, phi_top)
        tout = np.where(has_above[None], np.einsum("fin,i->fn", T[:, :, pa], phi_bot), text)
        uout = np.where(has_above[None], np.einsum("cin,i->cn", U[:, :, pa], phi_bot), uin)
        ub = _mean_trace(uin, uout)
        un = (ub[2] - ub[0] * zt_x - ub[1] * zt_y) * g.Jh * wt
        out += phi_top[None, :, None] * _upwind(un, tin, tout)[:, None, :]
        tin = np.einsum("fin,i->fn", g.Ts, phi_bot)
        uin = np.einsum("cin,i->cn", g.Us, phi_bot)
        tout = np.where(has_below[None], np.einsum("fin,i->fn", T[:, :, pb], phi_top), text)
        uout = np.where(has_below[None], np.einsum("cin,i->cn", U[:, :, pb], phi_top), uin)
        ub = _mean_trace(uin, uout)
        un = -(ub[2] - ub[0] * zb_x - ub[1] * zb_y) * g.Jh * wt
        out += phi_bot[None, :, None] * _upwind(un, tin, tout)[:, None, :]
    return out


def _residual_chunk(mesh, U, T, t_ext, sel):
    return (volume_term(mesh, U, T, sel)
            - lateral_flux_term(mesh, U, T, t_ext, sel)
            - horizontal_flux_term(mesh, U, T, t_ext, sel))


def advective_residual(mesh: PrismMesh, U, T, t_ext, prisms=None):
    """R(T) of shape (F, 6, n) for the selected prisms (all by default).

    U (3, 6, P) nodal velocity per prism; T (F, 6, P); t_ext (F,) exterior
    value on open boundaries.
    """
    sel = mesh.all_prisms() if prisms is None else np.asarray(prisms)
    out = np.empty((T.shape[0], 6, len(sel)))
    for i in range(0, len(sel), _CHUNK):
        out[:, :, i:i + _CHUNK] = _residual_chunk(mesh, U, T, t_ext, sel[i:i + _CHUNK])
    return out


def explicit_operator(mesh: PrismMesh, U, T, t_ext, prisms=None, kappa_h=None, eta=4.0):
    """L(T) = M^-1 R(T), element by element (block-diagonal M, section 2.2).
    With per-column horizontal diffusivities kappa_h, R also holds the
    horizontal diffusion term (``horizontal_diffusion``)."""
    sel = mesh.all_prisms() if prisms is None else np.asarray(prisms)
    out = np.empty((T.shape[0], 6, len(sel)))
    for i in range(0, len(sel), _CHUNK):
        s = sel[i:i + _CHUNK]
        R = _residual_chunk(mesh, U, T, t_ext, s)          # (F, 6, n)
        if kappa_h is not None:
            from .horizontal_diffusion import horizontal_diffusion_term
            R = R + horizontal_diffusion_term(mesh, kappa_h, T, eta, s)
        M = mass_matrix(mesh, s)                             # (n, 6, 6)
        out[:, :, i:i + _CHUNK] = np.linalg.solve(M, R.transpose(2, 1, 0)).transpose(2, 1, 0)
    return out


# SSP-RK3 in Shu-Osher form: T_out = a T^n + b (T_s + dt L(T_s)).
RK3_COEFFS = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def rk_stage(mesh: PrismMesh, U, stage, Tn, Ts, dt, t_ext, prisms=None, kappa_h=None, eta=4.0):
    """One explicit SSP-RK3 stage on the selected prisms."""
    sel = mesh.all_prisms() if prisms is None else np.asarray(prisms)
    a, b = RK3_COEFFS[stage]
    L = explicit_operator(mesh, U, Ts, t_ext, sel, kappa_h, eta)
    return a * Tn[:, :, sel] + b * (Ts[:, :, sel] + dt * L)


# ---------------------------------------------------------------------------
# Vertical diffusion (IIPG) and the implicit column solve
# ---------------------------------------------------------------------------

def vertical_diffusion_matrices(mesh: PrismMesh, kappa, cols, eta=4.0):
    """Dense A (6N x 6N) for each column in ``cols`` (all with N layers);
    unknowns ordered (layer, node).  Returns (len(cols), 6N, 6N).

    (A T)_i = - int_K kappa_K dT/dz dphi_i/dz dV
              - sum_{interior horizontal faces} int [phi_i] ({kappa dT/dz}
                + sigma_f [T]) J_h dxi deta,
    [v] = v_above - v_below, {.} the arithmetic mean, zero flux at the surface
    and the bottom, sigma_f = eta (kappa_above + kappa_below)/2 /
    min(hbar_above, hbar_below) with hbar the mean vertical edge length.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    cols = np.asarray(cols, dtype=np.int64)
    N = int(mesh.nl[cols[0]])
    if np.any(mesh.nl[cols] != N):
        raise ValueError("columns of one batch must share their layer count")
    ps = mesh.off[cols][:, None] + np.arange(N)[None, :]          # (nc, N)
    Jh = _horizontal_map(mesh.X[ps[:, 0]], mesh.Y[ps[:, 0]])[0]   # (nc,)
    zn = np.concatenate([mesh.ZT[ps], mesh.ZB[ps]], axis=2)       # (nc, N, 6)
    nc = len(cols)
    A = np.zeros((nc, 6 * N, 6 * N))
    for l in range(N):
        blk = slice(6 * l, 6 * l + 6)
        for (xi, eta_), wt in zip(TRI_PTS, TRI_W):
            for zeta, wz in zip(GL2_PTS, GL2_W):
                _, _, _, dzeta = reference_basis(xi, eta_, zeta)
                z_zeta = zn[:, l] @ dzeta                           # (nc,)
                dphi_dz = dzeta[None, :] / z_zeta[:, None]          # (nc, 6)
                A[:, blk, blk] -= (wt * wz * kappa[l] * Jh * z_zeta)[:, None, None] * \
                    dphi_dz[:, :, None] * dphi_dz[:, None, :]
    hbar = (mesh.ZT[ps] - mesh.ZB[ps]).mean(axis=2)               # (nc, N)
    for l in range(1, N):
        up, dn = l - 1, l
        sigma = eta * 0.5 * (kappa[up] + kappa[dn]) / np.minimum(hbar[:, up], hbar[:, dn])
        idx = np.r_[6 * up:6 * up + 6, 6 * dn:6 * dn + 6]
        for (xi, eta_), wt in zip(TRI_PTS, TRI_W):
            phi_up, _, _, dz_up = reference_basis(xi, eta_, -1.0)   # bottom trace of the upper prism
            phi_dn, _, _, dz_dn = reference_basis(xi, eta_, 1.0)    # top trace of the lower prism
            grad_up = dz_up[None, :] / (zn[:, up] @ dz_up)[:, None]
            grad_dn = dz_dn[None, :] / (zn[:, dn] @ dz_dn)[:, None]
            jump = np.concatenate([phi_up, -phi_dn])                # (12,)
            avg = np.concatenate([0.5 * kappa[up] * grad_up, 0.5 * kappa[dn] * grad_dn], axis=1)
            rhs = avg + sigma[:, None] * jump[None, :]              # (nc, 12)
            A[:, idx[:, None], idx[None, :]] -= (wt * Jh)[:, None, None] * jump[None, :, None] * rhs[:, None, :]
    return A


def vertical_diffusion_matrix(mesh: PrismMesh, kappa, c, eta=4.0):
    """Dense A (6N x 6N) of column c (see ``vertical_diffusion_matrices``)."""
    return vertical_diffusion_matrices(mesh, kappa, [c], eta)[0]


def _column_masses(mesh, cols):
    N = int(mesh.nl[cols[0]])
    ps = mesh.off[cols][:, None] + np.arange(N)[None, :]
    Mp = mass_matrix(mesh, ps.ravel()).reshape(len(cols), N, 6, 6)
    Mc = np.zeros((len(cols), 6 * N, 6 * N))
    for l in range(N):
        Mc[:, 6 * l:6 * l + 6, 6 * l:6 * l + 6] = Mp[:, l]
    return Mc


def column_system(mesh: PrismMesh, kappa, dt, c, eta=4.0):
    """(M - dt A, M) of column c (section 2.2, implicit system)."""
    Mc = _column_masses(mesh, np.array([c]))[0]
    return Mc - dt * vertical_diffusion_matrix(mesh, kappa, c, eta), Mc


def implicit_solve(mesh: PrismMesh, kappa, dt, Tstar, eta=4.0, columns=None, out=None):
    """Solve (M - dt A) T^{n+1} = M T* column by column with a dense solver.

    Tstar (F, 6, P).  Returns a copy with the selected columns replaced, or,
    given ``out`` (F, 6, P), writes the selected columns there and returns it.
    Columns with the same layer count are solved as one batch.
    """
    if out is None:
        out = np.array(Tstar, dtype=np.float64, copy=True)
    cols = np.arange(mesh.C) if columns is None else np.asarray(columns, dtype=np.int64)
    F = Tstar.shape[0]
    for N in np.unique(mesh.nl[cols]):
        group = cols[mesh.nl[cols] == N]
        step_c = max(1, (1 << 22) // (36 * int(N) * int(N)))
        for i in range(0, len(group), step_c):
            g = group[i:i + step_c]
            ps = mesh.off[g][:, None] + np.arange(N)[None, :]              # (nc, N)
            Mc = _column_masses(mesh, g)
            K = Mc - dt * vertical_diffusion_matrices(mesh, kappa, g, eta)
            rhs = Tstar[:, :, ps].transpose(2, 3, 1, 0).reshape(len(g), 6 * N, F)
            x = np.linalg.solve(K, Mc @ rhs)                                # (nc, 6N, F)
            out[:, :, ps] = x.reshape(len(g), N, 6, F).transpose(3, 2, 0, 1)
    return out


def step(mesh: PrismMesh, U, kappa, T, dt, t_ext, eta=4.0, return_stages=False, kappa_h=None):
    """Three SSP-RK3 stages of the explicit operator, then one implicit
    vertical-diffusion solve over dt (Lie splitting)."""
    T1 = rk_stage(mesh, U, 0, T, T, dt, t_ext, kappa_h=kappa_h, eta=eta)
    T2 = rk_stage(mesh, U, 1, T, T1, dt, t_ext, kappa_h=kappa_h, eta=eta)
    Ts = rk_stage(mesh, U, 2, T, T2, dt, t_ext, kappa_h=kappa_h, eta=eta)
    Tn1 = implicit_solve(mesh, kappa, dt, Ts, eta)
    if return_stages:
        return Tn1, (T1, T2, Ts)
    return Tn1


# ---------------------------------------------------------------------------
# Diagnostics
# ---------------------------------------------------------------------------

def mass(mesh: PrismMesh, T):
    """m_f = sum_K 1^T M_K T_K for each field."""
    out = np.zeros(T.shape[0])
    for i in range(0, mesh.P, _CHUNK):
        s = np.arange(i, min(i + _CHUNK, mesh.P))
        M = mass_matrix(mesh, s)
        out += np.einsum("nij,fjn->f", M, T[:, :, s])
    return out


def boundary_flux(mesh: PrismMesh, U, T, t_ext):
    """B(T) = sum over open boundary faces of int Fhat dS (outward positive)."""
    F = T.shape[0]
    text = np.asarray(t_ext, dtype=np.float64)[:, None]
    B = np.zeros(F)
    sel = mesh.all_prisms()
    X, Y, ZT, ZB = mesh.X, mesh.Y, mesh.ZT, mesh.ZB
    col, lay = mesh.col, mesh.lay
    Jh, xi_x, xi_y, eta_x, eta_y = _horizontal_map(X, Y)
    for k in range(3):
        bnd = mesh.nbr[col, k] < 0
        if not bnd.any():
            continue
        a, b = k, (k + 1) % 3
        s_ = sel[bnd]
        dx = X[s_, b] - X[s_, a]
        dy = Y[s_, b] - Y[s_, a]
        Le = np.hypot(dx, dy)
        nx, ny = dy / Le, -dx / Le
        dz_a = ZT[s_, a] - ZB[s_, a]
        dz_b = ZT[s_, b] - ZB[s_, b]
        for s, ws in zip(GL3_PTS, GL3_W):
            lam = np.zeros(3)
            lam[a], lam[b] = 1.0 - s, s
            for zeta, wz in zip(GL2_PTS, GL2_W):
                phi = reference_basis(lam[1], lam[2], zeta)[0]
                tin = np.einsum("fin,i->fn", T[:, :, s_], phi)
                uin = np.einsum("cin,i->cn", U[:, :, s_], phi)
                un = uin[0] * nx + uin[1] * ny
                dS = ws * wz * Le * 0.5 * ((1.0 - s) * dz_a + s * dz_b)
                B += (_upwind(un, tin, text) * dS).sum(axis=1)
    top = lay == 0
    bot = lay == mesh.nl[col] - 1
    for mask, zeta, sgn, Z in ((top, 1.0, 1.0, ZT), (bot, -1.0, -1.0, ZB)):
        s_ = sel[mask]
        z_x = (Z[s_, 1] - Z[s_, 0]) * xi_x[s_] + (Z[s_, 2] - Z[s_, 0]) * eta_x[s_]
        z_y = (Z[s_, 1] - Z[s_, 0]) * xi_y[s_] + (Z[s_, 2] - Z[s_, 0]) * eta_y[s_]
        for (xi, eta), wt in zip(TRI_PTS, TRI_W):
            phi = reference_basis(xi, eta, zeta)[0]
            tin = np.einsum("fin,i->fn", T[:, :, s_], phi)
            uin = np.einsum("cin,i->cn", U[:, :, s_], phi)
            un = sgn * (uin[2] - uin[0] * z_x - uin[1] * z_y) * Jh[s_] * wt
            B += _upwind(un, tin, text).sum(axis=1)
    return B
