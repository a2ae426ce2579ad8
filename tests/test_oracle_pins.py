"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here goes through a route other than the oracle's own formulas:
closed-form integrals, a different quadrature with a numerically inverted
Jacobian, the paper's printed 2D mass matrix and column sparsity pattern,
conservation and constant-preservation identities, closed forms of the IIPG
operator on fields it reproduces exactly, the Taylor form of SSP-RK3 on a
linear operator, and convergence orders against exact solutions.
"""

import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_matrix(name):
    rows = [l.split() for l in open(os.path.join(GOLD, name)) if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=np.float64)


def _mesh(w):
    return O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)


def _single_column_mesh(xy, ztop, zbot):
    """One triangle (CCW vertices xy (3,2)) extruded into one prism."""
    zlev = np.stack([ztop, zbot])
    return O.PrismMesh(np.asarray(xy, float), np.array([[0, 1, 2]]), np.array([[-1, -1, -1]]),
                       np.array([1]), zlev)


# ---------------------------------------------------------------------------
# quadrature and basis
# ---------------------------------------------------------------------------

def test_triangle_rule_exact_to_degree_4():
    for i in range(5):
        for j in range(5 - i):
            exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            q = np.sum(O.TRI_W * O.TRI_PTS[:, 0] ** i * O.TRI_PTS[:, 1] ** j)
            assert abs(q - exact) < 1e-16, (i, j, q, exact)
    # and not exact at degree 5 (it is the degree-4 rule, not a higher one)
    q = np.sum(O.TRI_W * O.TRI_PTS[:, 0] ** 5)
    assert abs(q - math.factorial(5) / math.factorial(7)) > 1e-6


def test_gauss_rules():
    for d in range(4):
        exact = (1 - (-1) ** (d + 1)) / (d + 1)
        assert abs(np.sum(O.GL2_W * O.GL2_PTS ** d) - exact) < 1e-15
    for d in range(6):
        assert abs(np.sum(O.GL3_W * O.GL3_PTS ** d) - 1.0 / (d + 1)) < 1e-15


def test_basis_partition_and_nodality():
    nodes = [(0, 0, 1), (1, 0, 1), (0, 1, 1), (0, 0, -1), (1, 0, -1), (0, 1, -1)]
    for j, (xi, eta, zeta) in enumerate(nodes):
        phi = O.reference_basis(xi, eta, zeta)[0]
        assert np.allclose(phi, np.eye(6)[j], atol=0, rtol=0)
    rng = np.random.default_rng(5)
    for _ in range(10):
        xi, eta = rng.dirichlet([1, 1, 1])[:2]
        zeta = rng.uniform(-1, 1)
        phi, dxi, deta, dzeta = O.reference_basis(xi, eta, zeta)
        assert abs(phi.sum() - 1) < 1e-15
        assert abs(dxi.sum()) < 1e-15 and abs(deta.sum()) < 1e-15 and abs(dzeta.sum()) < 1e-15


# ---------------------------------------------------------------------------
# mass matrix
# ---------------------------------------------------------------------------

def test_flat_prism_mass_is_paper_mh_times_vertical():
    Mh_over = _load_matrix("mass_2d.txt")          # 24 M_h / J_h (paper, section 2.3)
    xy = np.array([[0.0, 0.0], [3.0, 0.5], [1.0, 2.0]])
    Jh = (xy[1, 0] - xy[0, 0]) * (xy[2, 1] - xy[0, 1]) - (xy[2, 0] - xy[0, 0]) * (xy[1, 1] - xy[0, 1])
    dz = 2.5
    m = _single_column_mesh(xy, np.full(3, -1.0), np.full(3, -1.0 - dz))
    M = O.mass_matrix(m)[0]
    Mh = Jh / 24.0 * Mh_over
    expect = np.kron(dz / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]]), Mh)
    assert np.allclose(M, expect, rtol=1e-14, atol=0)


def _bary_integral(a, b, c):
    """int over the reference triangle of l0^a l1^b l2^c = a! b! c! / (a+b+c+2)!"""
    f = math.factorial
    return f(a) * f(b) * f(c) / f(a + b + c + 2)


def test_sloped_prism_mass_closed_form():
    rng = np.random.default_rng(11)
    xy = np.array([[0.0, 0.0], [2.0, 0.3], [0.4, 1.7]])
    ztop = rng.uniform(-0.2, 0.2, 3)
    zbot = ztop - rng.uniform(0.5, 3.0, 3)
    m = _single_column_mesh(xy, ztop, zbot)
    M = O.mass_matrix(m)[0]
    Jh = (xy[1, 0] - xy[0, 0]) * (xy[2, 1] - xy[0, 1]) - (xy[2, 0] - xy[0, 0]) * (xy[1, 1] - xy[0, 1])
    dz = ztop - zbot
    H = np.array([[2.0, 1.0], [1.0, 2.0]]) / 3.0    # int (1+-z)/2 (1+-z)/2 dz over [-1, 1]
    Mz = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                e = [0, 0, 0]
                e[a] += 1
                e[b] += 1
                e[c] += 1
                Mz[a, b] += Jh * 0.5 * dz[c] * _bary_integral(*e)
    assert np.allclose(M, np.kron(H, Mz), rtol=1e-14, atol=0)
    vol = 0.5 * Jh * dz.mean()                      # triangle area x mean height
    assert abs(M.sum() - vol) < 1e-14 * vol


# ---------------------------------------------------------------------------
# residual terms against an independent quadrature and Jacobian route
# ---------------------------------------------------------------------------

def _duffy_rule(n=8):
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1)
    w = 0.5 * w
    pts, wts = [], []
    for u, wu in zip(g, w):
        for v, wv in zip(g, w):
            pts.append((u, v * (1 - u)))
            wts.append(wu * wv * (1 - u))
    return np.array(pts), np.array(wts)


def _phys(mesh, p, xi, eta, zeta):
    phi, dxi, deta, dzeta = O.reference_basis(xi, eta, zeta)
    xn = np.concatenate([mesh.X[p], mesh.X[p]])
    yn = np.concatenate([mesh.Y[p], mesh.Y[p]])
    zn = np.concatenate([mesh.ZT[p], mesh.ZB[p]])
    J = np.array([[xn @ dxi, xn @ deta, xn @ dzeta],
                  [yn @ dxi, yn @ deta, yn @ dzeta],
                  [zn @ dxi, zn @ deta, zn @ dzeta]])
    return np.array([xn @ phi, yn @ phi, zn @ phi]), J, phi, np.stack([dxi, deta, dzeta])


def _independent_volume(mesh, U, T, p):
    pts, wts = _duffy_rule()
    g, gw = np.polynomial.legendre.leggauss(4)
    R = np.zeros((T.shape[0], 6))
    for (xi, eta), wt in zip(pts, wts):
        for zeta, wz in zip(g, gw):
            _, J, phi, dref = _phys(mesh, p, xi, eta, zeta)
            grad = np.linalg.solve(J.T, dref)          # physical gradients (3, 6)
            Uq = U[:, :, p] @ phi
            Tq = T[:, :, p] @ phi
            R += wt * wz * abs(np.linalg.det(J)) * Tq[:, None] * (Uq @ grad)[None]
    return R


def test_volume_term_matches_independent_quadrature():
    w = W.tiny(n_fields=2)
    m = _mesh(w)
    rng = np.random.default_rng(3)
    assert np.ptp(m.ZB, axis=1).max() > 0.1        # sigma levels over the bump: sloped prisms
    U = rng.standard_normal((3, 6, m.P))
    T = rng.standard_normal((2, 6, m.P))
    got = O.volume_term(m, U, T, np.arange(m.P))
    for p in range(m.P):
        ref = _independent_volume(m, U, T, p)
        assert np.allclose(got[:, :, p], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), p


def _independent_faces_single_prism(mesh, U, T, t_ext):
    """All faces of a lone prism (every face open) by a tensor Gauss rule with
    normals from the cross product of the face parametrisation's tangents."""
    p = 0
    g, gw = np.polynomial.legendre.leggauss(6)
    s_pts, s_w = 0.5 * (g + 1), 0.5 * gw
    out = np.zeros((T.shape[0], 6))
    centroid = np.array([mesh.X[p].mean(), mesh.Y[p].mean(),
                         0.5 * (mesh.ZT[p].mean() + mesh.ZB[p].mean())])

    def add(xi, eta, zeta, dX1, dX2, wgt):
        x, J, phi, _ = _phys(mesh, p, xi, eta, zeta)
        nds = np.cross(dX1, dX2)
        if np.dot(nds, x - centroid) < 0:
            nds = -nds
        un = (U[:, :, p] @ phi) @ nds
        tin = T[:, :, p] @ phi
        fl = np.where(un > 0, un * tin, un * np.asarray(t_ext))
        out[:] += wgt * fl[:, None] * phi[None]

    for k in range(3):
        a, b = k, (k + 1) % 3
        for s, ws in zip(s_pts, s_w):
            lam = np.zeros(3)
            lam[a], lam[b] = 1 - s, s
            dlam = np.zeros(3)
            dlam[a], dlam[b] = -1, 1
            for zeta, wz in zip(g, gw):
                _, J, _, _ = _phys(mesh, p, lam[1], lam[2], zeta)
                dX_ds = J[:, 0] * dlam[1] + J[:, 1] * dlam[2]
                add(lam[1], lam[2], zeta, dX_ds, J[:, 2], ws * wz)
    pts, wts = _duffy_rule()
    for zeta in (1.0, -1.0):
        for (xi, eta), wt in zip(pts, wts):
            _, J, _, _ = _phys(mesh, p, xi, eta, zeta)
            add(xi, eta, zeta, J[:, 0], J[:, 1], wt)
    return out


def test_face_terms_lone_prism_match_independent_route():
    rng = np.random.default_rng(7)
    xy = np.array([[0.0, 0.0], [2.0, 0.3], [0.4, 1.7]])
    ztop = rng.uniform(-0.3, 0.3, 3)
    zbot = ztop - rng.uniform(0.5, 2.0, 3)
    m = _single_column_mesh(xy, ztop, zbot)
    T = rng.standard_normal((2, 6, 1))
    t_ext = np.array([0.3, -1.2])
    for trial in range(4):
        # constant velocity: u.n has one sign on every planar face
        U = np.repeat(rng.standard_normal((3, 1, 1)), 6, axis=1)
        got = (O.lateral_flux_term(m, U, T, t_ext, [0]) + O.horizontal_flux_term(m, U, T, t_ext, [0]))[:, :, 0]
        ref = _independent_faces_single_prism(m, U, T, t_ext)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), trial


def _locate(mesh, p, x):
    """Reference coordinates of physical point x inside prism p (independent inversion)."""
    X, Y = mesh.X[p], mesh.Y[p]
    A = np.array([[X[1] - X[0], X[2] - X[0]], [Y[1] - Y[0], Y[2] - Y[0]]])
    xi, eta = np.linalg.solve(A, x[:2] - np.array([X[0], Y[0]]))
    lam = np.array([1 - xi - eta, xi, eta])
    zt, zb = lam @ mesh.ZT[p], lam @ mesh.ZB[p]
    zeta = (2 * x[2] - zt - zb) / (zt - zb)
    return xi, eta, zeta


def test_interior_faces_match_point_location():
    """Two columns x two layers: interior lateral and horizontal faces evaluated
    by locating each physical quadrature point in the neighbour."""
    w = W.tiny(n=1, n_layers=2, n_fields=1)
    m = _mesh(w)
    rng = np.random.default_rng(9)
    T = rng.standard_normal((1, 6, m.P))
    U = np.repeat(rng.standard_normal((3, 1, 1)), 6, axis=1)
    U = np.repeat(U, m.P, axis=2)
    t_ext = np.array([0.7])
    got = O.lateral_flux_term(m, U, T, t_ext, np.arange(m.P)) + O.horizontal_flux_term(m, U, T, t_ext, np.arange(m.P))
    g, gw = np.polynomial.legendre.leggauss(6)
    s_pts, s_w = 0.5 * (g + 1), 0.5 * gw
    pts, wts = _duffy_rule()
    for p in range(m.P):
        c, l = m.col[p], m.lay[p]
        ref = np.zeros(6)
        cen = np.array([m.X[p].mean(), m.Y[p].mean(), 0.5 * (m.ZT[p].mean() + m.ZB[p].mean())])

        def flux(xi, eta, zeta, nds, other, wgt):
            x, J, phi, _ = _phys(m, p, xi, eta, zeta)
            if np.dot(nds, x - cen) < 0:
                nds = -nds
            un = U[:, 0, p] @ nds
            tin = T[0, :, p] @ phi
            if other is None:
                tout = t_ext[0]
            else:
                phi2 = O.reference_basis(*_locate(m, other, x))[0]
                tout = T[0, :, other] @ phi2
            return wgt * (un * tin if un > 0 else un * tout) * phi

        for k in range(3):
            a, b = k, (k + 1) % 3
            c2 = m.nbr[c, k]
            other = None if c2 < 0 else m.off[c2] + l
            for s, ws in zip(s_pts, s_w):
                lam = np.zeros(3)
                lam[a], lam[b] = 1 - s, s
                dlam = np.zeros(3)
                dlam[a], dlam[b] = -1, 1
                for zeta, wz in zip(g, gw):
                    _, J, _, _ = _phys(m, p, lam[1], lam[2], zeta)
                    ref += flux(lam[1], lam[2], zeta, np.cross(J[:, 0] * dlam[1] + J[:, 1] * dlam[2], J[:, 2]), other, ws * wz)
        for zeta, other in ((1.0, p - 1 if l > 0 else None), (-1.0, p + 1 if l < m.nl[c] - 1 else None)):
            for (xi, eta), wt in zip(pts, wts):
                _, J, _, _ = _phys(m, p, xi, eta, zeta)
                ref += flux(xi, eta, zeta, np.cross(J[:, 0], J[:, 1]), other, wt)
        assert np.allclose(got[0, :, p], ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max()), p


# ---------------------------------------------------------------------------
# conservation and consistency identities
# ---------------------------------------------------------------------------

def test_constant_preservation_solid_body_rotation():
    w = W.rotating_blob(n=6, n_layers=3)
    m = _mesh(w)
    c = 3.7
    T = np.full((1, 6, m.P), c)
    R = O.advective_residual(m, w.U, T, [c])
    scale = np.abs(O.volume_term(m, w.U, T, np.arange(m.P))).max()
    assert np.abs(R).max() < 1e-13 * scale


def test_budget_identity_one_step():
    w = W.rotating_blob(n=6, n_layers=4)
    m = _mesh(w)
    Tn1, (T1, T2, _) = O.step(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, return_stages=True)
    dm = O.mass(m, Tn1) - O.mass(m, w.T0)
    B = [O.boundary_flux(m, w.U, X, w.t_ext) for X in (w.T0, T1, T2)]
    pred = -w.dt * (B[0] / 6 + B[1] / 6 + 2 * B[2] / 3)
    assert np.abs(dm - pred).max() < 1e-12 * np.abs(O.mass(m, w.T0)).max()


def _closed_flow(n=8, n_layers=3, seed=0, U0=200.0):
    """psi_h = P1 interpolant of sin(pi x/L) sin(pi y/L); U = U0 (d psi_h/dy,
    -d psi_h/dx, 0) per triangle; sigma layers over h = 20 + 10 psi_h."""
    w = W.rotating_blob(seed=seed, n=n, n_layers=n_layers)
    L = W.prism_mesh.DOMAIN_L
    psi = np.sin(np.pi * w.vxy[:, 0] / L) * np.sin(np.pi * w.vxy[:, 1] / L)
    p = w.vxy[w.tri]
    ps = psi[w.tri]
    # gradient of the linear interpolant on each triangle
    A = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]], axis=1)       # (C, 2, 2)
    rhs = np.stack([ps[:, 1] - ps[:, 0], ps[:, 2] - ps[:, 0]], axis=1)
    grad = np.linalg.solve(A, rhs[..., None])[..., 0]                   # (C, 2)
    ucol = U0 * np.stack([grad[:, 1], -grad[:, 0], np.zeros(len(grad))])
    col = np.repeat(np.arange(w.n_cols), w.nlayers)
    U = np.repeat(ucol[:, None, col], 6, axis=1)
    return w, U


def test_closed_flow_conserves_mass_and_constants():
    w, U = _closed_flow()
    m = _mesh(w)
    T = w.T0 + 0.3 * np.random.default_rng(1).standard_normal(w.T0.shape)
    assert np.abs(O.boundary_flux(m, U, T, [5.0])).max() < 1e-12 * np.abs(O.mass(m, T)).max() / w.dt
    c = 2.0
    R = O.advective_residual(m, U, np.full_like(T, c), [123.0])   # t_ext irrelevant: no boundary flux
    scale = np.abs(O.volume_term(m, U, np.full_like(T, c), np.arange(m.P))).max()
    assert np.abs(R).max() < 1e-13 * scale
    m0 = O.mass(m, T)
    X = T
    for _ in range(3):
        X = O.step(m, U, w.kappa, X, w.dt, [5.0])
    assert abs(O.mass(m, X)[0] - m0[0]) < 1e-13 * abs(m0[0])


# ---------------------------------------------------------------------------
# vertical diffusion operator (IIPG)
# ---------------------------------------------------------------------------

def _column_mesh(n_layers=3, sloped=True, seed=2):
    w = W.tiny(n=1, n_layers=n_layers)
    if sloped:
        return _mesh(w), w
    nl = w.nlayers
    zl = np.concatenate([np.repeat((-np.arange(n + 1) * 2.0)[:, None], 3, 1) for n in nl])
    return O.PrismMesh(w.vxy, w.tri, w.nbr, nl, zl), w


def test_column_sparsity_matches_paper_picture():
    pattern = _load_matrix("column_sparsity_3layer.txt")
    m, w = _column_mesh(3)
    K, _ = O.column_system(m, np.array([1e-2, 3e-3, 1e-3]), 50.0, 0)
    for r in range(6):                   # half-blocks of 3 rows
        for q in range(3):               # prisms
            blk = K[3 * r:3 * r + 3, 6 * q:6 * q + 6]
            if pattern[r, q]:
                assert np.all(blk != 0.0), (r, q)
            else:
                assert np.all(blk == 0.0), (r, q)


def test_iipg_annihilates_constants_and_conserves():
    m, w = _column_mesh(5)
    kappa = np.geomspace(1e-2, 1e-5, 5)
    for c in range(m.C):
        A = O.vertical_diffusion_matrix(m, kappa, c)
        s = np.abs(A).max()
        assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-14 * s
        assert np.abs(np.ones(A.shape[0]) @ A).max() < 1e-14 * s


def test_iipg_on_linear_profile_closed_form():
    """T = z is in the P1 space with dT/dz = 1: A z equals the face terms
    (kappa_above - kappa_below)/2 * J_h/6 at interface nodes, -kappa_0 J_h/6 at
    surface nodes and +kappa_{N-1} J_h/6 at bottom nodes (J_h/6 = rows of M_h)."""
    m, w = _column_mesh(4, sloped=True)
    kappa = np.array([3e-2, 1e-2, 4e-3, 1e-3])
    for c in range(m.C):
        N = int(m.nl[c])
        ps = m.off[c] + np.arange(N)
        z = np.concatenate([np.concatenate([m.ZT[p], m.ZB[p]]) for p in ps])
        A = O.vertical_diffusion_matrix(m, kappa, c)
        X, Y = m.X[ps[0]], m.Y[ps[0]]
        Jh = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0])
        expect = np.zeros(6 * N)
        expect[0:3] = -kappa[0] * Jh / 6
        expect[6 * N - 3:] = kappa[N - 1] * Jh / 6
        for l in range(1, N):
            d = 0.5 * (kappa[l - 1] - kappa[l]) * Jh / 6
            expect[6 * (l - 1) + 3:6 * (l - 1) + 6] += d
            expect[6 * l:6 * l + 3] += d
        assert np.allclose(A @ z, expect, rtol=1e-12, atol=1e-14 * np.abs(expect).max())


def test_iipg_penalty_on_layer_indicator():
    """T = 1 on prism l only: dT/dz = 0 everywhere, jumps -1 above and +1 below,
    so A T = +-sigma J_h/6 at the four half-layers touching the two faces."""
    m, w = _column_mesh(4, sloped=True)
    kappa = np.array([3e-2, 1e-2, 4e-3, 1e-3])
    eta = 4.0
    c, N = 0, 4
    ps = m.off[c] + np.arange(N)
    hbar = (m.ZT[ps] - m.ZB[ps]).mean(axis=1)
    X, Y = m.X[ps[0]], m.Y[ps[0]]
    Jh = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0])
    A = O.vertical_diffusion_matrix(m, kappa, c, eta)
    l = 2
    T = np.zeros(6 * N)
    T[6 * l:6 * l + 6] = 1.0
    sig_up = eta * 0.5 * (kappa[l - 1] + kappa[l]) / min(hbar[l - 1], hbar[l])
    sig_dn = eta * 0.5 * (kappa[l] + kappa[l + 1]) / min(hbar[l], hbar[l + 1])
    expect = np.zeros(6 * N)
    expect[6 * (l - 1) + 3:6 * (l - 1) + 6] = sig_up * Jh / 6     # bottom of the prism above
    expect[6 * l:6 * l + 3] = -sig_up * Jh / 6                      # top of prism l
    expect[6 * l + 3:6 * l + 6] = -sig_dn * Jh / 6                  # bottom of prism l
    expect[6 * (l + 1):6 * (l + 1) + 3] = sig_dn * Jh / 6           # top of the prism below
    assert np.allclose(A @ T, expect, rtol=1e-12, atol=1e-14 * np.abs(expect).max())


def test_implicit_solve_satisfies_system():
    w = W.tiny(n_fields=2)
    m = _mesh(w)
    rng = np.random.default_rng(4)
    Ts = rng.standard_normal((2, 6, m.P))
    X = O.implicit_solve(m, w.kappa, 300.0, Ts)
    for c in range(m.C):
        ps = m.off[c] + np.arange(m.nl[c])
        K, Mc = O.column_system(m, w.kappa, 300.0, c)
        x = X[:, :, ps].transpose(2, 1, 0).reshape(-1, 2)
        b = Ts[:, :, ps].transpose(2, 1, 0).reshape(-1, 2)
        assert np.abs(K @ x - Mc @ b).max() < 1e-12 * np.abs(Mc @ b).max()


# ---------------------------------------------------------------------------
# time integration
# ---------------------------------------------------------------------------

def test_ssp_rk3_is_third_order_taylor_on_linear_operator():
    w = W.tiny(n_fields=1)
    m = _mesh(w)
    n = 6 * m.P
    t_ext = [0.0]                                   # makes L linear
    Lmat = np.zeros((n, n))
    for j in range(n):
        e = np.zeros((1, 6, m.P))
        e.reshape(-1)[j] = 1.0
        Lmat[:, j] = O.explicit_operator(m, w.U, e, t_ext).reshape(-1)
    T = w.T0
    T1 = O.rk_stage(m, w.U, 0, T, T, w.dt, t_ext)
    T2 = O.rk_stage(m, w.U, 1, T, T1, w.dt, t_ext)
    T3 = O.rk_stage(m, w.U, 2, T, T2, w.dt, t_ext)
    A = w.dt * Lmat
    P3 = np.eye(n) + A + A @ A / 2 + A @ A @ A / 6
    ref = P3 @ T.reshape(-1)
    assert np.allclose(T3.reshape(-1), ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_whole_step_is_dense_composition():
    """The matrix-free step equals S P(dt L) x on the tiny mesh (linear with
    zero exterior values), with P the SSP-RK3 polynomial of the assembled L
    and S = (M - dt A)^-1 M assembled from the column systems: the Lie
    splitting order (three stages, then the solve) and both parts together."""
    w = W.tiny(n_fields=1)
    m = _mesh(w)
    n = 6 * m.P
    t_ext = [0.0]
    dt = 5.0 * w.dt
    Lmat = np.zeros((n, n))
    for j in range(n):
        e = np.zeros((1, 6, m.P))
        e.reshape(-1)[j] = 1.0
        Lmat[:, j] = O.explicit_operator(m, w.U, e, t_ext).reshape(-1)
    A = dt * Lmat
    P3 = np.eye(n) + A + A @ A / 2 + A @ A @ A / 6
    # S column by column: unknowns of the state vector are (node, prism)
    S = np.zeros((n, n))
    for c in range(m.C):
        K, Mc = O.column_system(m, w.kappa, dt, c)
        ps = m.off[c] + np.arange(m.nl[c])
        idx = (np.arange(6)[None, :] * m.P + ps[:, None]).ravel()      # column order (layer, node)
        S[np.ix_(idx, idx)] = np.linalg.solve(K, Mc)
    ref = S @ (P3 @ w.T0.reshape(-1))
    got = O.step(m, w.U, w.kappa, w.T0, dt, t_ext, w.penalty).reshape(-1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def _l2_error_vs(mesh, T, exact_fn):
    """sqrt(int (T_h - T_exact)^2) with the 12-point rule."""
    err = 0.0
    Jh = ((mesh.X[:, 1] - mesh.X[:, 0]) * (mesh.Y[:, 2] - mesh.Y[:, 0])
          - (mesh.X[:, 2] - mesh.X[:, 0]) * (mesh.Y[:, 1] - mesh.Y[:, 0]))
    zn = np.concatenate([mesh.ZT, mesh.ZB], axis=1)
    xn = np.concatenate([mesh.X, mesh.X], axis=1)
    yn = np.concatenate([mesh.Y, mesh.Y], axis=1)
    for (xi, eta), wt in zip(O.TRI_PTS, O.TRI_W):
        for zeta, wz in zip(O.GL2_PTS, O.GL2_W):
            phi, _, _, dzeta = O.reference_basis(xi, eta, zeta)
            d = T[0].T @ phi - exact_fn(xn @ phi, yn @ phi, zn @ phi)
            err += np.sum(wt * wz * Jh * (zn @ dzeta) * d * d)
    return math.sqrt(err)


@pytest.mark.slow
def test_advection_convergence_order():
    L = W.prism_mesh.DOMAIN_L
    om = W.prism_mesh.rotation_rate()
    # centred 1.5 km from the rotation centre: >= 4.3 sigma from the open
    # boundary, so the exterior value 0 is exact to ~1e-4
    sig, cx, cy = 800.0, 6500.0, 5000.0

    def blob(x, y, t):
        c, s = math.cos(om * t), math.sin(om * t)
        x0 = L / 2 + c * (cx - L / 2) - s * (cy - L / 2)
        y0 = L / 2 + s * (cx - L / 2) + c * (cy - L / 2)
        return np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / (2 * sig ** 2))

    t_end = (math.pi / 4) / om
    errs = []
    for n in (16, 32, 64):
        vxy, tri, nbr = W.square_mesh(n, jitter=0.0)
        nl, zl = W.sigma_levels(vxy, tri, 1, depth_fn=lambda x, y: 20.0 + 0 * x)
        x, y, z = W.prism_mesh.prism_node_xyz(vxy, tri, nl, zl)
        U = W.solid_body_velocity(x, y)
        m = O.PrismMesh(vxy, tri, nbr, nl, zl)
        nsteps = int(math.ceil(t_end / W.cfl_dt(vxy, tri, U)))
        dt = t_end / nsteps
        T = blob(x, y, 0.0)[None]
        for _ in range(nsteps):
            T = O.step(m, U, np.zeros(1), T, dt, [0.0])
        errs.append(_l2_error_vs(m, T, lambda X, Y, Z: blob(X, Y, t_end)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] >= 1.8, (errs, rates)


@pytest.mark.slow
def test_diffusion_convergence_order():
    H, kap = 20.0, 1e-2
    t_end = 0.1 * H * H / (kap * math.pi ** 2)

    def exact(z, t):
        return 1.0 + np.cos(np.pi * z / H) * math.exp(-kap * math.pi ** 2 * t / H ** 2)

    errs = []
    for N in (4, 8, 16):
        vxy, tri, nbr = W.square_mesh(1, jitter=0.0)
        nl, zl = W.sigma_levels(vxy, tri, N, depth_fn=lambda x, y: H + 0 * x)
        x, y, z = W.prism_mesh.prism_node_xyz(vxy, tri, nl, zl)
        m = O.PrismMesh(vxy, tri, nbr, nl, zl)
        U = np.zeros((3, 6, m.P))
        nsteps = 4 * N * N
        dt = t_end / nsteps
        T = exact(z, 0.0)[None]
        for _ in range(nsteps):
            T = O.step(m, U, np.full(N, kap), T, dt, [0.0])
        errs.append(_l2_error_vs(m, T, lambda X, Y, Z: exact(Z, t_end)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) >= 1.8, (errs, rates)
