"""Pins of the oracle's upwind face flux where the velocity is discontinuous
between prisms and its normal component changes sign inside a face.

The flux reading (section 1.1 tracer equation, upwind flux): at every face
quadrature point F = u_n T_up, with u_n the normal component of the average of
the two velocity traces and T_up the trace on the side u_n leaves.  With a
velocity constant over the mesh, or continuous and linear, averaging the two
traces and taking the inner one coincide and every planar face has one upwind
side, so the other pins cannot tell those readings apart.  Here:

* an independent route evaluates the face integrals at the rule's reference
  points, with normals and measures from cross products of the face tangents
  and the neighbour's traces found by inverting the neighbour's map at the
  physical point;
* a budget identity with a discontinuous velocity: mass changes only through
  the open boundary when both sides of every interior face use one u_n;
* two plausible mistakes are planted in the oracle (upwind side chosen once per
  face; u_n from the inner trace only) and each is caught.
"""

import contextlib

import numpy as np

import oracle as O
import oracle.prism_dg as P
import workloads as W


def _mesh(w):
    return O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)


def _phys(mesh, p, xi, eta, zeta):
    """Physical point and Jacobian d(x, y, z)/d(xi, eta, zeta) of prism p."""
    phi, dxi, deta, dzeta = O.reference_basis(xi, eta, zeta)
    xn = np.concatenate([mesh.X[p], mesh.X[p]])
    yn = np.concatenate([mesh.Y[p], mesh.Y[p]])
    zn = np.concatenate([mesh.ZT[p], mesh.ZB[p]])
    J = np.array([[xn @ dxi, xn @ deta, xn @ dzeta],
                  [yn @ dxi, yn @ deta, yn @ dzeta],
                  [zn @ dxi, zn @ deta, zn @ dzeta]])
    return np.array([xn @ phi, yn @ phi, zn @ phi]), J, phi


def _locate(mesh, p, x):
    """Reference coordinates of the physical point x in prism p: invert the
    affine horizontal map, then the linear vertical one."""
    X, Y = mesh.X[p], mesh.Y[p]
    A = np.array([[X[1] - X[0], X[2] - X[0]], [Y[1] - Y[0], Y[2] - Y[0]]])
    xi, eta = np.linalg.solve(A, x[:2] - np.array([X[0], Y[0]]))
    lam = np.array([1 - xi - eta, xi, eta])
    zt, zb = lam @ mesh.ZT[p], lam @ mesh.ZB[p]
    return xi, eta, (2 * x[2] - zt - zb) / (zt - zb)


def _independent_face_terms(mesh, U, T, t_ext):
    """sum over the faces of prism p of int phi_i F dS, (F, 6, P), with
    F = u_n T_in where u_n > 0 and u_n T_out elsewhere, point by point.

    The points are the rule's (3 x 2 on a lateral face, the 6-point triangle
    rule on a horizontal face): with a sign change inside a face the integrand
    is not polynomial and the rule defines the integral.  Also returns the
    number of faces whose u_n takes both signs."""
    n_f = T.shape[0]
    out = np.zeros((n_f, 6, mesh.P))
    mixed = 0
    for p in range(mesh.P):
        c, l = mesh.col[p], mesh.lay[p]
        cen = np.array([mesh.X[p].mean(), mesh.Y[p].mean(), 0.5 * (mesh.ZT[p].mean() + mesh.ZB[p].mean())])
        faces = []
        for k in range(3):
            a, b = k, (k + 1) % 3
            c2 = mesh.nbr[c, k]
            other = None if c2 < 0 else mesh.off[c2] + l
            if c2 >= 0 and l >= mesh.nl[c2]:
                continue                       # z-level step: wall, no flux
            pts = []
            for s, ws in zip(O.GL3_PTS, O.GL3_W):
                lam = np.zeros(3)
                lam[a], lam[b] = 1 - s, s
                dlam = np.zeros(3)
                dlam[a], dlam[b] = -1, 1
                for zeta, wz in zip(O.GL2_PTS, O.GL2_W):
                    _, J, _ = _phys(mesh, p, lam[1], lam[2], zeta)
                    t_s = J[:, 0] * dlam[1] + J[:, 1] * dlam[2]
                    pts.append((lam[1], lam[2], zeta, np.cross(t_s, J[:, 2]), ws * wz))
            faces.append((pts, other))
        for zeta, other in ((1.0, p - 1 if l > 0 else None), (-1.0, p + 1 if l < mesh.nl[c] - 1 else None)):
            pts = []
            for (xi, eta), wt in zip(O.TRI_PTS, O.TRI_W):
                _, J, _ = _phys(mesh, p, xi, eta, zeta)
                pts.append((xi, eta, zeta, np.cross(J[:, 0], J[:, 1]), wt))
            faces.append((pts, other))
        for pts, other in faces:
            signs = set()
            for xi, eta, zeta, nds, wgt in pts:
                x, _, phi = _phys(mesh, p, xi, eta, zeta)
                if np.dot(nds, x - cen) < 0:
                    nds = -nds                 # outward
                u_in = U[:, :, p] @ phi
                t_in = T[:, :, p] @ phi
                if other is None:
                    u_out, t_out = u_in, np.asarray(t_ext, dtype=float)
                else:
                    phi2 = O.reference_basis(*_locate(mesh, other, x))[0]
                    u_out, t_out = U[:, :, other] @ phi2, T[:, :, other] @ phi2
                un_dS = 0.5 * (u_in + u_out) @ nds        # u_n times the area element
                signs.add(un_dS > 0)
                fl = un_dS * (t_in if un_dS > 0 else t_out)
                out[:, :, p] += wgt * fl[:, None] * phi[None, :]
            mixed += len(signs) == 2
    return out, mixed


def _face_terms(mesh, U, T, t_ext):
    sel = np.arange(mesh.P)
    return P.lateral_flux_term(mesh, U, T, t_ext, sel) + P.horizontal_flux_term(mesh, U, T, t_ext, sel)


def _rel_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


# --- the three pins, each returning its error over its tolerance ------------

def _lone_prism_pin():
    """One open prism with a random P1 velocity (every face open, so u_n is
    the inner trace's and changes sign inside faces)."""
    rng = np.random.default_rng(11)
    xy = np.array([[0.0, 0.0], [2.0, 0.3], [0.4, 1.7]])
    ztop = rng.uniform(-0.3, 0.3, 3)
    zbot = ztop - rng.uniform(0.5, 2.0, 3)
    m = O.PrismMesh(xy, np.array([[0, 1, 2]]), np.array([[-1, -1, -1]]), np.array([1]), np.stack([ztop, zbot]))
    U = rng.standard_normal((3, 6, 1))
    T = rng.standard_normal((2, 6, 1))
    t_ext = np.array([0.3, -1.2])
    ref, mixed = _independent_face_terms(m, U, T, t_ext)
    assert mixed >= 2, mixed
    return _rel_err(_face_terms(m, U, T, t_ext), ref) / 1e-12


def _discontinuous_mesh_pin(w, seed):
    """Every prism its own random P1 velocity: discontinuous across every
    interior face, so {U}.n differs from either trace's normal component."""
    m = _mesh(w)
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((3, 6, m.P))
    T = rng.standard_normal((2, 6, m.P))
    t_ext = np.array([0.7, -0.4])
    ref, mixed = _independent_face_terms(m, U, T, t_ext)
    assert mixed >= 10, mixed
    return _rel_err(_face_terms(m, U, T, t_ext), ref) / 1e-12


def _budget_pin(w, seed):
    """m(T^{n+1}) - m(T^n) = -dt [B(T^n)/6 + B(T^1)/6 + 2 B(T^2)/3] with a
    discontinuous random velocity (the vertical solve adds nothing: 1^T A = 0).
    Interior face fluxes cancel only if both sides use the same u_n."""
    m = _mesh(w)
    rng = np.random.default_rng(seed)
    U = 0.3 * rng.standard_normal((3, 6, m.P))
    T0 = 1.0 + rng.standard_normal((1, 6, m.P))
    t_ext = np.array([0.5])
    # a step the explicit stages keep bounded (the identity itself holds for
    # any dt, but round-off scales with the stage values)
    dt = 0.2 * (m.ZT - m.ZB).mean(axis=1).min() / np.abs(U).max()
    Tn1, (T1, T2, _) = O.step(m, U, w.kappa, T0, dt, t_ext, return_stages=True)
    dm = O.mass(m, Tn1) - O.mass(m, T0)
    B = [O.boundary_flux(m, U, X, t_ext) for X in (T0, T1, T2)]
    pred = -dt * (B[0] / 6 + B[1] / 6 + 2 * B[2] / 3)
    assert np.abs(pred).max() > 1e-4 * np.abs(O.mass(m, T0)).max()    # the boundary moves mass
    return float(np.abs(dm - pred).max() / (1e-12 * np.abs(O.mass(m, T0)).max()))


def _tiny():
    return W.tiny(n=2, n_layers=3)


def _ragged():
    return W.ragged(n=3, n_fields=1)


def test_lone_prism_sign_changing_velocity():
    assert _lone_prism_pin() <= 1.0


def test_discontinuous_velocity_point_location_sigma():
    assert _discontinuous_mesh_pin(_tiny(), 5) <= 1.0


def test_discontinuous_velocity_point_location_zlevel_walls():
    w = _ragged()
    assert (w.nlayers.min() < w.nlayers.max())
    assert _discontinuous_mesh_pin(w, 6) <= 1.0


def test_budget_identity_discontinuous_velocity():
    assert _budget_pin(W.rotating_blob(n=5, n_layers=3), 8) <= 1.0
    assert _budget_pin(_ragged(), 9) <= 1.0


# --- planted mistakes --------------------------------------------------------

@contextlib.contextmanager
def _inner_trace_plant():
    """u_n taken from the inner velocity trace alone."""
    orig = P._mean_trace
    P._mean_trace = lambda uin, uout: uin
    try:
        yield
    finally:
        P._mean_trace = orig


@contextlib.contextmanager
def _per_face_upwind_plant():
    """Upwind side chosen once per face, from the sign of the face's summed
    u_n, instead of at every quadrature point.  Each face-term call runs twice:
    the first pass records u_n at every point (calls come face by face in a
    fixed order), the second applies each face's one sign."""
    orig_up, orig_lat, orig_hor = P._upwind, P.lateral_flux_term, P.horizontal_flux_term

    def two_pass(fn, face_of_call):
        def wrapped(*args, **kw):
            rec = []

            def record(un, tin, tout):
                rec.append(np.array(un))
                return orig_up(un, tin, tout)

            P._upwind = record
            try:
                fn(*args, **kw)
            finally:
                P._upwind = orig_up
            groups = {}
            for i, un in enumerate(rec):
                groups.setdefault(face_of_call(i), []).append(un)
            sign = {f: np.sum(v, axis=0) > 0 for f, v in groups.items()}
            calls = iter(range(len(rec)))

            def apply(un, tin, tout):
                up = sign[face_of_call(next(calls))]
                return un * np.where(up, tin, tout)

            P._upwind = apply
            try:
                return fn(*args, **kw)
            finally:
                P._upwind = orig_up
        return wrapped

    # lateral: 3 faces x (3 x 2) points, face-major; horizontal: top and
    # bottom alternate at each of the 6 triangle points
    P.lateral_flux_term = two_pass(orig_lat, lambda i: i // 6)
    P.horizontal_flux_term = two_pass(orig_hor, lambda i: i % 2)
    try:
        yield
    finally:
        P.lateral_flux_term, P.horizontal_flux_term = orig_lat, orig_hor


def test_planted_mistakes_are_caught():
    pins = {
        "lone prism": _lone_prism_pin,
        "sigma mesh": lambda: _discontinuous_mesh_pin(_tiny(), 5),
        "z-level mesh": lambda: _discontinuous_mesh_pin(_ragged(), 6),
        "budget": lambda: _budget_pin(W.rotating_blob(n=5, n_layers=3), 8),
    }
    with _per_face_upwind_plant():
        caught = {k: f() > 1.0 for k, f in pins.items() if k != "budget"}
    assert caught["lone prism"] and caught["sigma mesh"] and caught["z-level mesh"], caught
    with _inner_trace_plant():
        caught = {k: f() > 1.0 for k, f in pins.items()}
    assert caught["sigma mesh"] and caught["z-level mesh"] and caught["budget"], caught
    assert not caught["lone prism"]     # on open faces the two readings agree
