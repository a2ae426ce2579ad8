"""Seeded synthetic meshes and inputs for the extruded-prism tracer workloads.

Everything here is input generation: vertex coordinates, triangle
connectivity, layer levels, nodal velocity samples, initial tracer values,
diffusivity per layer and the time step.  The geometric factors, mass
matrices, fluxes and solves of the method are computed by the oracle and by
the HIP library from these arrays, never here.

Conventions shared by every consumer:

* triangles are counter-clockwise; edge ``k`` of a triangle runs from its
  vertex ``k`` to vertex ``(k+1) % 3``; ``nbr[t, k]`` is the triangle on the
  other side of that edge or ``-1`` on the domain boundary;
* every triangle is extruded into a column of ``nlayers[t]`` prisms, layers
  ordered from the surface down;
* ``zlev`` concatenates, column by column, ``nlayers[t] + 1`` levels of three
  vertex heights (top level first);
* prism nodes are the three top vertices followed by the three bottom ones;
* "natural" prism order enumerates columns in triangle order and layers top to
  bottom inside each column; nodal arrays are ``[component][node][prism]``.

The workloads follow the paper's test shapes: an unstructured triangulation
extruded in sigma layers (section 2, SoA layout figure), or in z-levels with
bathymetry-dependent layer counts (sections 2.1.1 and 5, variable column
depth).  Random draws use ``numpy.random.default_rng`` (PCG64) with the seeds
stated per function.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

DOMAIN_L = 10_000.0  # square side [m]


@dataclasses.dataclass
class Workload:
    """One synthetic run: mesh, layering, velocity, fields and parameters."""

    name: str
    vxy: np.ndarray          # (n_vert, 2) float64
    tri: np.ndarray          # (C, 3) int32, CCW
    nbr: np.ndarray          # (C, 3) int32, -1 = boundary
    nlayers: np.ndarray      # (C,) int32
    zlev: np.ndarray         # (sum(nlayers+1), 3) float64
    U: np.ndarray            # (3, 6, P) float64, natural prism order
    T0: np.ndarray           # (F, 6, P) float64, natural prism order
    kappa: np.ndarray        # (max(nlayers),) float64, per layer index
    dt: float
    t_ext: np.ndarray        # (F,) float64
    penalty: float = 4.0
    w_is_zero: bool = True
    n_steps: int = 1
    member_tri_off: np.ndarray | None = None

    @property
    def n_cols(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_prisms(self) -> int:
        return int(self.nlayers.sum())

    @property
    def n_fields(self) -> int:
        return int(self.T0.shape[0])


def natural_prism_count(nlayers: np.ndarray) -> int:
    return int(np.asarray(nlayers).sum())


# ---------------------------------------------------------------------------
# 2D mesh
# ---------------------------------------------------------------------------

def hilbert_order(px: np.ndarray, py: np.ndarray, bits: int = 16) -> np.ndarray:
    """Permutation sorting points along a Hilbert curve (locality ordering of
    the 2D mesh, section 2.1).  Only the storage order depends on it."""
    n = 1 << bits
    x0, x1 = px.min(), px.max()
    y0, y1 = py.min(), py.max()
    span = max(x1 - x0, y1 - y0, 1e-300)
    x = np.minimum(((px - x0) / span * (n - 1)).astype(np.int64), n - 1)
    y = np.minimum(((py - y0) / span * (n - 1)).astype(np.int64), n - 1)
    d = np.zeros_like(x)
    s = n // 2
    while s > 0:
        rx = ((x & s) > 0).astype(np.int64)
        ry = ((y & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        flip = (ry == 0) & (rx == 1)
        x = np.where(flip, n - 1 - x, x)
        y = np.where(flip, n - 1 - y, y)
        swap = ry == 0
        x, y = np.where(swap, y, x), np.where(swap, x, y)
        s //= 2
    return np.argsort(d, kind="stable")


def triangle_neighbours(tri: np.ndarray) -> np.ndarray:
    """nbr[t, k] = triangle sharing edge (tri[t,k], tri[t,(k+1)%3]), else -1."""
    C = tri.shape[0]
    a = tri
    b = np.roll(tri, -1, axis=1)
    lo = np.minimum(a, b).ravel().astype(np.int64)
    hi = np.maximum(a, b).ravel().astype(np.int64)
    key = lo * (int(tri.max()) + 1) + hi
    owner = np.repeat(np.arange(C, dtype=np.int64), 3)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nbr = np.full(3 * C, -1, dtype=np.int64)
    same = ks[1:] == ks[:-1]
    i0 = order[:-1][same]
    i1 = order[1:][same]
    nbr[i0] = owner[i1]
    nbr[i1] = owner[i0]
    return nbr.reshape(C, 3).astype(np.int32)


def square_mesh(n: int, L: float = DOMAIN_L, jitter: float = 0.2, seed: int = 0,
                hilbert: bool = True):
    """Split-square triangulation of [0,L]^2 with n squares per side.

    Vertex (i, j) sits at (i, j) * L/n; interior vertices are displaced by
    U(-jitter, jitter) * L/n in each coordinate (rng seeded with ``seed``),
    boundary vertices stay fixed.  Each square is cut along its
    (i,j)-(i+1,j+1) diagonal into two CCW triangles.  Triangles are then put
    in Hilbert order of their centroids.  Returns (vxy, tri, nbr).
    """
    h = L / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    vid = (ii * (n + 1) + jj).astype(np.int32)
    vxy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    rng = np.random.default_rng(seed)
    disp = rng.uniform(-jitter, jitter, size=vxy.shape) * h
    interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n)).ravel()
    vxy[interior] += disp[interior]
    bl = vid[:-1, :-1].ravel()
    br = vid[1:, :-1].ravel()
    tr = vid[1:, 1:].ravel()
    tl = vid[:-1, 1:].ravel()
    tri = np.concatenate([np.stack([bl, br, tr], 1), np.stack([bl, tr, tl], 1)])
    tri = tri.astype(np.int32)
    if hilbert:
        cxy = vxy[tri].mean(axis=1)
        tri = tri[hilbert_order(cxy[:, 0], cxy[:, 1])]
    nbr = triangle_neighbours(tri)
    return vxy, tri, nbr


# ---------------------------------------------------------------------------
# layering
# ---------------------------------------------------------------------------

def bump_bathymetry(x, y, L: float = DOMAIN_L):
    """h(x, y) = 20 + 10 sin(pi x/L) sin(pi y/L) [m]."""
    return 20.0 + 10.0 * np.sin(np.pi * x / L) * np.sin(np.pi * y / L)


def sigma_levels(vxy, tri, n_layers: int, depth_fn=bump_bathymetry):
    """Uniform sigma layers: level k at vertex v is -k/N * h(v), surface 0."""
    C = tri.shape[0]
    hv = depth_fn(vxy[:, 0], vxy[:, 1])                       # (n_vert,)
    frac = np.arange(n_layers + 1, dtype=np.float64) / n_layers
    z = -frac[None, :, None] * hv[tri][:, None, :]            # (C, N+1, 3)
    nl = np.full(C, n_layers, dtype=np.int32)
    return nl, z.reshape(-1, 3).copy()


def zlevel_levels(vxy, tri, depth_c, dz: float, n_min: int, n_max: int):
    """Flat z-levels -k*dz; column t gets clamp(ceil(depth_c[t]/dz), n_min, n_max)
    layers (stair-step bottom)."""
    nl = np.clip(np.ceil(depth_c / dz), n_min, n_max).astype(np.int32)
    rows = (nl + 1).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(rows)[:-1]])
    k = np.arange(int(rows.sum()), dtype=np.int64) - np.repeat(start, rows)
    return nl, np.repeat((-dz * k.astype(np.float64))[:, None], 3, axis=1)


def prism_node_xyz(vxy, tri, nlayers, zlev):
    """Node coordinates per prism in natural order: x, y, z of shape (6, P)."""
    C = tri.shape[0]
    P = int(nlayers.sum())
    col = np.repeat(np.arange(C), nlayers)
    off = np.concatenate([[0], np.cumsum(nlayers)])
    lay = np.arange(P) - off[col]
    loff = off[:-1] + np.arange(C)               # first level row of column
    xv = vxy[tri[col], 0].T                      # (3, P)
    yv = vxy[tri[col], 1].T
    zt = zlev[loff[col] + lay].T                 # (3, P)
    zb = zlev[loff[col] + lay + 1].T
    x = np.concatenate([xv, xv])
    y = np.concatenate([yv, yv])
    z = np.concatenate([zt, zb])
    return x, y, z


# ---------------------------------------------------------------------------
# velocity, time step
# ---------------------------------------------------------------------------

def rotation_rate(L: float = DOMAIN_L, umax: float = 0.5) -> float:
    """Solid-body rotation about the square's centre, |U| = umax at corners."""
    return umax * math.sqrt(2.0) / L


def solid_body_velocity(x, y, L: float = DOMAIN_L, umax: float = 0.5):
    """Nodal (u, v, w) of the rotation u = -w (y-L/2), v = w (x-L/2), w = 0."""
    om = rotation_rate(L, umax)
    out = np.empty((3,) + np.shape(x), dtype=np.float64)
    np.multiply(y - 0.5 * L, -om, out=out[0])
    np.multiply(x - 0.5 * L, om, out=out[1])
    out[2] = 0.0
    return out


def cfl_dt(vxy, tri, U=None, cfl: float = 0.3, umax: float | None = None) -> float:
    """dt = cfl * min_K d_K / max|U| with d_K = 4 area / perimeter (max|U|
    over the nodal velocity U, or given as ``umax``)."""
    p = vxy[tri]
    e0 = p[:, 1] - p[:, 0]
    e1 = p[:, 2] - p[:, 1]
    e2 = p[:, 0] - p[:, 2]
    area = 0.5 * np.abs(e0[:, 0] * (-e2[:, 1]) - e0[:, 1] * (-e2[:, 0]))
    per = (np.hypot(e0[:, 0], e0[:, 1]) + np.hypot(e1[:, 0], e1[:, 1])
           + np.hypot(e2[:, 0], e2[:, 1]))
    d = 4.0 * area / per
    if umax is None:
        umax = float(np.sqrt(np.einsum("cip,cip->ip", U, U)).max())
    return float(cfl * d.min() / umax)


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def _blob(x, y, cx=7000.0, cy=5000.0, sigma=1000.0):
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * sigma ** 2))


def rotating_blob(seed: int = 0, n: int = 30, n_layers: int = 10) -> Workload:
    """Plain method, FP64: 31x31-vertex split squares (1800 triangles) with
    20% jitter, 10 sigma layers over h = 20 + 10 sin sin, solid-body rotation
    (0.5 m/s max, w = 0), Gaussian blob (sigma 1 km, centre (7 km, 5 km),
    uniform in depth), kappa = 1e-3 m^2/s, CFL 0.3, 10 steps."""
    vxy, tri, nbr = square_mesh(n, seed=seed)
    nl, zlev = sigma_levels(vxy, tri, n_layers)
    x, y, _ = prism_node_xyz(vxy, tri, nl, zlev)
    U = solid_body_velocity(x, y)
    T0 = _blob(x, y)[None]
    return Workload("rotating_blob", vxy, tri, nbr, nl, zlev, U, T0,
                    kappa=np.full(n_layers, 1e-3), dt=cfl_dt(vxy, tri, U),
                    t_ext=np.zeros(1), n_steps=10)


def adjoint_blob(seed: int = 0, n: int = 158, n_layers: int = 20) -> Workload:
    """Differentiation form: the rotating-blob tracer problem on 158 x 158 split
    squares (49,928 triangles) x 20 sigma layers (998,560 prisms), FP64, 200
    steps with a checkpoint every 20."""
    w = rotating_blob(seed=seed, n=n, n_layers=n_layers)
    w.name = "adjoint_blob"
    w.n_steps = 200
    return w


def four_field_ocean(seed: int = 0, n: int = 316, n_layers: int = 30) -> Workload:
    """FP64 vs FP32 at scale: n=316 split squares (199,712 triangles), 30 sigma
    layers (5,991,360 prisms), 4 advected scalars: u, v (the rotation's
    components), temperature 25 + 15 z/h + U(+-0.1), salinity 35 + U(+-0.5);
    kappa_l = 10^(-2 - 3 l/(N-1)); exterior values (0, 0, 17.5, 35).
    Field noise uses default_rng([seed, 1])."""
    vxy, tri, nbr = square_mesh(n, seed=seed)
    nl, zlev = sigma_levels(vxy, tri, n_layers)
    x, y, z = prism_node_xyz(vxy, tri, nl, zlev)
    U = solid_body_velocity(x, y)
    h = bump_bathymetry(x, y)
    rng = np.random.default_rng([seed, 1])
    temp = 25.0 + 15.0 * z / h + rng.uniform(-0.1, 0.1, size=z.shape)
    salt = 35.0 + rng.uniform(-0.5, 0.5, size=z.shape)
    T0 = np.stack([U[0], U[1], temp, salt])
    lvl = np.arange(n_layers, dtype=np.float64)
    kappa = 10.0 ** (-2.0 - 3.0 * lvl / max(n_layers - 1, 1))
    return Workload("four_field_ocean", vxy, tri, nbr, nl, zlev, U, T0, kappa=kappa,
                    dt=cfl_dt(vxy, tri, U), t_ext=np.array([0.0, 0.0, 17.5, 35.0]),
                    n_steps=100)


def tiny(seed: int = 0, n: int = 2, n_layers: int = 3, n_fields: int = 1) -> Workload:
    """2x2 split squares x 3 sigma layers = 24 prisms (dense brute force)."""
    vxy, tri, nbr = square_mesh(n, seed=seed)
    nl, zlev = sigma_levels(vxy, tri, n_layers)
    x, y, z = prism_node_xyz(vxy, tri, nl, zlev)
    U = solid_body_velocity(x, y)
    rng = np.random.default_rng([seed, 2])
    T0 = rng.standard_normal((n_fields, 6, x.shape[1]))
    kappa = np.geomspace(1e-2, 1e-4, n_layers)
    return Workload("tiny", vxy, tri, nbr, nl, zlev, U, T0, kappa=kappa,
                    dt=cfl_dt(vxy, tri, U), t_ext=np.linspace(0.0, 1.0, n_fields))


def smooth_field(vxy_x, vxy_y, seed: int, L: float = DOMAIN_L, modes: int = 3):
    """Seeded smooth field in [0, 1]: normalised sum of a few cosine modes."""
    rng = np.random.default_rng([seed, 3])
    g = np.zeros_like(vxy_x)
    for _ in range(modes):
        kx, ky = rng.integers(1, 4, size=2)
        ph = rng.uniform(0, 2 * np.pi, size=2)
        g += np.cos(np.pi * kx * vxy_x / L + ph[0]) * np.cos(np.pi * ky * vxy_y / L + ph[1])
    g -= g.min()
    return g / max(g.max(), 1e-300)


def ragged(seed: int = 0, n: int = 12, n_fields: int = 2, dz: float = 5.0,
           n_min: int = 2, n_max: int = 9, depth_max: float = 45.0) -> Workload:
    """Small z-level mesh with bathymetry-dependent layer counts (walls where a
    neighbour column is shallower), for ragged-column tests."""
    vxy, tri, nbr = square_mesh(n, seed=seed)
    cxy = vxy[tri].mean(axis=1)
    depth = 5.0 + (depth_max - 5.0) * smooth_field(cxy[:, 0], cxy[:, 1], seed)
    nl, zlev = zlevel_levels(vxy, tri, depth, dz, n_min, n_max)
    x, y, z = prism_node_xyz(vxy, tri, nl, zlev)
    U = solid_body_velocity(x, y)
    rng = np.random.default_rng([seed, 4])
    T0 = 1.0 + rng.uniform(-0.5, 0.5, size=(n_fields, 6, x.shape[1]))
    T0[0] = _blob(x, y) + 0.01 * z
    kappa = np.geomspace(1e-2, 1e-5, int(nl.max()))
    return Workload("ragged", vxy, tri, nbr, nl, zlev, U, T0, kappa=kappa,
                    dt=cfl_dt(vxy, tri, U), t_ext=np.linspace(0.5, 1.5, n_fields))


def _concat_members(parts):
    """Concatenate independent member meshes (disjoint vertex and column ids)."""
    vxy, tri, nbr, nl, zl, moff = [], [], [], [], [], [0]
    voff = coff = 0
    for (v, t, nb, n, z) in parts:
        vxy.append(v)
        tri.append(t + voff)
        nbr.append(np.where(nb >= 0, nb + coff, -1))
        nl.append(n)
        zl.append(z)
        voff += len(v)
        coff += len(t)
        moff.append(coff)
    return (np.concatenate(vxy), np.concatenate(tri).astype(np.int32),
            np.concatenate(nbr).astype(np.int32), np.concatenate(nl).astype(np.int32),
            np.concatenate(zl), np.array(moff, dtype=np.int32))


def zlevel_ensemble(seed: int = 0, n_members: int = 16, n_lo: int = 100, n_hi: int = 244,
            dz: float = 5.0, n_min: int = 5, n_max: int = 60, with_fields: bool = True) -> Workload:
    """Batched form: independently seeded members (member m uses seed 1000 + m)
    of n ~ U{n_lo..n_hi} split squares (about 20k-120k triangles each), flat
    z-levels every dz metres, column depth h_c = 25 + 275 g(x, y) at the
    centroid (g a seeded smooth field in [0, 1]), layer count
    clamp(ceil(h_c/dz), n_min, n_max); stair-step bottom (steps are walls).
    Four fields as in four_field_ocean (temperature linear in depth over 300 m)."""
    parts = []
    for m in range(n_members):
        ms = 1000 + seed * 100 + m
        n = int(np.random.default_rng([ms, 5]).integers(n_lo, n_hi + 1))
        v, t, nb = square_mesh(n, seed=ms)
        cxy = v[t].mean(axis=1)
        depth = 25.0 + 275.0 * smooth_field(cxy[:, 0], cxy[:, 1], ms)
        nl, zl = zlevel_levels(v, t, depth, dz, n_min, n_max)
        parts.append((v, t, nb, nl, zl))
    vxy, tri, nbr, nl, zl, moff = _concat_members(parts)
    x, y, z = prism_node_xyz(vxy, tri, nl, zl)
    U = solid_body_velocity(x, y)
    vel_v = solid_body_velocity(vxy[:, 0], vxy[:, 1])
    umax = float(np.hypot(vel_v[0], vel_v[1]).max())
    del x, y
    if with_fields:
        rng = np.random.default_rng([seed, 6])
        temp = 25.0 + 15.0 * z / 300.0 + rng.uniform(-0.1, 0.1, size=z.shape)
        salt = 35.0 + rng.uniform(-0.5, 0.5, size=z.shape)
        T0 = np.empty((4,) + z.shape)
        T0[0], T0[1], T0[2], T0[3] = U[0], U[1], temp, salt
    else:
        T0 = np.zeros((4,) + z.shape)
    lvl = np.arange(n_max, dtype=np.float64)
    kappa = 10.0 ** (-2.0 - 3.0 * lvl / (n_max - 1))
    return Workload("zlevel_ensemble", vxy, tri, nbr, nl, zl, U, T0, kappa=kappa,
                    dt=cfl_dt(vxy, tri, umax=umax), t_ext=np.array([0.0, 0.0, 17.5, 35.0]),
                    n_steps=50, member_tri_off=moff)


def small_ensemble(seed: int = 0, n_members: int = 3, n_lo: int = 6, n_hi: int = 10,
                   n_fields: int = 2) -> Workload:
    """A few small z-level members (test-sized batched form)."""
    w = zlevel_ensemble(seed=seed, n_members=n_members, n_lo=n_lo, n_hi=n_hi, dz=10.0, n_min=2, n_max=12)
    rng = np.random.default_rng([seed, 8])
    T0 = 1.0 + rng.uniform(-0.5, 0.5, size=(n_fields, 6, w.n_prisms))
    return Workload("ensemble", w.vxy, w.tri, w.nbr, w.nlayers, w.zlev, w.U, T0,
                    kappa=np.geomspace(1e-2, 1e-5, int(w.nlayers.max())), dt=w.dt,
                    t_ext=np.linspace(0.0, 1.0, n_fields), n_steps=5,
                    member_tri_off=w.member_tri_off)
