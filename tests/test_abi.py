"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point its header declares, lays meshes out as documented and
rejects malformed meshes with the documented status codes."""

import os
import re

import numpy as np
import pytest

import paper_2605_16082_amd as P
import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "slimdg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    names = _declared()
    assert "sdg_step" in names and "sdg_vertical_implicit_solve" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.EXPORTED)
    assert lib.sdg_abi_version() == 8


def test_layout_matches_cell_formula():
    w = W.ragged(n=10)
    m = P.Mesh.from_workload(w)
    L = m.layout()
    slots = m.prism_slots()
    C = w.n_cols
    assert L.n_prisms == w.n_prisms
    assert L.n_cells == (C + 63) // 64
    assert len(np.unique(slots)) == len(slots)
    assert slots.max() < L.n_slots
    # recompute from the documented formula
    depth = [w.nlayers[k * 64:(k + 1) * 64].max() for k in range(L.n_cells)]
    base = np.concatenate([[0], np.cumsum(np.array(depth) * 64)])
    assert L.n_slots == base[-1]
    q = 0
    for c in range(C):
        for l in range(w.nlayers[c]):
            assert slots[q] == base[c // 64] + l * 64 + c % 64
            q += 1
    assert L.state_bytes == w.n_fields * 6 * L.n_slots * 8
    assert L.workspace_bytes > 2 * L.state_bytes


def test_fp32_layout_halves_state():
    w = W.tiny(n_fields=3)
    L64 = P.Mesh.from_workload(w, P.SDG_FP64).layout()
    L32 = P.Mesh.from_workload(w, P.SDG_FP32).layout()
    assert L32.state_elem_bytes == 4 and L64.state_elem_bytes == 8
    assert 2 * L32.state_bytes == L64.state_bytes


def _status(fn):
    with pytest.raises(P.SlimDGError) as e:
        fn()
    return e.value.status


def test_rejects_malformed_meshes():
    w = W.tiny()
    # clockwise triangle
    tri = w.tri.copy()
    tri[0] = tri[0, ::-1]
    assert _status(lambda: P.Mesh(w.vxy, tri, w.nbr, w.nlayers, w.zlev, 1).layout()) == -2
    # asymmetric neighbours
    nbr = w.nbr.copy()
    k = int(np.nonzero(nbr[0] >= 0)[0][0])
    nbr[0, k] = -1
    assert _status(lambda: P.Mesh(w.vxy, w.tri, nbr, w.nlayers, w.zlev, 1).layout()) == -2
    # zero-thickness layer
    z = w.zlev.copy()
    z[1] = z[0]
    assert _status(lambda: P.Mesh(w.vxy, w.tri, w.nbr, w.nlayers, z, 1).layout()) == -2
    # non-conforming levels on a shared edge
    z = w.zlev.copy()
    z[1, 1] -= 0.25
    assert _status(lambda: P.Mesh(w.vxy, w.tri, w.nbr, w.nlayers, z, 1).layout()) == -2
    # no layers
    nl = w.nlayers.copy()
    nl[0] = 0
    assert _status(lambda: P.Mesh(w.vxy, w.tri, w.nbr, nl, w.zlev, 1).layout()) == -2
    # vertex id out of range
    tri = w.tri.copy()
    tri[1, 2] = len(w.vxy)
    assert _status(lambda: P.Mesh(w.vxy, tri, w.nbr, w.nlayers, w.zlev, 1).layout()) == -2
    # no triangles at all
    assert _status(lambda: P.Mesh(w.vxy, w.tri[:0], w.nbr[:0], w.nlayers[:0], w.zlev[:0], 1).layout()) == -2
    # unsupported field count
    assert _status(lambda: P.Mesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev, 5).layout()) == -5
    assert _status(lambda: P.Mesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev, 0).layout()) == -5


def test_members_must_be_disjoint():
    w = W.tiny()
    C = w.n_cols
    off = np.array([0, C // 2, C])
    # the split cuts through neighbour pairs of one connected mesh
    assert _status(lambda: P.Mesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev, 1, member_tri_off=off).layout()) == -2
    # two copies of the mesh side by side are fine
    nv = len(w.vxy)
    tri2 = np.concatenate([w.tri, w.tri + nv])
    nbr2 = np.concatenate([w.nbr, np.where(w.nbr >= 0, w.nbr + C, -1)])
    m = P.Mesh(np.concatenate([w.vxy, w.vxy]), tri2, nbr2, np.concatenate([w.nlayers, w.nlayers]),
               np.concatenate([w.zlev, w.zlev]), 1, member_tri_off=np.array([0, C, 2 * C]))
    assert m.layout().n_prisms == 2 * w.n_prisms


def test_error_message_is_set():
    w = W.tiny()
    tri = w.tri.copy()
    tri[0] = tri[0, ::-1]
    with pytest.raises(P.SlimDGError) as e:
        P.Mesh(w.vxy, tri, w.nbr, w.nlayers, w.zlev, 1).layout()
    assert "counter-clockwise" in e.value.message


def test_layer_count_limits():
    """A column may hold 1 to 65,535 layers (tile tables index layers in 16
    bits): the deepest allowed column is laid out, one more layer is refused
    with SDG_E_MESH."""
    vxy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    nbr = np.full((1, 3), -1, dtype=np.int32)
    for n, ok in ((65535, True), (65536, False)):
        zlev = np.repeat(-np.arange(n + 1, dtype=np.float64)[:, None], 3, axis=1)
        mesh = P.Mesh(vxy, tri, nbr, np.array([n], dtype=np.int32), zlev, 1)
        if ok:
            lay = mesh.layout()
            assert lay.max_layers == n and lay.n_prisms == n and lay.n_slots == 64 * n
        else:
            assert _status(lambda: mesh.layout()) == -2


def test_slot_count_limit():
    """The kernels address one field's six node rows with 32-bit byte offsets,
    so a mesh is laid out only while 6 x n_slots x 8 bytes fits 32 bits
    (89,478,485 slots, whatever the precision): 22 cells of 64 isolated
    columns, one column per cell deep, are laid out at 89,478,464 slots and
    refused with SDG_E_UNSUPPORTED at 89,478,528."""
    n_cells = 22
    C = 64 * n_cells
    vxy = np.zeros((3 * C, 2))
    for c in range(C):
        x0, y0 = 2.0 * (c % 64), 2.0 * (c // 64)
        vxy[3 * c:3 * c + 3] = [[x0, y0], [x0 + 1.0, y0], [x0, y0 + 1.0]]
    tri = np.arange(3 * C, dtype=np.int32).reshape(C, 3)
    nbr = np.full((C, 3), -1, dtype=np.int32)
    for last, ok in ((21866, True), (21867, False)):
        nl = np.ones(C, dtype=np.int32)
        nl[::64] = 65535
        nl[64 * (n_cells - 1)] = last
        zlev = np.concatenate([np.repeat(-np.arange(n + 1, dtype=np.float64)[:, None], 3, axis=1) for n in nl])
        slots = 64 * int(nl[::64].sum())
        assert (6 * slots * 8 < 2 ** 32) == ok
        for prec in (P.SDG_FP64, P.SDG_FP32_STATE_FP64_SOLVE):
            mesh = P.Mesh(vxy, tri, nbr, nl, zlev, 1, prec)
            if ok:
                assert mesh.layout().n_slots == slots
            else:
                assert _status(lambda: mesh.layout()) == -5
