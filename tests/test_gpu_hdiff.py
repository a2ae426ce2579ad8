"""GPU parity of the horizontal (Okubo) diffusion term against the oracle,
through the C ABI: the explicit operator alone and with advection, stages,
both time schemes, float forms, launch shapes, graph replay, and constants
kept at full size.

Metric: per field ||x_gpu - x_oracle||_inf / ||x_oracle||_inf, FP64 bar
1e-12.  The diffusivity is Okubo's scaled up 50x (okubo_scale) so that the
term is not negligible next to advection on these small meshes while the
explicit steps stay stable.
"""

import numpy as np
import pytest

import oracle as O
import paper_2605_16082_amd as P
import workloads as W
from oracle.horizontal_diffusion import okubo_diffusivity
from oracle.split_imex import imex_step
from tests.test_gpu_parity import case, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
SCALE = 50.0


def upload(w, precision=P.SDG_FP64, scheme=P.SDG_SCHEME_SSPRK3_LIE, scale=SCALE):
    return P.from_workload(w, precision, time_scheme=scheme, okubo_scale=scale)


@pytest.mark.parametrize("name", ["tiny", "single", "rotating_blob", "ragged", "deep_ragged"])
def test_pure_diffusion_operator(name):
    w, m = case(name)
    s, U, kappa, state = upload(w)
    U0 = np.zeros_like(w.U)
    s.scatter(U0, out=U)
    kh = okubo_diffusivity(m, SCALE)
    L = s.rhs_3d(state)
    s.sync()
    ref = O.explicit_operator(m, U0, w.T0, w.t_ext, kappa_h=kh, eta=w.penalty)
    err = rel_err(s.gather(L), ref)
    print(name, "pure diffusion", err)
    assert np.all(err <= TOL64), err


def _shuffled_columns(w, seed=4):
    """The workload with its triangles in random order: a 64-column cell then
    has most of its lateral faces on neighbours in other cells."""
    C = len(w.tri)
    perm = np.random.default_rng(seed).permutation(C)
    inv = np.empty(C, dtype=np.int64)
    inv[perm] = np.arange(C)
    nbr = np.where(w.nbr[perm] >= 0, inv[np.maximum(w.nbr[perm], 0)], -1).astype(w.nbr.dtype)
    zoff = np.concatenate([[0], np.cumsum(w.nlayers + 1)])
    poff = np.concatenate([[0], np.cumsum(w.nlayers)])
    zlev = np.concatenate([w.zlev[zoff[c]:zoff[c + 1]] for c in perm])
    pr = np.concatenate([np.arange(poff[c], poff[c + 1]) for c in perm])
    return W.Workload(w.name + "_shuffled", w.vxy, w.tri[perm], nbr, w.nlayers[perm], zlev, w.U[:, :, pr],
                      w.T0[:, :, pr], w.kappa, w.dt, w.t_ext, penalty=w.penalty, w_is_zero=w.w_is_zero)


def _most_other_cell_faces_per_cell(w):
    C = len(w.tri)
    cell = np.arange(C) // 64
    cross = (w.nbr >= 0) & ((w.nbr // 64) != cell[:, None])
    return int(np.bincount(cell, weights=cross.sum(axis=1)).max())


@pytest.mark.parametrize("shuffled", [False, True])
def test_other_cell_neighbours_staged_or_gathered(shuffled):
    """In locality order a cell has at most a few dozen faces on other cells,
    whose values the kernel stages in LDS (64 at most); in random order it has
    far more, and the kernel gathers them per thread instead.  Both against
    the oracle, with advection and three steps."""
    w0, _ = case("rotating_blob")
    w = _shuffled_columns(w0) if shuffled else w0
    most = _most_other_cell_faces_per_cell(w)
    assert (most > 64) == shuffled, most
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    s, U, kappa, state = upload(w)
    kh = okubo_diffusivity(m, SCALE)
    L = s.rhs_3d(state)
    s.sync()
    ref = O.explicit_operator(m, w.U, w.T0, w.t_ext, kappa_h=kh, eta=w.penalty)
    err = rel_err(s.gather(L), ref)
    s.step(3)
    s.sync()
    x = w.T0
    for _ in range(3):
        x = O.step(m, w.U, w.kappa, x, w.dt, w.t_ext, w.penalty, kappa_h=kh)
    err3 = rel_err(s.gather(state), x)
    print("shuffled" if shuffled else "locality order", most, "faces on other cells at most;", err, err3)
    assert np.all(err <= TOL64) and np.all(err3 <= TOL64), (err, err3)


@pytest.mark.parametrize("name", ["rotating_blob", "ragged", "wnonzero"])
def test_rhs_and_stages_with_advection(name):
    w, m = case(name)
    s, U, kappa, state = upload(w)
    kh = okubo_diffusivity(m, SCALE)
    L = s.rhs_3d(state)
    s.sync()
    err = rel_err(s.gather(L), O.explicit_operator(m, w.U, w.T0, w.t_ext, kappa_h=kh, eta=w.penalty))
    assert np.all(err <= TOL64), err
    rng = np.random.default_rng([13, len(name)])
    Ts_np = w.T0 + 0.1 * rng.standard_normal(w.T0.shape)
    Ts = s.scatter(Ts_np)
    for stage in range(3):
        out = s.rk_stage(stage, state, Ts)
        s.sync()
        ref = O.rk_stage(m, w.U, stage, w.T0, Ts_np, w.dt, w.t_ext, kappa_h=kh, eta=w.penalty)
        err = rel_err(s.gather(out), ref)
        print(name, "stage", stage, err)
        assert np.all(err <= TOL64), (stage, err)


@pytest.mark.parametrize("scheme,name,n_steps", [(P.SDG_SCHEME_SSPRK3_LIE, "rotating_blob", 3),
                                                 (P.SDG_SCHEME_SSPRK3_LIE, "deep_ragged", 2),
                                                 (P.SDG_SCHEME_SPLIT_IMEX, "rotating_blob", 3),
                                                 (P.SDG_SCHEME_SPLIT_IMEX, "ragged", 2)])
def test_steps_with_horizontal_diffusion(scheme, name, n_steps):
    w, m = case(name)
    s, U, kappa, state = upload(w, scheme=scheme)
    kh = okubo_diffusivity(m, SCALE)
    s.step(n_steps)
    s.sync()
    ref = w.T0
    for _ in range(n_steps):
        if scheme == P.SDG_SCHEME_SPLIT_IMEX:
            ref = imex_step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty, kappa_h=kh)
        else:
            ref = O.step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty, kappa_h=kh)
    err = rel_err(s.gather(state), ref)
    print(scheme, name, n_steps, err)
    assert np.all(err <= TOL64), err


@pytest.mark.parametrize("precision", [P.SDG_FP32_STATE_FP64_SOLVE, P.SDG_FP32])
def test_float_forms(precision):
    w, m = case("rotating_blob")
    s, U, kappa, state = upload(w, precision)
    kh = okubo_diffusivity(m, SCALE)
    s.step(3)
    s.sync()
    ref = w.T0
    for _ in range(3):
        ref = O.step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty, kappa_h=kh)
    err = rel_err(s.gather(state), ref)
    print("hdiff", precision, err)
    assert np.all(err <= 2e-5), err


@pytest.mark.parametrize("shape", [(1, 1, 0), (4, 0, 1), (8, 1, 0), (32, 0, 0)])
def test_launch_shapes_bitwise(shape):
    w, m = case("deep_ragged")
    ref_s, _, _, ref_state = upload(w)
    ref_s.set_tuning(2, 1, 0)
    ref_s.step(2)
    s, U, kappa, state = upload(w)
    s.set_tuning(*shape)
    s.step(2)
    s.sync()
    ref_s.sync()
    assert np.array_equal(s.gather(state), ref_s.gather(ref_state))


def test_graph_replay_matches_eager():
    w, m = case("ragged")
    g, _, _, gstate = upload(w, scheme=P.SDG_SCHEME_SPLIT_IMEX)
    e, _, _, estate = upload(w, scheme=P.SDG_SCHEME_SPLIT_IMEX)
    g.graph_capture_step()
    for k in range(3):
        g.graph_launch(1)
        e.step(1)
        g.sync()
        e.sync()
        assert np.array_equal(g.gather(gstate), e.gather(estate)), k


def test_four_field_ocean_sampled_stage_parity():
    """Full size (199,712 columns x 30 layers, 4 fields), Okubo's own
    diffusivity: the three stages on 3000 sampled prisms, autotuned shape."""
    w = W.four_field_ocean()
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    kh = okubo_diffusivity(m, 1.0)
    s, U, kappa, state = upload(w, scale=1.0)
    s.autotune(reps=2)
    rng = np.random.default_rng([3, 9])
    Ts_np = w.T0 + 0.05 * rng.standard_normal(w.T0.shape)
    Ts = s.scatter(Ts_np)
    sample = np.sort(rng.choice(m.P, 3000, replace=False))
    for stage in range(3):
        out = s.rk_stage(stage, state, Ts)
        s.sync()
        got = out[:, :, s.slots[sample]].double().cpu().numpy()
        ref = O.rk_stage(m, w.U, stage, w.T0, Ts_np, w.dt, w.t_ext, prisms=sample, kappa_h=kh, eta=w.penalty)
        err = rel_err(got, ref)
        print("four_field_ocean hdiff stage", stage, err)
        assert np.all(err <= TOL64), (stage, err)


def test_four_field_ocean_keeps_constants():
    w = W.four_field_ocean()
    c = np.array([0.25, -1.5, 17.5, 35.0])
    w.T0 = np.broadcast_to(c[:, None, None], w.T0.shape).copy()
    w.t_ext = c.copy()
    s, U, kappa, state = upload(w, scale=1.0)
    s.step(2)
    s.sync()
    got = state[:, :, s.slots].double()
    dev = (got - s.torch.as_tensor(c, device=got.device)[:, None, None]).abs().amax(dim=(1, 2)).cpu().numpy()
    print("four_field_ocean constants", dev)
    assert np.all(dev <= 1e-12 * np.abs(c).max()), dev


@pytest.mark.parametrize("name", ["tiny", "ragged"])
def test_adjoint_with_horizontal_diffusion_matches_oracle(name):
    import torch
    import oracle.adjoint as OA
    # a stiff vertical diffusion makes the column solve matter; dt stays stable
    if name == "tiny":
        w = W.tiny(n_fields=2)
        w.kappa = w.kappa * 1000.0
    else:
        w = W.ragged(n=6, n_fields=1)
        w.kappa = w.kappa * 300.0
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    kh = okubo_diffusivity(m, SCALE)
    n_steps = 3
    s, U, kappa, state = upload(w)
    T0 = s.scatter(w.T0).requires_grad_(True)
    kap = torch.as_tensor(w.kappa, dtype=torch.float64, device=s.device).requires_grad_(True)
    xN = P.TracerSteps.apply(T0, kap, s, n_steps, 2)
    J = P.MNorm.apply(xN, s)
    J.backward()
    Jr, gTr, gkr, gka = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n_steps, w.penalty, kappa_h=kh,
                                    return_scale=True)
    gT = s.gather(T0.grad)
    gk = kap.grad.detach().cpu().numpy()
    eT = np.abs(gT - gTr).max() / np.abs(gTr).max()
    ek = (np.abs(gk - gkr) / gka).max()
    print(name, "J", float(J.detach()), Jr, "dT0", eT, "dkappa / term magnitudes", ek)
    assert abs(float(J.detach()) - Jr) <= 1e-12 * abs(Jr)
    assert Jr < 2.0 * OA.objective(m, w.T0)                         # a stable run
    # dJ/dkappa_l is a cancelling sum: bar 1e-12 of its terms' magnitudes
    assert eT <= 1e-12 and ek <= 1e-12


def test_argument_errors():
    w, m = case("tiny")
    s, U, kappa, state = upload(w, scheme=P.SDG_SCHEME_SPLIT_IMEX)
    with pytest.raises(P.SlimDGError) as e:
        s.step_adjoint(s.new_state(), s.new_state())
    assert e.value.status == -5
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(P.SlimDGError) as e:
            s.set_params(w.dt, w.t_ext, w.penalty, w.w_is_zero, okubo_scale=bad)
        assert e.value.status == -1


def test_mesh_upload_forgets_params():
    """A mesh upload drops the parameters, whose exterior values and per-column
    diffusivity belong to the old mesh: the operator refuses to run until they
    are set again, and then matches the oracle."""
    import ctypes
    from paper_2605_16082_amd.slimdg import _check, _ptr

    w, m = case("rotating_blob")
    s, U, kappa, state = upload(w)
    _check(s.lib.sdg_mesh_upload(s.ctx, ctypes.byref(s.mesh.desc), _ptr(s.workspace),
                                 int(s.layout.workspace_bytes)))
    s.set_velocity(U)
    with pytest.raises(P.SlimDGError) as e:
        s.rhs_3d(state)
    assert e.value.status == -4
    s.set_params(w.dt, w.t_ext, w.penalty, w.w_is_zero, okubo_scale=SCALE)
    L = s.rhs_3d(state)
    s.sync()
    kh = okubo_diffusivity(m, SCALE)
    err = rel_err(s.gather(L), O.explicit_operator(m, w.U, w.T0, w.t_ext, kappa_h=kh, eta=w.penalty))
    assert np.all(err <= TOL64), err
