"""GPU parity of the split-IMEX step (sdg_step with SDG_SCHEME_SPLIT_IMEX)
against the oracle's two-step scheme, through the C ABI.

Metric as in the other parity tests: per field, ||x_gpu - x_oracle||_inf /
||x_oracle||_inf.  FP64 bar 1e-12.  At full size (199,712 columns x 30
layers) one step is checked on sampled columns against the oracle
evaluated where those columns need it, and a property that holds at any
size: constants with matching exterior values are kept.
"""

import numpy as np
import pytest

import oracle as O
import paper_2605_16082_amd as P
import workloads as W
from oracle.split_imex import imex_step
from tests.test_gpu_parity import case, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
IMEX = P.SDG_SCHEME_SPLIT_IMEX


def upload(w, precision=P.SDG_FP64):
    return P.from_workload(w, precision, time_scheme=IMEX)


@pytest.mark.parametrize("name,n_steps", [("tiny", 2), ("single", 2), ("rotating_blob", 4), ("ragged", 3),
                                          ("deep_ragged", 2), ("wnonzero", 2)])
def test_imex_step_parity(name, n_steps):
    w, m = case(name)
    s, U, kappa, state = upload(w)
    s.step(n_steps)
    s.sync()
    got = s.gather(state)
    ref = w.T0
    for _ in range(n_steps):
        ref = imex_step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty)
    err = rel_err(got, ref)
    print(name, n_steps, "imex steps", err)
    assert np.all(err <= TOL64), err


def test_imex_stiff_diffusion_parity():
    """dt 50x the advective one: the vertical part far past its explicit limit."""
    w, m = case("ragged")
    s, U, kappa, state = upload(w)
    U0 = np.zeros_like(w.U)
    s.scatter(U0, out=U)
    dt = 50.0 * w.dt
    s.set_params(dt, w.t_ext, w.penalty, w.w_is_zero, time_scheme=IMEX)
    s.step(2)
    s.sync()
    ref = imex_step(m, U0, w.kappa, imex_step(m, U0, w.kappa, w.T0, dt, w.t_ext, w.penalty), dt, w.t_ext,
                    w.penalty)
    err = rel_err(s.gather(state), ref)
    print("stiff", err)
    assert np.all(err <= TOL64), err


@pytest.mark.parametrize("precision", [P.SDG_FP32_STATE_FP64_SOLVE, P.SDG_FP32])
def test_imex_float_forms(precision):
    w, m = case("rotating_blob")
    s, U, kappa, state = upload(w, precision)
    s.step(4)
    s.sync()
    ref = w.T0
    for _ in range(4):
        ref = imex_step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty)
    err = rel_err(s.gather(state), ref)
    print("imex", precision, err)
    assert np.all(err <= 2e-5), err


@pytest.mark.parametrize("shape", [(1, 1, 0), (4, 0, 0), (8, 1, 0), (16, 1, 1), (32, 0, 0)])
def test_imex_launch_shapes_bitwise(shape):
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


def test_imex_graph_replay_matches_eager():
    w, m = case("rotating_blob")
    g, _, _, gstate = upload(w)
    e, _, _, estate = upload(w)
    g.graph_capture_step()
    for k in range(3):
        g.graph_launch(1)
        e.step(1)
        g.sync()
        e.sync()
        assert np.array_equal(g.gather(gstate), e.gather(estate)), k


def test_imex_four_field_ocean_keeps_constants():
    w = W.four_field_ocean()
    c = np.array([0.25, -1.5, 17.5, 35.0])
    w.T0 = np.broadcast_to(c[:, None, None], w.T0.shape).copy()
    w.t_ext = c.copy()
    s, U, kappa, state = upload(w)
    s.autotune(reps=2)
    s.step(2)
    s.sync()
    got = state[:, :, s.slots].double()
    dev = (got - s.torch.as_tensor(c, device=got.device)[:, None, None]).abs().amax(dim=(1, 2)).cpu().numpy()
    print("four_field_ocean constants", dev)
    assert np.all(dev <= 1e-12 * np.abs(c).max()), dev


def test_imex_four_field_ocean_step_sampled_against_oracle():
    """One split-IMEX step at full size (199,712 columns x 30 layers, 4
    fields) in the autotuned launch shape, against the oracle's two steps
    evaluated only where 60 sampled columns need them: x_h on the samples and
    their lateral neighbours (its residual on those prisms), then x_1 on the
    samples."""
    from oracle.split_imex import _residual, imex_full_step, imex_half_step
    w = W.four_field_ocean()
    s, U, kappa, state = upload(w)
    print("tuning", s.autotune(reps=2))
    s.scatter(w.T0, out=state)
    s.step(1)
    s.sync()
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    rng = np.random.default_rng(21)
    cols = np.sort(rng.choice(m.C, 60, replace=False))
    ring = np.unique(np.concatenate([cols, m.nbr[cols].ravel()]))
    ring = ring[ring >= 0]

    def prisms(cs):
        return np.concatenate([m.off[c] + np.arange(m.nl[c]) for c in cs])

    shape = w.T0.shape
    R0, H, Rh, X1 = (np.zeros(shape) for _ in range(4))
    pr_ring, pr_cols = prisms(ring), prisms(cols)
    R0[:, :, pr_ring] = _residual(m, w.U, w.T0, w.t_ext, None, w.penalty, pr_ring)
    imex_half_step(m, w.kappa, w.T0, R0, w.dt, w.penalty, H, columns=ring)
    Rh[:, :, pr_cols] = _residual(m, w.U, H, w.t_ext, None, w.penalty, pr_cols)
    imex_full_step(m, w.kappa, w.T0, H, Rh, w.dt, w.penalty, X1, columns=cols)
    got = state[:, :, s.slots[pr_cols]].double().cpu().numpy()
    err = rel_err(got, X1[:, :, pr_cols])
    print("four_field_ocean split-IMEX step, sampled columns", err)
    assert np.all(err <= TOL64), err


def test_imex_rejects_adjoint_and_bad_scheme():
    w, m = case("tiny")
    s, U, kappa, state = upload(w)
    z = s.new_state()
    with pytest.raises(P.SlimDGError) as e:
        s.step_adjoint(z, s.new_state())
    assert e.value.status == -5
    with pytest.raises(P.SlimDGError) as e:
        s.set_params(w.dt, w.t_ext, w.penalty, w.w_is_zero, time_scheme=7)
    assert e.value.status == -1
