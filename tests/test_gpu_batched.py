"""GPU tests of the batched form: several members with ragged z-level
columns, launch-shape tuning, the autotuner and graph-captured steps.

Launch shapes change only which workgroup computes a prism, never the
arithmetic, so results must be bitwise identical across shapes; a replayed
graph must be bitwise identical to the eager step.  Parity with the FP64
oracle uses the per-field max-norm relative error (bar 1e-12 in FP64)."""

import numpy as np
import pytest

import oracle as O
import paper_2605_16082_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def rel_err(got, ref):
    F = ref.shape[0]
    return (np.abs(got - ref).reshape(F, -1).max(axis=1)
            / np.maximum(np.abs(ref).reshape(F, -1).max(axis=1), 1e-300))


_W = {}


def ensemble():
    if "e" not in _W:
        w = W.small_ensemble()
        _W["e"] = (w, O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev))
    return _W["e"]


# every (tile height, XCD remap, persistent) shape; heights from 8 up are the
# column-walk kernel
SHAPES = [(4, 1, 0), (1, 0, 1), (8, 1, 0), (2, 1, 1), (16, 0, 1), (1, 1, 0), (32, 1, 1), (4, 0, 1),
          (2, 0, 0), (8, 0, 1), (1, 0, 0), (16, 1, 0), (4, 1, 1), (32, 0, 0), (2, 1, 0), (8, 1, 1),
          (1, 1, 1), (16, 0, 0), (4, 0, 0), (32, 1, 0), (2, 0, 1), (8, 0, 0), (16, 1, 1), (32, 0, 1),
          (12, 1, 0), (12, 0, 1), (12, 1, 1), (12, 0, 0)]


@pytest.mark.parametrize("precision", [P.SDG_FP64, P.SDG_FP32])
def test_launch_shape_does_not_change_results(precision):
    w, m = ensemble()
    s, U, kappa, state = P.from_workload(w, precision)
    rng = np.random.default_rng(3)
    Ts = s.scatter(w.T0 + 0.1 * rng.standard_normal(w.T0.shape))
    ref = None
    for tl, x, pers in SHAPES:
        s.set_tuning(tl, x, pers)
        assert s.get_tuning() == (tl, x, pers)
        outs = [s.rk_stage(k, state, Ts) for k in range(3)] + [s.rhs_3d(Ts)]
        s.sync()
        got = [s.gather(o) for o in outs]
        if ref is None:
            ref = got
        else:
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (tl, x, pers)


def test_persistent_grid_walks_many_tiles():
    """A mesh with several times more tiles than the chip holds at once, so
    every persistent workgroup walks several tiles: bitwise the same stage
    output as one workgroup per tile, for every tile height and remap."""
    w = W.rotating_blob(n=100, n_layers=20, seed=4)
    s, U, kappa, state = P.from_workload(w)
    rng = np.random.default_rng(8)
    Ts = s.scatter(w.T0 + 0.1 * rng.standard_normal(w.T0.shape))
    for tl in (1, 2, 4, 8, 12, 16, 32):
        outs = []
        for x, pers in ((1, 0), (1, 1), (0, 1)):
            s.set_tuning(tl, x, pers)
            outs.append(s.rk_stage(2, state, Ts))
        s.sync()
        for o in outs[1:]:
            assert torch_equal(o, outs[0]), tl


def torch_equal(a, b):
    return bool((a == b).all().item())


def test_bad_tuning_rejected():
    w, m = ensemble()
    s = P.from_workload(w)[0]
    for bad in [(3, 1, 0), (64, 1, 0), (2, 2, 0), (2, 1, 2)]:
        with pytest.raises(P.SlimDGError) as e:
            s.set_tuning(*bad)
        assert e.value.status == -1, bad


def test_bad_bucket_walks_rejected():
    w, m = ensemble()
    s = P.from_workload(w)[0]
    for bad in ([8, 8, 8, 8, 8, 7], [8, 8, 65, 8, 8, 8], [-7, 8, 8, 8, 8, 8], [0] * 6):
        with pytest.raises(P.SlimDGError) as e:
            s.set_tuning(0, 1, 0, bad)
        assert e.value.status == -1, bad


# walk segmentations per depth bucket (1-8, 9-16, 17-24, 25-32, 33-48, > 48
# layers): fixed lengths, balanced lengths (negative) and mixtures
BUCKET_WALKS = [([8] * 6, 1, 0), ([-8] * 6, 0, 1), ([12, -12, 16, -16, 32, -24], 1, 1),
                ([64, 64, 64, 64, 64, 64], 0, 0), ([-64, 9, -10, 13, -17, 33], 1, 0)]


@pytest.mark.parametrize("precision", [P.SDG_FP64, P.SDG_FP32])
def test_bucket_walks_do_not_change_results(precision):
    """Per-depth-bucket walk tables give bitwise the stage outputs of the
    2-layer one-thread-per-prism tile, on ragged z-level columns of 1-60
    layers (cells of 17-60), the small ensemble (cells of 2-12) and a deep
    uniform mesh where persistent workgroups walk many tiles."""
    deep = W.ragged(seed=3, n=40, n_min=1, n_max=60, depth_max=300.0, n_fields=2)   # cells of 17-60 layers
    assert deep.nlayers.min() <= 8 and deep.nlayers.max() > 48
    for w in (deep, ensemble()[0], W.rotating_blob(n=60, n_layers=37, seed=5)):
        s, U, kappa, state = P.from_workload(w, precision)
        rng = np.random.default_rng(6)
        Ts = s.scatter(w.T0 + 0.1 * rng.standard_normal(w.T0.shape))
        s.set_tuning(2, 1, 0)
        ref = [s.rk_stage(k, state, Ts) for k in range(3)]
        for wl, x, pers in BUCKET_WALKS:
            s.set_tuning(0, x, pers, wl)
            assert s.get_tuning() == (0, x, pers) and s.walk_layers() == wl
            outs = [s.rk_stage(k, state, Ts) for k in range(3)]
            s.sync()
            for a, b in zip(outs, ref):
                assert torch_equal(a, b), (wl, x, pers)


def test_autotune_keeps_results():
    w, m = ensemble()
    a = P.from_workload(w)
    b = P.from_workload(w)
    choice = a[0].autotune(reps=3)
    assert choice[0] in (0, 1, 2, 4, 8, 12, 16, 32) and choice[1] in (0, 1) and choice[2] in (0, 1)
    if choice[0] == 0:
        assert all(8 <= abs(v) <= 64 for v in a[0].walk_layers())
    a[0].step(2)
    b[0].step(2)
    a[0].sync()
    b[0].sync()
    assert np.array_equal(a[0].gather(a[3]), b[0].gather(b[3]))


@pytest.mark.parametrize("precision", [P.SDG_FP64, P.SDG_FP32_STATE_FP64_SOLVE])
def test_graph_replay_matches_eager(precision):
    import torch
    w, m = ensemble()
    g = P.from_workload(w, precision)
    e = P.from_workload(w, precision)
    g[0].graph_capture_step()
    scratch = torch.ones(1 << 20, device="cuda")
    for rep in range(4):
        g[0].graph_launch(1)
        e[0].step(1)
        # unrelated eager work and a synchronisation between replays
        scratch.mul_(1.0001)
        torch.cuda.synchronize()
        assert np.array_equal(g[0].gather(g[3]), e[0].gather(e[3])), rep
    g[0].graph_launch(3)
    e[0].step(3)
    g[0].sync()
    e[0].sync()
    assert np.array_equal(g[0].gather(g[3]), e[0].gather(e[3]))


def test_graph_invalidated_by_setters():
    w, m = ensemble()
    s, U, kappa, state = P.from_workload(w)
    s.graph_capture_step()
    s.graph_launch(1)
    s.set_params(w.dt * 0.5, w.t_ext, w.penalty, w.w_is_zero)
    with pytest.raises(P.SlimDGError) as e:
        s.graph_launch(1)
    assert e.value.status == -4
    s.graph_capture_step()
    s.graph_launch(1)
    s.sync()


def test_ensemble_step_and_member_mass_parity():
    w, m = ensemble()
    s, U, kappa, state = P.from_workload(w)
    mass0 = s.mass(state)
    s.step(3)
    s.sync()
    ref = w.T0
    for _ in range(3):
        ref = O.step(m, w.U, w.kappa, ref, w.dt, w.t_ext, w.penalty)
    err = rel_err(s.gather(state), ref)
    print("ensemble 3 steps", err)
    assert np.all(err <= 1e-12), err
    # per-member mass sums
    Mp = O.mass_matrix(m)
    per_prism = np.einsum("nij,fjn->fn", Mp, w.T0)
    off = m.off[w.member_tri_off]
    ref_mass = np.stack([per_prism[:, off[k]:off[k + 1]].sum(axis=1) for k in range(len(off) - 1)])
    assert np.allclose(mass0, ref_mass, rtol=1e-13, atol=0), (mass0, ref_mass)


@pytest.mark.parametrize("precision", [P.SDG_FP64, P.SDG_FP32_STATE_FP64_SOLVE])
def test_zlevel_ensemble_sampled_parity(precision):
    """16 members, 1.1M ragged z-level columns (5-60 layers), in FP64 (bar
    1e-12) and with FP32 state and the FP64 solve (5e-5, the oracle fed the
    same FP32-representable inputs), checked on sampled prisms and columns
    in the autotuned launch shape."""
    w = W.zlevel_ensemble()
    tol = 1e-12 if precision == P.SDG_FP64 else 5e-5
    if precision != P.SDG_FP64:
        # the GPU holds FP32 copies of the inputs: feed the oracle the same values
        w.U = w.U.astype(np.float32).astype(np.float64)
        w.T0 = w.T0.astype(np.float32).astype(np.float64)
    s, U, kappa, state = P.from_workload(w, precision)
    print("tuning", s.autotune(reps=2))
    m = O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)
    rng = np.random.default_rng([4, 2])
    sample = np.sort(rng.choice(m.P, 3000, replace=False))
    out = s.rk_stage(1, state, state)
    s.sync()
    got = out[:, :, s.slots[sample]].double().cpu().numpy()
    ref = O.rk_stage(m, w.U, 1, w.T0, w.T0, w.dt, w.t_ext, prisms=sample)
    err = rel_err(got, ref)
    print("zlevel_ensemble stage 1", err)
    assert np.all(err <= tol), err
    cols = np.sort(rng.choice(m.C, 100, replace=False))
    out = s.vertical_implicit_solve(state)
    s.sync()
    ref_full = O.implicit_solve(m, w.kappa, w.dt, w.T0, w.penalty, columns=cols)
    pr = np.concatenate([m.off[c] + np.arange(m.nl[c]) for c in cols])
    err = rel_err(out[:, :, s.slots[pr]].double().cpu().numpy(), ref_full[:, :, pr])
    print("zlevel_ensemble solve", err)
    assert np.all(err <= tol), err
