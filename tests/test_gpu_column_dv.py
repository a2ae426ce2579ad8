"""GPU parity of the matrix-free column solves (section 2.3) against the dense
oracle, through the C ABI.

Metric: per component, ||x_gpu - x_oracle||_inf / ||x_oracle||_inf over live
prisms.  FP64 bar 1e-12; the float-state forms are compared with the oracle
run on the float-rounded input (the values the kernel reads).  Inputs are
seeded normal right-hand sides in natural prism order.
"""

import numpy as np
import pytest

import oracle as O
import paper_2605_16082_amd as P
import workloads as W

pytestmark = pytest.mark.gpu

CD = O.column_dv
TOL = {P.SDG_FP64: 1e-12, P.SDG_FP32_STATE_FP64_SOLVE: 1e-6, P.SDG_FP32: 2e-5}
KINDS = {"vu": P.SDG_DV_VU, "vd": P.SDG_DV_VD}


def rel_err(got, ref):
    K = ref.shape[0]
    num = np.abs(got - ref).reshape(K, -1).max(axis=1)
    den = np.abs(ref).reshape(K, -1).max(axis=1)
    return num / np.maximum(den, 1e-300)


def _workload(name):
    if name == "ragged":          # 288 columns (4.5 cells), 2..9 layers
        return W.ragged(seed=1)
    if name == "deep_ragged":     # 162 columns, 1..37 layers
        return W.ragged(seed=3, n=9, n_min=1, n_max=37, depth_max=190.0)
    if name == "rotating_blob":         # 1800 columns x 10 layers
        return W.rotating_blob()
    if name == "single":          # one prism
        w = W.tiny(n=1, n_layers=1)
        return W.Workload("single", w.vxy, w.tri[:1], np.full((1, 3), -1, np.int32), w.nlayers[:1],
                          w.zlev[:2], w.U[:, :, :1], w.T0[:, :, :1], w.kappa[:1], w.dt, np.zeros(1))
    raise KeyError(name)


def _session(w, precision):
    return P.SlimDG(P.Mesh.from_workload(w, precision))


def _rhs(w, n_comp, seed):
    rng = np.random.default_rng([seed, 21])
    return rng.standard_normal((n_comp, 6, w.n_prisms))


def _reference(kind, w, F, precision):
    Fin = F.astype(np.float32).astype(np.float64) if precision != P.SDG_FP64 else F
    return CD.dv_solve(kind, w.vxy, w.tri, w.nlayers, Fin)


@pytest.mark.parametrize("name", ["single", "ragged", "deep_ragged", "rotating_blob"])
@pytest.mark.parametrize("kind", ["vu", "vd"])
def test_column_dv_parity(name, kind):
    w = _workload(name)
    s = _session(w, P.SDG_FP64)
    for n_comp in (1, 2, 3, 4):
        F = _rhs(w, n_comp, seed=n_comp)
        x = s.column_dv_solve(KINDS[kind], s.scatter(F))
        s.sync()
        err = rel_err(s.gather(x), _reference(kind, w, F, P.SDG_FP64))
        print(name, kind, n_comp, err)
        assert np.all(err <= TOL[P.SDG_FP64]), (n_comp, err)


@pytest.mark.parametrize("precision", [P.SDG_FP32_STATE_FP64_SOLVE, P.SDG_FP32])
@pytest.mark.parametrize("kind", ["vu", "vd"])
def test_column_dv_float_forms(kind, precision):
    w = _workload("deep_ragged")
    s = _session(w, precision)
    F = _rhs(w, 2, seed=7)
    x = s.column_dv_solve(KINDS[kind], s.scatter(F))
    s.sync()
    err = rel_err(s.gather(x), _reference(kind, w, F, precision))
    print(kind, precision, err)
    assert np.all(err <= TOL[precision]), err


@pytest.mark.parametrize("kind", ["vu", "vd"])
def test_column_dv_in_place_and_padding(kind):
    w = _workload("ragged")
    s = _session(w, P.SDG_FP64)
    F = _rhs(w, 2, seed=3)
    buf = s.scatter(F)
    # padding slots hold a sentinel that must survive the call
    live = np.zeros(s.n_slots, dtype=bool)
    live[s.slots_np] = True
    pad = s.torch.from_numpy(~live).to(s.device)
    buf[:, :, pad] = 1234.5
    out = s.column_dv_solve(KINDS[kind], buf, out=buf)
    s.sync()
    assert out.data_ptr() == buf.data_ptr()
    err = rel_err(s.gather(buf), _reference(kind, w, F, P.SDG_FP64))
    assert np.all(err <= TOL[P.SDG_FP64]), err
    assert bool((buf[:, :, pad] == 1234.5).all())


def test_column_dv_argument_errors():
    w = _workload("single")
    s = _session(w, P.SDG_FP64)
    F = s.zeros(1)
    lib, ctx = s.lib, s.ctx
    p = F.data_ptr()
    assert lib.sdg_column_dv_solve(ctx, 2, 1, p, p) == -1
    assert lib.sdg_column_dv_solve(ctx, P.SDG_DV_VU, 0, p, p) == -1
    assert lib.sdg_column_dv_solve(ctx, P.SDG_DV_VU, P.SDG_DV_MAX_COMP + 1, p, p) == -1
    assert lib.sdg_column_dv_solve(ctx, P.SDG_DV_VD, 1, None, p) == -1
    assert lib.sdg_column_dv_solve(ctx, P.SDG_DV_VD, 1, p, p) == 0
    s.sync()


@pytest.fixture(scope="module")
def big():
    return W.four_field_ocean()


@pytest.mark.parametrize("precision", [P.SDG_FP64, P.SDG_FP32_STATE_FP64_SOLVE])
@pytest.mark.parametrize("kind,n_comp", [("vu", 2), ("vd", 1)])
def test_column_dv_four_field_ocean_sampled(big, kind, n_comp, precision):
    """Full size (199,712 columns x 30 layers), checked on 300 sampled columns."""
    w = big
    s = _session(w, precision)
    F = _rhs(w, n_comp, seed=11)
    x = s.column_dv_solve(KINDS[kind], s.scatter(F))
    s.sync()
    rng = np.random.default_rng([4, 21])
    cols = np.sort(rng.choice(w.n_cols, 300, replace=False))
    off = np.concatenate([[0], np.cumsum(w.nlayers)])
    pr = np.concatenate([np.arange(off[c], off[c + 1]) for c in cols])
    got = x[:, :, s.slots[pr]].double().cpu().numpy()
    Fs = F[:, :, pr]
    if precision != P.SDG_FP64:
        Fs = Fs.astype(np.float32).astype(np.float64)
    ref = CD.dv_solve(kind, w.vxy, w.tri[cols], w.nlayers[cols], Fs)
    err = rel_err(got, ref)
    print("four_field_ocean", kind, n_comp, precision, err)
    assert np.all(err <= TOL[precision]), err
