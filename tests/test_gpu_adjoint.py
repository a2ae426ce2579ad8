"""GPU tests of the hand-written adjoint (through the C ABI and the
torch.autograd wrappers): parity with the oracle's sparse-matrix adjoint on
small meshes, invariance to the checkpoint interval, and central finite
differences of the GPU forward objective on a larger mesh."""

import numpy as np
import pytest

import oracle as O
import oracle.adjoint as OA
import paper_2605_16082_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def rel(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _case(name):
    """Small meshes with a stiff vertical diffusion (kappa dt / dz^2 from 1 to
    ~280) so that the column solve matters, at the stable advective dt."""
    if name == "tiny":
        w = W.tiny(n_fields=2)
        w.kappa = w.kappa * 1000.0
    elif name == "ragged":
        w = W.ragged(n=6, n_fields=1)
        w.kappa = w.kappa * 300.0
    else:
        w = W.rotating_blob(n=6, n_layers=4)
        w.kappa = w.kappa * 100.0
    return w, O.PrismMesh(w.vxy, w.tri, w.nbr, w.nlayers, w.zlev)


def _gpu_gradient(w, n_steps, every):
    import torch
    s, U, kappa, state = P.from_workload(w)
    T0 = s.scatter(w.T0).requires_grad_(True)
    kap = torch.as_tensor(w.kappa, dtype=torch.float64, device=s.device).requires_grad_(True)
    xN = P.TracerSteps.apply(T0, kap, s, n_steps, every)
    J = P.MNorm.apply(xN, s)
    J.backward()
    return float(J), s.gather(T0.grad), kap.grad.detach().cpu().numpy(), s


def assert_kappa_gradient(gk, gkr, gk_abs):
    """dJ/dkappa_l = sum_n dt mu_n^T A_l x^{n+1} is a cancelling sum: each
    layer's total may be thousands of times smaller than the sum of its
    terms' magnitudes (gk_abs, from the oracle), and rounding in the terms
    moves it relative to that sum.  The bar is 1e-12 of it, per layer."""
    bound = 1e-12 * gk_abs
    assert np.all(np.abs(gk - gkr) <= bound), (np.abs(gk - gkr) / gk_abs).max()


def test_mass_apply_and_m_dot():
    w, m = _case("rotating_blob")
    s, U, kappa, state = P.from_workload(w)
    Mp = O.mass_matrix(m)
    ref = np.einsum("nij,fjn->fin", Mp, w.T0)
    got = s.gather(s.apply_mass(state))
    assert rel(got, ref) <= 1e-13
    back = s.gather(s.apply_mass(s.apply_mass(state), inverse=True))
    assert rel(back, w.T0) <= 1e-12
    md = s.m_dot(state, state).sum()
    assert abs(md - float(np.einsum("fin,fin->", ref, w.T0))) <= 1e-12 * abs(md)


def test_adjoint_rejects_x_next_written_by_the_solve():
    """With dkappa the kappa gradient reads x_next after the transposed solve
    has overwritten z_out, so the two may not be one buffer; the call fails
    before any launch."""
    import torch
    w, m = _case("tiny")
    s, U, kappa, state = P.from_workload(w)
    z = s.new_state()
    dk = torch.zeros(64, dtype=torch.float64, device=s.device)
    with pytest.raises(P.SlimDGError):
        s.step_adjoint(z, z, z, dk)
    s.step_adjoint(z, z, z, None)          # without dkappa x_next is not read
    s.sync()


@pytest.mark.parametrize("name", ["tiny", "ragged", "rotating_blob"])
def test_adjoint_gradient_matches_oracle(name):
    w, m = _case(name)
    n_steps = 3
    J, gT, gk, s = _gpu_gradient(w, n_steps, 2)
    Jr, gTr, gkr, gka = OA.gradient(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n_steps, w.penalty, return_scale=True)
    print(name, "J", J, Jr, "dT0", rel(gT, gTr), "dkappa", rel(gk, gkr),
          "dkappa / term magnitudes", (np.abs(gk - gkr) / gka).max())
    assert abs(J - Jr) <= 1e-12 * abs(Jr)
    assert rel(gT, gTr) <= 1e-12
    assert_kappa_gradient(gk, gkr, gka)


def _golden_long_horizon():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "adjoint_rotating_blob_200steps.txt")
    rec = {"dkappa": [], "dT0": []}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        if k in rec:
            rec[k].append([float(x) for x in v])
        else:
            rec[k] = float(v[0])
    return rec


def test_adjoint_long_horizon_matches_oracle():
    """200 steps of the rotating-blob workload (1,800 triangles x 10 layers), a
    checkpoint every 20: the GPU gradient against the oracle's, stored by
    tests/golden/make_adjoint_rotating_blob.py (dJ/dkappa per layer, and
    dJ/dT0 through its maximum, its 2-norm and 4,160 sampled entries)."""
    g = _golden_long_horizon()
    w = W.rotating_blob()
    J, gT, gk, s = _gpu_gradient(w, 200, 20)
    gT = gT[0].ravel()
    dk = np.array(g["dkappa"])
    samp = np.array(g["dT0"])
    idx = samp[:, 0].astype(np.int64)
    e_s = np.abs(gT[idx] - samp[:, 1]).max() / g["dT0_max"]
    print("J", J, g["J"], "dT0 sampled", e_s, "max", np.abs(gT).max() / g["dT0_max"] - 1,
          "norm", np.sqrt(np.sum(gT * gT)) / g["dT0_norm2"] - 1,
          "dkappa / term magnitudes", (np.abs(gk - dk[:, 1]) / dk[:, 2]).max())
    assert abs(J - g["J"]) <= 1e-12 * g["J"]
    assert e_s <= 1e-12
    assert abs(np.abs(gT).max() - g["dT0_max"]) <= 1e-12 * g["dT0_max"]
    assert abs(np.sqrt(np.sum(gT * gT)) - g["dT0_norm2"]) <= 1e-12 * g["dT0_norm2"]
    assert_kappa_gradient(gk, dk[:, 1], dk[:, 2])


def test_adjoint_blob_gradient_matches_oracle():
    """The differentiation configuration in full (49,928 triangles x 20
    layers, 998,560 prisms; 200 steps, a checkpoint every 20): the GPU
    gradient against the oracle's, stored by
    tests/golden/make_adjoint_blob_reference.py (J; dJ/dkappa per layer with
    its magnitude sums; dJ/dT0 through its maximum, its 2-norm and 20,064
    sampled entries)."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "adjoint_blob_200steps.npz"))
    w = W.adjoint_blob()
    J, gT, gk, s = _gpu_gradient(w, int(g["steps"]), 20)
    gT = gT[0].ravel()
    e_s = np.abs(gT[g["idx"]] - g["vals"]).max() / float(g["dT0_max"])
    print("J", J, float(g["J"]), "dT0 sampled", e_s, "max", np.abs(gT).max() / float(g["dT0_max"]) - 1,
          "norm", np.sqrt(np.sum(gT * gT)) / float(g["dT0_norm2"]) - 1,
          "dkappa / term magnitudes", (np.abs(gk[:len(g["dkappa"])] - g["dkappa"]) / g["dkappa_abs"]).max())
    assert abs(J - float(g["J"])) <= 1e-12 * float(g["J"])
    assert e_s <= 1e-12
    assert abs(np.abs(gT).max() - float(g["dT0_max"])) <= 1e-12 * float(g["dT0_max"])
    assert abs(np.sqrt(np.sum(gT * gT)) - float(g["dT0_norm2"])) <= 1e-12 * float(g["dT0_norm2"])
    assert_kappa_gradient(gk[:len(g["dkappa"])], g["dkappa"], g["dkappa_abs"])


def test_checkpoint_interval_does_not_change_gradient():
    w, m = _case("ragged")
    ref = None
    for every in (1, 3, 7):
        J, gT, gk, s = _gpu_gradient(w, 7, every)
        if ref is None:
            ref = (gT, gk)
        else:
            assert np.array_equal(gT, ref[0]) and np.array_equal(gk, ref[1]), every


def test_adjoint_matches_finite_differences_on_gpu():
    """Directional derivatives against central differences (eps = 1e-6) of
    the GPU forward objective, on a 7,200-column x 12-layer mesh."""
    import torch
    w = W.rotating_blob(n=60, n_layers=12)
    w.kappa = np.geomspace(1e-2, 1e-5, 12)
    w.dt *= 2.0
    n_steps, every = 30, 10
    J, gT, gk, s = _gpu_gradient(w, n_steps, every)

    def objective(T0_nat, kap_np):
        st = s.scatter(T0_nat)
        kt = torch.as_tensor(kap_np, dtype=torch.float64, device=s.device)
        s.set_diffusivity(kt)
        s.set_fields(st)
        s.step(n_steps)
        return float(np.sqrt(s.m_dot(st, st).sum()))

    assert abs(objective(w.T0, w.kappa) - J) <= 1e-13 * J
    rng = np.random.default_rng(17)
    eps = 1e-6
    for trial in range(3):
        d = rng.standard_normal(w.T0.shape)
        d /= np.abs(d).max()
        fd = (objective(w.T0 + eps * d, w.kappa) - objective(w.T0 - eps * d, w.kappa)) / (2 * eps)
        ad = float(np.sum(gT * d))
        print("T0 dir", trial, fd, ad)
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J
        dk = rng.standard_normal(w.kappa.shape) * w.kappa
        fd = (objective(w.T0, w.kappa + eps * dk) - objective(w.T0, w.kappa - eps * dk)) / (2 * eps)
        ad = float(np.sum(gk * dk))
        print("kappa dir", trial, fd, ad)
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J


def test_adjoint_blob_gradient_finite_differences():
    """The differentiation configuration in full: 49,928 triangles x 20
    layers, 200 steps, a checkpoint every 20; 20 seeded directions for the
    initial field and 20 for the per-layer diffusivity, central differences
    with eps = 1e-6 of the GPU forward objective; pass when
    |FD - grad.d| <= 1e-6 |grad.d| + 1e-10 J.

    J moves by only ~1e-12 J over a kappa step, near the rounding of J
    itself, so the difference J+ - J- is formed without cancellation:
    J+^2 - J-^2 = (x+ - x-)^T M (x+ + x-), subtracted slot by slot before
    the sum, divided by J+ + J-."""
    import torch
    w = W.adjoint_blob()
    n_steps, every = w.n_steps, 20
    J, gT, gk, s = _gpu_gradient(w, n_steps, every)
    st = s.new_state()

    def final_state(T0_nat, kap_np):
        s.scatter(T0_nat, out=st)
        s.set_diffusivity(torch.as_tensor(kap_np, dtype=torch.float64, device=s.device))
        s.set_fields(st)
        s.step(n_steps)
        return st.clone()

    def norm(x):
        return float(np.sqrt(s.m_dot(x, x).sum()))

    def central_difference(xp, xm, eps):
        d2 = float(((xp - xm) * s.apply_mass(xp + xm)).sum())
        return d2 / (norm(xp) + norm(xm)) / (2 * eps)

    assert abs(norm(final_state(w.T0, w.kappa)) - J) <= 1e-13 * J
    rng = np.random.default_rng(2605)
    eps = 1e-6
    worst = 0.0
    for trial in range(20):
        d = rng.standard_normal(w.T0.shape)
        d /= np.abs(d).max()
        fd = central_difference(final_state(w.T0 + eps * d, w.kappa), final_state(w.T0 - eps * d, w.kappa), eps)
        ad = float(np.sum(gT * d))
        worst = max(worst, abs(fd - ad) / abs(ad))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("T0", trial, fd, ad)
    for trial in range(20):
        dk = rng.standard_normal(w.kappa.shape) * w.kappa
        fd = central_difference(final_state(w.T0, w.kappa + eps * dk), final_state(w.T0, w.kappa - eps * dk), eps)
        ad = float(np.sum(gk * dk))
        worst = max(worst, abs(fd - ad) / abs(ad))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-10 * J, ("kappa", trial, fd, ad)
    print("adjoint_blob J", J, "worst relative FD mismatch", worst)


def _gpu_gradient_imex(w, n_steps, every, okubo_scale=0.0):
    import torch
    s, U, kappa, state = P.from_workload(w, time_scheme=P.SDG_SCHEME_SPLIT_IMEX, okubo_scale=okubo_scale)
    T0 = s.scatter(w.T0).requires_grad_(True)
    kap = torch.as_tensor(w.kappa, dtype=torch.float64, device=s.device).requires_grad_(True)
    xN = P.TracerSteps.apply(T0, kap, s, n_steps, every)
    J = P.MNorm.apply(xN, s)
    J.backward()
    return float(J), s.gather(T0.grad), kap.grad.detach().cpu().numpy(), s


@pytest.mark.parametrize("name,okubo", [("tiny", 0.0), ("ragged", 0.0), ("rotating_blob", 0.0), ("ragged", 50.0)])
def test_imex_adjoint_matches_oracle(name, okubo):
    from oracle.horizontal_diffusion import okubo_diffusivity
    w, m = _case(name)
    n_steps = 3
    J, gT, gk, s = _gpu_gradient_imex(w, n_steps, 2, okubo)
    kh = okubo_diffusivity(m, okubo) if okubo > 0 else None
    Jr, gTr, gkr, gka = OA.gradient_imex(m, w.U, w.kappa, w.T0, w.dt, w.t_ext, n_steps, w.penalty, kh,
                                         return_scale=True)
    print(name, okubo, "J", J, Jr, "dT0", rel(gT, gTr), "dkappa", rel(gk, gkr),
          "dkappa / term magnitudes", (np.abs(gk - gkr) / gka).max())
    assert abs(J - Jr) <= 1e-12 * abs(Jr)
    assert rel(gT, gTr) <= 1e-12
    assert_kappa_gradient(gk, gkr, gka)


@pytest.mark.parametrize("okubo", [0.0, 50.0])
def test_imex_reverse_step_from_kept_half_state(okubo):
    """sdg_step_keep_half + sdg_step_adjoint_imex_half (x_h kept by the
    forward step) give bitwise what sdg_step + sdg_step_adjoint_imex (x_h
    rebuilt from the state before the step) give, over three steps; the kept
    step advances the state exactly as sdg_step does."""
    import torch
    w, m = _case("ragged")
    s, U, kappa, state = P.from_workload(w, time_scheme=P.SDG_SCHEME_SPLIT_IMEX, okubo_scale=okubo)
    x0 = state.clone()
    xs_prev, xs_half = [], []
    for _ in range(3):
        xs_prev.append(state.clone())
        s.step(1)
    after = state.clone()
    state.copy_(x0)
    for _ in range(3):
        xh = s.new_state()
        s.step_keep_half(xh)
        xs_half.append(xh)
    assert torch.equal(state, after)
    rng = np.random.default_rng(11)
    z1 = s.scatter(rng.standard_normal(w.T0.shape))
    z2 = z1.clone()
    dk1 = torch.zeros(64, dtype=torch.float64, device=s.device)
    dk2 = torch.zeros_like(dk1)
    for j in range(2, -1, -1):
        zn = s.new_state()
        s.step_adjoint_imex(z1, zn, xs_prev[j], dk1)
        z1 = zn
        zn = s.new_state()
        s.step_adjoint_imex_half(z2, zn, xs_half[j], dk2)
        z2 = zn
    assert torch.equal(z1, z2) and torch.equal(dk1, dk2)
    with pytest.raises(P.SlimDGError):
        s.step_keep_half(state)              # the set fields themselves


def test_imex_checkpoint_interval_does_not_change_gradient():
    w, m = _case("ragged")
    ref = None
    for every in (1, 3, 7):
        J, gT, gk, s = _gpu_gradient_imex(w, 7, every)
        if ref is None:
            ref = (gT, gk)
        else:
            assert np.array_equal(gT, ref[0]) and np.array_equal(gk, ref[1]), every


def test_imex_adjoint_argument_errors():
    w, m = _case("tiny")
    s, U, kappa, state = P.from_workload(w, time_scheme=P.SDG_SCHEME_SPLIT_IMEX)
    z = s.new_state()
    with pytest.raises(P.SlimDGError) as e:
        s.step_adjoint_imex(z, z, state)           # z_out aliases z_next
    assert e.value.status == -1
    lie, _, _, lstate = P.from_workload(w)
    with pytest.raises(P.SlimDGError) as e:
        lie.step_adjoint_imex(lie.new_state(), lie.new_state(), lstate)
    assert e.value.status == -5
