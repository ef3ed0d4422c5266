"""The lagged regularization (reg='lagged': each system's resistance in a
load step raised by eta times its mean slip rate over the previous step,
the rate from the plain Norton law) on the device, through the C-ABI,
against the oracle: FP64 solves of twinned RVEs to 1e-10 (both twin laws,
a ragged grid, a case whose steps alternate), the one-system closed forms,
a batch, save/restore of the raises, reset, FP32 against the FP64 oracle,
and the entry points that reject the option.  The laws here are not stiff
(K = 2000, n = 2): under the lagged reading a plastic step with no raise
runs the plain Norton law, which explicit RK4 integrates stably only for
such laws."""
import dataclasses

import numpy as np
import pytest

import oracle
import rvegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
cp = pytest.importorskip("paper_2402_09996_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cp._lib.lib()
    yield


def _relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _wl(shape=(8, 8, 8), steps=6, eta=2e4, K=2000.0, n=2.0, mode=0, seed=21, per_step=1e-3):
    C, law = rvegen.config_law()
    law = dataclasses.replace(law, slip=dataclasses.replace(law.slip, K=K, n=n),
                              twin=dataclasses.replace(law.twin, K=K, n=n), eta=eta, twin_mode=mode)
    if mode == 1:
        law.K_c, law.f_m = 1.45, 0.8
    rve = rvegen.make_rve(shape, 5, seed, twin_share=0.5)
    S = rvegen.config_systems(with_twins=True)
    return rvegen.Workload("lagged", rve, S, C, law, rvegen.uniaxial_path(per_step * steps, steps))


def _solver(w, precision="fp64", **kw):
    kw.setdefault("tol", 1e-12)
    return cp.Solver(cp.Problem.from_workload(w), precision=precision, reg="lagged", **kw)


FIELDS = ("stress", "strain", "plastic_strain", "acc_slip", "back_strain")


@pytest.mark.parametrize("shape,eta,mode", [((8, 8, 8), 2e4, 0), ((6, 8, 9), 2e4, 1), ((8, 8, 8), 2e5, 0)])
def test_lagged_fp64_parity(shape, eta, mode):
    print("case lagged fp64", shape, eta, mode, flush=True)
    w = _wl(shape, eta=eta, mode=mode)
    gs = _solver(w)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12, reg="lagged")).run(w.path, keep_fields=True)
    print("iters", R["iters"], ref.iters, flush=True)
    assert np.array_equal(R["iters"], ref.iters)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    assert _relerr(R["mean_v"], ref.mean_v) < 1e-10
    assert _relerr(R["mean_f"], ref.mean_f) < 1e-10
    for name in FIELDS:
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-10, name
    # the option changes the solution
    Ri = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12).run(w.path)
    assert _relerr(R["Sigma"], Ri["Sigma"]) > 1e-3
    if eta == 2e5:
        # the steps alternate: the mean stress is not monotone under the
        # monotone load
        assert np.any(np.diff(R["Sigma"][:, 0]) < 0.0)


def _single_system(eta, steps=60):
    E_, nu = 150000.0, 0.3
    lam, mu = E_ * nu / ((1 + nu) * (1 - 2 * nu)), E_ / (2 * (1 + nu))
    C = rvegen.cubic_stiffness(lam + 2 * mu, lam, mu)
    fam = rvegen.FamilyLaw(Q=0.0, b=10.0, c=0.0, d=0.0, K=20000.0, n=1.0, q_self=1.0, q_latent=1.0)
    law = rvegen.Law(slip=fam, twin=rvegen.FamilyLaw(**vars(fam)), eta=eta)
    prob = cp.Problem(np.zeros((2, 2, 2), np.int32), np.array([[0.0, 0.0, 0.0]]), C,
                      np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]), np.array([0], np.int32),
                      np.array([50.0]), law)
    t = np.linspace(0.0, steps * 0.5, steps + 1)
    target = np.zeros((steps, 6))
    target[:, 5] = 1e-3 * t[1:]
    path = rvegen.LoadPath(t=t, strain_ctrl=np.ones((steps, 6), np.uint8), target=target)
    return prob, path


def test_lagged_single_system_closed_forms():
    """One slip system, n = 1, imposed shear rate dE12/dt = 1e-3 (slip rate
    2e-3 at steady state): with eta < K the steps reach tau = tau0 + (K +
    eta) 2e-3 = 98 MPa; with eta >> K they alternate between exactly zero
    slip and slip at twice the imposed rate."""
    print("case lagged single system", flush=True)
    prob, path = _single_system(4000.0)
    R = cp.Solver(prob, precision="fp64", tol=1e-12, rk4_M=4, reg="lagged").run(path)
    assert R["Sigma"][-1, 5] == pytest.approx(98.0, rel=1e-9)
    assert np.allclose(np.diff(R["mean_v"])[-5:] / 0.5, 2e-3, rtol=1e-9)
    prob, path = _single_system(2e5)
    R = cp.Solver(prob, precision="fp64", tol=1e-12, rk4_M=4, reg="lagged").run(path)
    rate = np.diff(R["mean_v"])[-20:] / 0.5
    zero, slip = (rate[0::2], rate[1::2]) if rate[0] < rate[1] else (rate[1::2], rate[0::2])
    assert np.all(zero == 0.0)
    assert np.allclose(slip, 4e-3, rtol=1e-9)


def test_lagged_batch_matches_single_solves():
    print("case lagged batch", flush=True)
    ws = [_wl((8, 8, 8), seed=21), _wl((6, 8, 9), seed=22)]
    b = cp.Solver([cp.Problem.from_workload(w) for w in ws], precision="fp64", tol=1e-12, reg="lagged")
    path = ws[0].path
    outs = [b.step_batch(path, n) for n in range(path.n_steps)]
    for i, w in enumerate(ws):
        gs = _solver(w)
        R = gs.run(path)
        assert np.array_equal([o[i]["iters"] for o in outs], R["iters"])
        assert _relerr([o[i]["Sigma"] for o in outs], R["Sigma"]) < 1e-13
        for name in ("stress", "acc_slip"):
            assert _relerr(b.field_of(i, name).cpu().numpy(), gs.field(name).cpu().numpy()) < 1e-13, name


def _run_from(s, path, first):
    return [s.step(path, n) for n in range(first, path.n_steps)]


def test_lagged_state_restore_carries_the_raises_and_reset_clears_them():
    """The raises of the next step are part of the saved state: a fresh
    solver restored from a state saved after three steps continues exactly
    as the solver that saved it (a fresh solver starts with no raise, so a
    state without them would continue differently); reset clears them."""
    print("case lagged state", flush=True)
    w = _wl(steps=6)
    a = _solver(w)
    first = _run_from(a, w.path, 0)
    a.reset()
    for n in range(3):
        a.step(w.path, n)
    saved = a.save_state().clone()
    cont = _run_from(a, w.path, 3)
    for x, y in zip(cont, first[3:]):
        assert np.array_equal(x["Sigma"], y["Sigma"]) and x["iters"] == y["iters"]
    b = _solver(w)
    b.restore_state(saved)
    again = _run_from(b, w.path, 3)
    for x, y in zip(again, cont):
        assert np.array_equal(x["Sigma"], y["Sigma"]) and x["iters"] == y["iters"]
    assert np.array_equal(a.field("acc_slip").cpu().numpy(), b.field("acc_slip").cpu().numpy())


@pytest.mark.parametrize("graph_iters", [3, "adaptive"])
def test_lagged_graph_replays_equal_direct_launches(graph_iters):
    """The raises are written at commit, outside the captured iterations:
    graph replays give the direct launches' results bit for bit."""
    print("case lagged graphs", graph_iters, flush=True)
    w = _wl(steps=5)
    Rd = _solver(w, "fp32", tol=1e-6, stag_tol=1e-4).run(w.path)
    Rg = _solver(w, "fp32", tol=1e-6, stag_tol=1e-4, graph_iters=graph_iters).run(w.path)
    assert np.array_equal(Rd["iters"], Rg["iters"])
    assert np.array_equal(Rd["Sigma"], Rg["Sigma"])
    assert np.array_equal(Rd["mean_v"], Rg["mean_v"])


def test_lagged_cut_back_like_the_oracle():
    """Load steps of 2e-3 with at most 40 iterations: every step is cut
    back (2-3 failed attempts), and each committed half step sets the raises
    of the next from its own slip and duration; retries, iterations and
    fields as the oracle's."""
    print("case lagged cut-back", flush=True)
    w = _wl(steps=4, per_step=2e-3)
    gs = _solver(w, tol=1e-10, max_iter=40, cutback=5)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-10, reg="lagged", max_iter=40, cutback=5)).run(
        w.path, keep_fields=True)
    print("cutbacks", R["cutbacks"], ref.cutbacks, "iters", R["iters"], ref.iters, flush=True)
    assert np.all(ref.cutbacks >= 1)
    assert np.array_equal(R["cutbacks"], ref.cutbacks)
    assert np.array_equal(R["iters"], ref.iters)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    for name in FIELDS:
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-10, name


def test_state_of_the_other_reading_is_rejected():
    """A state saved under one regularization reading is rejected by a
    solver of the other before anything is copied (the lagged state holds
    one more section, so the buffers differ in size)."""
    w = _wl(steps=2)
    imp = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12)
    lag = _solver(w)
    imp.step(w.path, 0)
    lag.step(w.path, 0)
    s_imp, s_lag = imp.save_state(), lag.save_state()
    assert s_lag.numel() > s_imp.numel()
    with pytest.raises(cp.CpfError):
        lag.restore_state(s_imp)
    with pytest.raises(cp.CpfError):
        imp.restore_state(s_lag)
    lag.restore_state(s_lag)          # its own state is accepted


def test_lagged_fp32_against_fp64_oracle():
    print("case lagged fp32", flush=True)
    w = _wl(steps=6)
    gs = _solver(w, "fp32", tol=1e-6, stag_tol=1e-4)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-10, reg="lagged")).run(w.path, keep_fields=True)
    assert np.all(R["status"] == 0)
    assert np.abs(R["Sigma"] - ref.Sigma).max() / np.abs(ref.Sigma[:, 0]).max() < 1e-4
    for name in ("stress", "plastic_strain", "acc_slip"):
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-3, name


def test_lagged_rejected_where_not_supported():
    w = _wl(steps=2)
    gs = _solver(w)
    with pytest.raises(cp.CpfError):
        gs.adjoint_workspace_size(w.path)
    z = torch.zeros((6,) + w.rve.labels.shape, dtype=torch.float64)
    st = torch.zeros((6 + 2 * w.systems.family.shape[0],) + w.rve.labels.shape, dtype=torch.float64)
    with pytest.raises(cp.CpfError):
        gs.constitutive(z, z, st, 0.5, 4)
    with pytest.raises(cp.CpfError):
        _solver(w, rk_tol=1e-6)
    with pytest.raises(cp.CpfError):
        _solver(w, aa_depth=2)
