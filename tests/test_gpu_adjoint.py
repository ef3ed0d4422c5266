"""Discrete adjoint on the device: the gradient of the effective stress
loss with respect to the 14 law parameters matches the FP64 oracle's
adjoint (itself pinned to finite differences on the CPU), central
differences of the device's own forward solves, and does not depend on
the checkpoint interval; the torch.autograd binding returns the same
gradient."""
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


def _case(shape=(4, 4, 6), grains=3, seed=77, steps=3, total=0.006, twin_mode=rvegen.TWIN_NORTON):
    C, law = rvegen.config_law()
    law.twin_mode = twin_mode
    if twin_mode == rvegen.TWIN_PAPER:
        law.K_c, law.f_m = 1.45, 0.8
    S = rvegen.config_systems(True)
    rve = rvegen.make_rve(shape, grains, seed, twin_share=0.5)
    path = rvegen.uniaxial_path(total, steps, rate=1e-2)
    return rvegen.Workload("adj", rve, S, C, law, path)


def _theta(w):
    return np.array([[80.0] + [getattr(w.law.slip, k) for k in ("Q", "b", "c", "d", "K", "n")],
                     [120.0] + [getattr(w.law.twin, k) for k in ("Q", "b", "c", "d", "K", "n")]])


def _target(w):
    sv = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12)
    return sv.run(w.path)["Sigma"][:, 0] * 1.03


@pytest.mark.parametrize("twin_mode", [rvegen.TWIN_NORTON, rvegen.TWIN_PAPER])
def test_adjoint_matches_oracle_fp64(twin_mode):
    w = _case(twin_mode=twin_mode)
    tgt = _target(w)
    print("adjoint vs oracle, twin_mode", twin_mode, flush=True)
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12)
    L, g, sxx = s.gradient(w.path, tgt, checkpoint_every=2, adj_tol=1e-12)
    Lo, go, so = oracle.solver_for(w, oracle.Options(tol=1e-12)).gradient(w.path, tgt, adj_tol=1e-12)
    assert np.abs(sxx - so).max() <= 1e-10 * np.abs(so).max()
    assert L == pytest.approx(Lo, rel=1e-9)
    for f in (0, 1):
        scale = np.abs(go[f]).max()
        assert scale > 0
        assert np.abs(g[f] - go[f]).max() <= 1e-9 * scale, (f, g[f], go[f])


def test_adjoint_independent_of_checkpoint_interval():
    """Recomputation from checkpoints replays the same deterministic
    forward steps, so every interval (1, a ragged 2 of 5, all) gives the
    same numbers bit for bit."""
    w = _case(shape=(8, 8, 8), grains=5, seed=5, steps=5, total=0.008)
    tgt = _target(w)
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-10)
    res = []
    for c in (1, 2, 5):
        res.append(s.gradient(w.path, tgt, checkpoint_every=c, adj_tol=1e-10))
        st = s.adjoint_stats()
        assert st["recomputed_steps"] == 5 - (5 + c - 1) // c
        assert st["adjoint_iterations"] > 0 and st["forward_iterations"] > 0
    for L, g, sxx in res[1:]:
        assert L == res[0][0]
        assert np.array_equal(g, res[0][1])
        assert np.array_equal(sxx, res[0][2])
    # the solver is back at the undeformed state
    assert float(s.field("strain").abs().max()) == 0.0


def test_adjoint_matches_device_finite_differences():
    w = _case(shape=(8, 8, 8), grains=5, seed=5, steps=4, total=0.008)
    tgt = _target(w)
    base = cp.Problem.from_workload(w)
    s = cp.Solver(base, precision="fp64", tol=1e-12)
    L, g, _ = s.gradient(w.path, tgt, checkpoint_every=2, adj_tol=1e-12)
    theta = _theta(w)

    def loss(th):
        sv = cp.Solver(cp.with_theta(base, th), precision="fp64", tol=1e-12)
        return float(np.sum((sv.run(w.path)["Sigma"][:, 0] - tgt) ** 2))

    for f, k in [(0, 0), (0, 1), (0, 3), (0, 5), (0, 6), (1, 0), (1, 5)]:
        h = 1e-5 * max(abs(theta[f, k]), 1.0)
        tp, tm = theta.copy(), theta.copy()
        tp[f, k] += h
        tm[f, k] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        print("fd", f, k, fd, g[f, k], flush=True)
        assert abs(g[f, k] - fd) <= 1e-5 * abs(fd) + 1e-7 * np.abs(g).max(), (f, k, g[f, k], fd)


def test_adjoint_fp32_close_to_fp64():
    w = _case(shape=(8, 8, 8), grains=5, seed=5, steps=4, total=0.008)
    tgt = _target(w)
    p = cp.Problem.from_workload(w)
    L64, g64, _ = cp.Solver(p, precision="fp64", tol=1e-10).gradient(w.path, tgt, adj_tol=1e-10)
    L32, g32, _ = cp.Solver(p, precision="fp32", tol=1e-6, stag_tol=1e-4).gradient(
        w.path, tgt, adj_tol=1e-6)
    print("fp32 vs fp64", L32, L64, np.abs(g32 - g64).max() / np.abs(g64).max(), flush=True)
    assert L32 == pytest.approx(L64, rel=1e-4)
    assert np.abs(g32 - g64).max() <= 1e-4 * np.abs(g64).max()


def test_autograd_binding():
    w = _case()
    tgt = _target(w)
    p = cp.Problem.from_workload(w)
    theta = torch.tensor(_theta(w), dtype=torch.float64, requires_grad=True)
    opts = dict(precision="fp64", tol=1e-12, adj_tol=1e-12, checkpoint_every=10)
    L = cp.StressCurveLoss.apply(theta, p, w.path, tgt, opts)
    (3.0 * L).backward()
    L2, g2, _ = cp.Solver(p, precision="fp64", tol=1e-12).gradient(w.path, tgt, adj_tol=1e-12)
    assert float(L.detach()) == L2
    assert np.array_equal(theta.grad.numpy(), 3.0 * g2)


def test_adjoint_argument_errors():
    w = _case()
    tgt = _target(w)
    p = cp.Problem.from_workload(w)
    s = cp.Solver(p, precision="fp64")
    with pytest.raises(ValueError):
        s.gradient(w.path, tgt[:-1])
    with pytest.raises(cp.CpfError):
        s.gradient(w.path, tgt, checkpoint_every=0)
    with pytest.raises(cp.CpfError):
        s.gradient(w.path, tgt, adj_tol=0.0)
    b = cp.Solver([p, p], precision="fp64")
    with pytest.raises(cp.CpfError):
        b.gradient(w.path, tgt)


def test_vjp_general_cotangent_matches_oracle():
    """A cotangent on all six mean-stress components (shear included)."""
    w = _case()
    sb = np.random.default_rng(3).standard_normal((w.path.n_steps, 6))
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12)
    g, sig = s.vjp(w.path, sb, checkpoint_every=2, adj_tol=1e-12)
    go, so = oracle.solver_for(w, oracle.Options(tol=1e-12)).vjp(w.path, sb, adj_tol=1e-12)
    assert np.abs(sig - so).max() <= 1e-10 * np.abs(so).max()
    for f in (0, 1):
        assert np.abs(g[f] - go[f]).max() <= 1e-9 * np.abs(go[f]).max(), (f, g[f], go[f])
    # the stress-curve loss is the cotangent 2 (Sigma_11 - target) e_11
    tgt = sig[:, 0] * 1.03
    L, g2, _ = s.gradient(w.path, tgt, checkpoint_every=2, adj_tol=1e-12)
    cot = np.zeros_like(sb)
    cot[:, 0] = 2 * (sig[:, 0] - tgt)
    g3, _ = s.vjp(w.path, cot, checkpoint_every=2, adj_tol=1e-12)
    assert np.array_equal(g2, g3)


def test_effective_stress_autograd():
    """Any torch loss of the mean stress history: the backward is the
    device VJP with the loss's cotangent."""
    w = _case()
    p = cp.Problem.from_workload(w)
    theta = torch.tensor(_theta(w), dtype=torch.float64, requires_grad=True)
    opts = dict(precision="fp64", tol=1e-12, adj_tol=1e-12, checkpoint_every=2)
    sig = cp.EffectiveStress.apply(theta, p, w.path, opts)
    assert sig.shape == (w.path.n_steps, 6)
    wts = torch.tensor([1.0, 0.5, 0.5, 2.0, 2.0, 2.0], dtype=torch.float64)
    loss = ((sig - 0.9 * sig.detach()) ** 2 * wts).sum()
    loss.backward()
    cot = (2 * (sig.detach() - 0.9 * sig.detach()) * wts).numpy()
    g, _ = cp.Solver(p, precision="fp64", tol=1e-12).vjp(w.path, cot, checkpoint_every=2, adj_tol=1e-12)
    assert np.array_equal(theta.grad.numpy(), g)


def test_vjp_argument_errors():
    w = _case()
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp64")
    with pytest.raises(ValueError):
        s.vjp(w.path, np.zeros((w.path.n_steps, 5)))
    bad = np.zeros((w.path.n_steps, 6))
    bad[1, 2] = np.nan
    with pytest.raises(cp.CpfError):
        s.vjp(w.path, bad)


def test_autograd_on_the_paper_systems_keeps_per_system_tau0():
    """Table 1 with the paper's resistances (130 MPa ordinary, 200 MPa
    superdislocations, 130 MPa twins): at theta_of(problem) the autograd
    forward is the plain solve, and the r0 gradient is the derivative of a
    uniform shift of the family's resistances (central differences)."""
    C, law = rvegen.paper_law()
    S = rvegen.table1_systems(True)
    rve = rvegen.make_rve((4, 4, 6), 3, 77, twin_share=0.5)
    path = rvegen.uniaxial_path(0.006, 3, rate=1e-2)
    w = rvegen.Workload("adj_paper", rve, S, C, law, path)
    p = cp.Problem.from_workload(w)
    th0 = cp.theta_of(p)
    assert th0[0, 0] == 130.0 and th0[1, 0] == 130.0
    plain = cp.Solver(p, precision="fp64", tol=1e-12).run(path)["Sigma"]
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    opts = dict(precision="fp64", tol=1e-12, adj_tol=1e-12, checkpoint_every=2)
    sig = cp.EffectiveStress.apply(theta, p, path, opts)
    assert np.array_equal(sig.detach().numpy(), plain)
    sig[:, 0].sum().backward()
    g = theta.grad.numpy()

    def j(th):
        return float(cp.Solver(cp.with_theta(p, th), precision="fp64", tol=1e-12).run(path)["Sigma"][:, 0].sum())

    for f in (0, 1):
        tp, tm = th0.copy(), th0.copy()
        tp[f, 0] += 1e-3
        tm[f, 0] -= 1e-3
        fd = (j(tp) - j(tm)) / 2e-3
        print("r0 family", f, "adjoint", g[f, 0], "fd", fd, flush=True)
        assert abs(g[f, 0] - fd) <= 1e-5 * abs(fd) + 1e-8 * np.abs(g).max()
