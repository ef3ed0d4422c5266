"""Failure handling on the device, through the C-ABI, against the oracle:
the per-step count of Section 4's local-stress condition (FP64, count for
count), a diverging load step reported as CPF_E_NAN, and the same step
completed by cut-back into the oracle's half steps (FP64 to 1e-10 with the
same iterations and retries)."""
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


@pytest.mark.parametrize("shape,steps,per_step", [((6, 8, 9), 4, 1e-3), ((8, 8, 8), 4, 1e-3), ((8, 8, 8), 3, 2e-3)])
def test_symptom_counts_match_oracle(shape, steps, per_step):
    print("case symptom", shape, steps, per_step, flush=True)
    C, law = rvegen.config_law()
    rve = rvegen.make_rve(shape, 5, 21, twin_share=0.5)
    S = rvegen.config_systems(with_twins=True)
    w = rvegen.Workload("s", rve, S, C, law, rvegen.uniaxial_path(per_step * steps, steps))
    R = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12).run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12)).run(w.path)
    print("counts", R["n_symptom"], "oracle", ref.n_symptom, flush=True)
    assert np.array_equal(R["n_symptom"], ref.n_symptom)
    assert np.array_equal(R["cutbacks"], np.zeros(steps, np.int64))


def _stiff_step_workload(strain=2e-3):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve((4, 4, 4), 3, 4)
    S = rvegen.config_systems(with_twins=False)
    return rvegen.Workload("cb", rve, S, C, law, rvegen.uniaxial_path(strain, 1))


def test_diverging_step_reported_then_cut_back_like_the_oracle():
    w = _stiff_step_workload()
    print("case cut-back 4^3", flush=True)
    with pytest.raises(cp.CpfError) as e:
        cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-10, rk4_M=1).run(w.path)
    assert e.value.code in (cp._lib.CPF_E_NAN, cp._lib.CPF_E_NOT_CONVERGED)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-10, rk4_M=1, cutback=6)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-10, M=1, cutback=6)).run(w.path, keep_fields=True)
    print("cutbacks", R["cutbacks"], ref.cutbacks, "iters", R["iters"], ref.iters, flush=True)
    assert R["cutbacks"][0] >= 1
    assert np.array_equal(R["cutbacks"], ref.cutbacks)
    assert np.array_equal(R["iters"], ref.iters)
    assert np.array_equal(R["n_symptom"], ref.n_symptom)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    for name in ("stress", "strain", "plastic_strain", "acc_slip"):
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-10, name
    with pytest.raises(cp.CpfError):
        cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-10, rk4_M=1, cutback=21)


def test_nan_injected_into_the_committed_state_is_reported():
    """A non-finite value restored into the committed state makes the next
    load step end with CPF_E_NAN, also where it never reaches the stress:
    the end of the last state component (the back strain of the last twin
    system, inactive in these voxels) and, separately, the start of the
    plastic strain; the state saved before continues normally."""
    C, law = rvegen.config_law()
    rve = rvegen.make_rve((8, 8, 8), 4, 9, twin_share=0.5)
    S = rvegen.config_systems(with_twins=True)
    w = rvegen.Workload("nan", rve, S, C, law, rvegen.uniaxial_path(3e-3, 3))
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-10)
    s.step(w.path, 0)
    good = s.save_state().clone()
    nv, D = 512, 6 + 2 * 16
    start = good.numel() // 8 - D * nv           # the state section ends the buffer (no padding here)
    for sl in (slice(-32, None), slice(start, start + 32)):
        bad = good.clone()
        bad.view(torch.float64)[sl] = float("nan")
        s.restore_state(bad)
        with pytest.raises(cp.CpfError) as e:
            s.step(w.path, 1)
        assert e.value.code == cp._lib.CPF_E_NAN
    s.restore_state(good)
    o = s.step(w.path, 1)
    assert o["status"] == 0 and np.all(np.isfinite(o["Sigma"]))
