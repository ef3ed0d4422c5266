"""Frozen error-controlled substep counts on the device against the oracle:
FP64 solves (1e-10, same iteration counts, the same per-voxel counts),
reduction to the fixed count when every voxel passes, FP32 accuracy,
batches, and the argument checks (the adjoint needs fixed counts)."""
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


def _w(shape=(6, 6, 6), grains=4, seed=3, steps=3):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve(shape, grains, seed, twin_share=0.5)
    return rvegen.Workload("t", rve, rvegen.config_systems(True), C, law,
                           rvegen.uniaxial_path(0.006, steps, rate=1e-2))


def _relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("rk_tol,shape", [(1e-7, (6, 6, 6)), (1e-8, (6, 6, 6)), (1e-7, (8, 12, 16))])
def test_fp64_parity(rk_tol, shape):
    print("case", rk_tol, shape, flush=True)
    w = _w(shape)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-11, rk_tol=rk_tol)
    R = gs.run(w.path)
    o = oracle.solver_for(w, oracle.Options(tol=1e-11, rk_tol=rk_tol))
    ref = o.run(w.path, keep_fields=True)
    assert np.all(R["status"] == 0)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    assert np.array_equal(R["iters"], ref.iters)
    M = oracle.substeps(w.path.t[1] - w.path.t[0], 0.05)
    counts = gs.field("substeps").cpu().numpy().ravel()
    ref_counts = M * 2.0 ** o.substep_j
    assert np.array_equal(counts, ref_counts)
    assert len(np.unique(counts)) >= 2
    for name in ("stress", "plastic_strain", "acc_slip"):
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-10, name


def test_loose_tolerance_is_the_fixed_count():
    w = _w()
    R = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-11, rk_tol=1.0)
    Ra = R.run(w.path)
    assert np.all(R.field("substeps").cpu().numpy() == oracle.substeps(w.path.t[1] - w.path.t[0], 0.05))
    Rf = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-11).run(w.path)
    assert np.array_equal(Ra["iters"], Rf["iters"])
    assert _relerr(Ra["Sigma"], Rf["Sigma"]) < 1e-13


def test_fp32_close_to_fp64_oracle():
    w = rvegen.workload(0)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp32", tol=1e-6, stag_tol=1e-4, rk_tol=1e-7)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-10, rk_tol=1e-7)).run(w.path)
    assert np.all(R["status"] == 0)
    assert np.abs(R["Sigma"][:, 0] - ref.Sigma[:, 0]).max() / np.abs(ref.Sigma[:, 0]).max() < 1e-4


def test_batch_members_match_solo_solves():
    ws = [_w((6, 6, 6), 4, 3), _w((8, 8, 8), 5, 4)]
    probs = [cp.Problem.from_workload(w) for w in ws]
    b = cp.Solver(probs, precision="fp64", tol=1e-11, rk_tol=1e-7)
    outs = [[] for _ in ws]
    for n in range(ws[0].path.n_steps):
        for i, o in enumerate(b.step_batch(ws[0].path, n)):
            outs[i].append(o["Sigma"])
    for i, p in enumerate(probs):
        R = cp.Solver(p, precision="fp64", tol=1e-11, rk_tol=1e-7).run(ws[0].path)
        assert _relerr(np.array(outs[i]), R["Sigma"]) < 1e-12


def test_argument_checks():
    w = _w()
    p = cp.Problem.from_workload(w)
    with pytest.raises(cp.CpfError):
        cp.Solver(p, precision="fp64", rk_tol=-1.0)
    s = cp.Solver(p, precision="fp64", rk_tol=1e-6)
    with pytest.raises(cp.CpfError):
        s.gradient(w.path, np.ones(w.path.n_steps))


def test_substeps_with_the_rotated_operator():
    w = _w((6, 6, 6))
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-11, rk_tol=1e-8, green="rotated")
    R = gs.run(w.path)
    o = oracle.solver_for(w, oracle.Options(tol=1e-11, rk_tol=1e-8, green="rotated"))
    ref = o.run(w.path)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    assert np.array_equal(R["iters"], ref.iters)
