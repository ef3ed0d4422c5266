"""The Anderson-accelerated fixed point on the device against the oracle's:
FP64 solves with the same iterates (results to 1e-10, iteration counts
within one), the basic scheme's fixed point in fewer iterations, FP32
accuracy, batches and graph launches, argument checks."""
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


def _w(shape=(6, 12, 18), grains=5, seed=21, steps=4):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve(shape, grains, seed, twin_share=0.5)
    return rvegen.Workload("t", rve, rvegen.config_systems(True), C, law,
                           rvegen.uniaxial_path(0.008, steps, rate=1e-2))


def _relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("m,shape", [(4, (6, 12, 18)), (2, (8, 8, 8)), (8, (8, 8, 8))])
def test_fp64_parity_with_the_oracle(m, shape):
    print("case", m, shape, flush=True)
    w = _w(shape)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, aa_depth=m)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12, aa_depth=m)).run(w.path, keep_fields=True)
    print("iters", R["iters"], ref.iters, flush=True)
    assert np.all(R["status"] == 0)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    assert _relerr(R["E"], ref.E) < 1e-10
    assert np.abs(np.asarray(R["iters"]) - ref.iters).max() <= 1
    for name in ("stress", "strain", "plastic_strain"):
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-9, name


def test_basic_fixed_point_in_fewer_iterations():
    w = _w()
    p = cp.Problem.from_workload(w)
    Rb = cp.Solver(p, precision="fp64", tol=1e-12).run(w.path)
    Ra = cp.Solver(p, precision="fp64", tol=1e-12, aa_depth=4).run(w.path)
    assert _relerr(Ra["Sigma"], Rb["Sigma"]) < 1e-8
    assert np.sum(Ra["iters"]) * 1.5 < np.sum(Rb["iters"]), (Ra["iters"], Rb["iters"])


def test_fp32_close_to_fp64_oracle():
    w = rvegen.workload(0)
    R = cp.Solver(cp.Problem.from_workload(w), precision="fp32", tol=1e-6, stag_tol=1e-4, aa_depth=4).run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-10)).run(w.path)
    assert np.all(R["status"] == 0)
    assert np.abs(R["Sigma"][:, 0] - ref.Sigma[:, 0]).max() / np.abs(ref.Sigma[:, 0]).max() < 1e-4


@pytest.mark.parametrize("graph", [0, 4])
def test_batch_members_match_solo_solves(graph):
    ws = [_w((6, 6, 6), 4, 3), _w((8, 8, 8), 5, 4)]
    probs = [cp.Problem.from_workload(w) for w in ws]
    b = cp.Solver(probs, precision="fp64", tol=1e-11, aa_depth=4, graph_iters=graph)
    outs = [[] for _ in ws]
    for n in range(ws[0].path.n_steps):
        for i, o in enumerate(b.step_batch(ws[0].path, n)):
            outs[i].append(o["Sigma"])
    for i, p in enumerate(probs):
        R = cp.Solver(p, precision="fp64", tol=1e-11, aa_depth=4).run(ws[0].path)
        assert _relerr(np.array(outs[i]), R["Sigma"]) < 1e-12


def test_argument_checks():
    w = _w((6, 6, 6), 4, 3)
    p = cp.Problem.from_workload(w)
    with pytest.raises(cp.CpfError):
        cp.Solver(p, precision="fp64", aa_depth=9)
    with pytest.raises(cp.CpfError):
        cp.Solver(p, precision="fp64", aa_depth=4, rk_tol=1e-6)
    s = cp.Solver(p, precision="fp64", aa_depth=4)
    with pytest.raises(cp.CpfError):
        s.gradient(w.path, np.ones(w.path.n_steps))


def test_anderson_with_the_rotated_operator():
    w = _w((8, 8, 8))
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, aa_depth=4, green="rotated")
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12, aa_depth=4, green="rotated")).run(w.path)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    assert np.abs(np.asarray(R["iters"]) - ref.iters).max() <= 1
