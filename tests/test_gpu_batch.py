"""Batched solves of uneven RVEs: per-member results equal the single-RVE
solves bit for bit, the captured-graph path equals direct launches on every
step, autotuned tiles do not change results, and a member matches the
FP64 oracle."""
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


def _members():
    C, law = rvegen.config_law()
    S = rvegen.config_systems(with_twins=True)
    # generic and fixed-length y/z transforms in one batch (32: fixed)
    shapes = [(8, 8, 8), (12, 12, 12), (6, 12, 18), (16, 16, 16), (32, 32, 32)]
    rves = [rvegen.make_rve(sh, 4 + i, 300 + i, twin_share=0.5 if i % 2 == 0 else 0.0)
            for i, sh in enumerate(shapes)]
    path = rvegen.uniaxial_path(0.004, 4)
    wl = [rvegen.Workload("m%d" % i, r, S, C, law, path) for i, r in enumerate(rves)]
    return wl, path


def _run_batch(wl, path, precision, **kw):
    s = cp.Solver([cp.Problem.from_workload(w) for w in wl], precision=precision, **kw)
    outs = [s.step_batch(path, n) for n in range(path.n_steps)]
    fields = [s.field_of(i, "stress").cpu().numpy() for i in range(len(wl))]
    return s, outs, fields


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_members_equal_single_solves(precision):
    wl, path = _members()
    tol = 1e-10 if precision == "fp64" else 1e-6
    kw = dict(tol=tol, stag_tol=0.0 if precision == "fp64" else 1e-4)
    s, outs, fields = _run_batch(wl, path, precision, **kw)
    for i, w in enumerate(wl):
        print("member", i, w.rve.labels.shape, flush=True)
        g = cp.Solver(cp.Problem.from_workload(w), precision=precision, **kw)
        R = g.run(path)
        for n in range(path.n_steps):
            assert np.array_equal(outs[n][i]["Sigma"], R["Sigma"][n])
            assert outs[n][i]["iters"] == R["iters"][n]
        assert np.array_equal(fields[i], g.field("stress").cpu().numpy())


def test_batch_member_matches_oracle():
    wl, path = _members()
    s, outs, fields = _run_batch(wl, path, "fp64", tol=1e-12)
    i = 2       # 6 x 12 x 18, twinned
    ref = oracle.solver_for(wl[i], oracle.Options(tol=1e-12)).run(path, keep_fields=True)
    sig = np.array([outs[n][i]["Sigma"] for n in range(path.n_steps)])
    assert np.linalg.norm(sig - ref.Sigma) / np.linalg.norm(ref.Sigma) < 1e-10
    assert np.linalg.norm(fields[i] - ref.fields["stress"]) / np.linalg.norm(ref.fields["stress"]) < 1e-10
    assert [outs[n][i]["iters"] for n in range(path.n_steps)] == list(ref.iters)


@pytest.mark.parametrize("graph_iters", [3, 64, "adaptive"])
def test_graph_replays_equal_direct_launches(graph_iters):
    """Each load step replays the captured graph one or more times, with the
    host's own step setup and synchronizations between replays; every
    step's result must equal the direct-launch result."""
    wl, path = _members()
    kw = dict(tol=1e-6, stag_tol=1e-4)
    _, direct, fd = _run_batch(wl, path, "fp32", **kw)
    _, graphed, fg = _run_batch(wl, path, "fp32", graph_iters=graph_iters, **kw)
    for n in range(path.n_steps):
        for i in range(len(wl)):
            assert np.array_equal(direct[n][i]["Sigma"], graphed[n][i]["Sigma"]), (n, i)
            assert direct[n][i]["iters"] == graphed[n][i]["iters"]
    for a, b in zip(fd, fg):
        assert np.array_equal(a, b)
    if graph_iters == "adaptive":
        # after the first step the graph length mostly covers the step
        syncs = [graphed[n][0]["host_syncs"] for n in range(path.n_steps)]
        print("host syncs per step", syncs, [graphed[n][0]["iters"] for n in range(path.n_steps)], flush=True)
        assert all(x <= 2 for x in syncs[1:]), syncs


def test_stalled_residual_acceptance_is_reported():
    """FP32 with an unreachable tolerance ends each step by the stalled
    residual acceptance: status 0, the flag set, residual above tol."""
    wl, path = _members()
    _, outs, _ = _run_batch(wl[:2], path, "fp32", tol=1e-13, stag_tol=1e-4)
    for n in range(path.n_steps):
        for o in outs[n]:
            assert o["status"] == 0 and o["stagnated"] == 1
            assert 1e-13 < max(o["err_eq"], o["err_bc"]) < 1e-4
    _, outs, _ = _run_batch(wl[:2], path, "fp64", tol=1e-10)
    assert all(o["stagnated"] == 0 for step in outs for o in step)


def test_autotuned_tiles_are_valid_and_do_not_change_results():
    wl, path = _members()
    kw = dict(tol=1e-6, stag_tol=1e-4)
    _, base, fb = _run_batch(wl, path, "fp32", **kw)
    s, tuned, ft = _run_batch(wl, path, "fp32", autotune=True, **kw)
    assert s.autotuned > 0 or all(s.tiles(i)[0] > 0 for i in range(len(wl)))
    for i, w in enumerate(wl):
        ty, tz = s.tiles(i)
        nhx = w.rve.labels.shape[2] // 2 + 1
        assert 1 <= ty <= nhx and 1 <= tz <= nhx
    for n in range(path.n_steps):
        for i in range(len(wl)):
            assert np.array_equal(base[n][i]["Sigma"], tuned[n][i]["Sigma"])
    for a, b in zip(fb, ft):
        assert np.array_equal(a, b)


def test_batch_rejects_mixed_laws():
    wl, path = _members()
    C, law = rvegen.config_law()
    law.eta = 5e3
    other = rvegen.Workload("x", wl[0].rve, wl[0].systems, C, law, path)
    with pytest.raises(cp.CpfError):
        cp.Solver([cp.Problem.from_workload(wl[1]), cp.Problem.from_workload(other)])
