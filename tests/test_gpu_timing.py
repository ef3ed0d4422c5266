"""Per-kernel timing with HIP events (the figures the benchmark's roofline
divides by): the solve is bit for bit the same with timing on or off, every
timed launch of a load step has been read when the step returns (the
events of a finished chunk are read while the next chunk runs, the last
chunk's at the end of the step), enabling timing resets the counts, and
the x-pass-only mode times that kernel alone."""
import numpy as np
import pytest

import rvegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
cp = pytest.importorskip("paper_2402_09996_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cp._lib.lib()
    yield


def _workload():
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    path = rvegen.uniaxial_path(0.008, 6)
    # 32 points per edge: the fixed-length y and z kernels, whose inverse y
    # launch also runs the first stage of the scalar reduction
    return rvegen.Workload("timing", rvegen.make_rve((32, 32, 32), 6, 11, twin_share=0.5), S, C, law, path), path


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("check_every", [0, 1, 3])
def test_timing_reads_every_launch_and_leaves_the_solve_unchanged(precision, check_every):
    w, path = _workload()
    kw = dict(tol=1e-6 if precision == "fp32" else 1e-9, stag_tol=1e-4 if precision == "fp32" else 0.0,
              check_every=check_every)
    plain = cp.Solver(cp.Problem.from_workload(w), precision=precision, **kw)
    timed = cp.Solver(cp.Problem.from_workload(w), precision=precision, **kw)
    timed.set_timing(True)
    assert all(v == (0.0, 0) for v in timed.timing().values())
    its = 0
    for n in range(path.n_steps):
        a = plain.step(path, n)
        b = timed.step(path, n)
        assert np.array_equal(a["Sigma"], b["Sigma"]) and a["iters"] == b["iters"]
        its += int(b["iters"])
        t = timed.timing()
        counts = {k: c for k, (_, c) in t.items()}
        # the five kernels of an iteration are launched together
        assert len(set(counts.values())) == 1, counts
        launched = counts["xpass_law"]
        # every launch of the step read back: none pending at its end
        assert launched >= its
        if check_every == 1:
            # one iteration per poll: exactly the iterations the step made
            assert launched == its
        assert all(ms > 0.0 for ms, _ in t.values())
    assert plain.timing()["xpass_law"] == (0.0, 0)
    timed.set_timing(True)
    assert all(v == (0.0, 0) for v in timed.timing().values())
    timed.step(path, 0)
    assert timed.timing()["xpass_law"][1] >= 1


def test_xpass_only_timing_counts_the_x_pass_alone():
    w, path = _workload()
    kw = dict(tol=1e-6, stag_tol=1e-4)
    full = cp.Solver(cp.Problem.from_workload(w), precision="fp32", **kw)
    xonly = cp.Solver(cp.Problem.from_workload(w), precision="fp32", **kw)
    full.set_timing(True)
    xonly.set_timing("xpass")
    its = 0
    for n in range(3):
        a = full.step(path, n)
        b = xonly.step(path, n)
        assert np.array_equal(a["Sigma"], b["Sigma"]) and a["iters"] == b["iters"]
        its += int(b["iters"])
    tx, tf = xonly.timing(), full.timing()
    assert tx["xpass_law"][1] == tf["xpass_law"][1] >= its and tx["xpass_law"][0] > 0.0
    assert all(tx[k] == (0.0, 0) for k in cp.Solver.KERNELS if k != "xpass_law")
    # x-pass figures of the two modes agree (same launches; fewer markers)
    assert tx["xpass_law"][0] == pytest.approx(tf["xpass_law"][0], rel=0.25)
    for bad in (3, -1):
        assert cp._lib.lib().cpf_solver_set_timing(xonly._h, bad) == cp._lib.CPF_E_INVALID_ARG
