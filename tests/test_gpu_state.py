"""Saving and restoring the committed state: a restart from a saved state
repeats the continuation bit for bit, for single solves and batches."""
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


def _workloads():
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    path = rvegen.uniaxial_path(0.008, 8)
    return [rvegen.Workload("s%d" % i, rvegen.make_rve(sh, 5, 40 + i, twin_share=0.5), S, C, law, path)
            for i, sh in enumerate([(8, 12, 16), (16, 16, 16)])], path


def _fields(s, i):
    return np.concatenate([s.field_of(i, k).double().cpu().numpy().ravel()
                           for k in ("strain", "plastic_strain", "acc_slip", "back_strain", "stress")])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_restart_from_saved_state_is_bitwise(precision):
    wl, path = _workloads()
    kw = dict(tol=1e-10 if precision == "fp64" else 1e-6, stag_tol=0.0 if precision == "fp64" else 1e-4)
    s = cp.Solver([cp.Problem.from_workload(w) for w in wl], precision=precision, **kw)
    for n in range(4):
        s.step_batch(path, n)
    saved = s.save_state()
    first = [s.step_batch(path, n) for n in range(4, 8)]
    f_first = [_fields(s, i) for i in range(len(wl))]
    s.reset()                                   # anything else in between
    s.step_batch(path, 0)
    s.restore_state(saved)
    again = [s.step_batch(path, n) for n in range(4, 8)]
    for a, b in zip(first, again):
        for x, y in zip(a, b):
            assert np.array_equal(x["Sigma"], y["Sigma"]) and x["iters"] == y["iters"]
    for i in range(len(wl)):
        assert np.array_equal(f_first[i], _fields(s, i))
    # a second solver of the same problems takes the same state
    t = cp.Solver([cp.Problem.from_workload(w) for w in wl], precision=precision, **kw)
    t.restore_state(saved)
    other = [t.step_batch(path, n) for n in range(4, 8)]
    for a, b in zip(first, other):
        for x, y in zip(a, b):
            assert np.array_equal(x["Sigma"], y["Sigma"])


def test_restore_rejects_foreign_buffer():
    wl, path = _workloads()
    s = cp.Solver(cp.Problem.from_workload(wl[0]), precision="fp64")
    saved = s.save_state()
    junk = torch.full_like(saved, 255)
    with pytest.raises(cp.CpfError):
        s.restore_state(junk)
