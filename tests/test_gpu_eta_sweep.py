"""Fig. 3 analogue (Section 4): the yield stress of a single-crystal
material point as a function of the regularization eta, device (FP64)
against the oracle.  A one-orientation 2x2x2 RVE has uniform fields and is
a material point under the mixed macroscopic conditions; uniaxial tension
along x at 1e-3 /s to 0.5 % in 20 large steps of one RK4 step each, the
paper's parameter set.  The
yield stress is read at 0.02 % axial plastic strain (E11 - S11 / E_x with
E_x the initial slope), interpolated between steps.  Too small an eta makes
the explicit integration diverge on both sides."""
import math

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


def yield_offset(E11, S11, offset=2e-4):
    Ex = S11[0] / E11[0]
    ep = E11 - S11 / Ex
    k = int(np.argmax(ep >= offset))
    assert ep[k] >= offset and k > 0
    a = (offset - ep[k - 1]) / (ep[k] - ep[k - 1])
    return S11[k - 1] + a * (S11[k] - S11[k - 1])


def _workload(eta, euler=(0.3, 0.7, 1.1), steps=20):
    C, law = rvegen.paper_law()
    law.eta = eta
    S = rvegen.table1_systems(True)
    rve = rvegen.Microstructure(labels=np.zeros((2, 2, 2), np.int32), euler=np.array([euler]),
                                n_grains=1, twinned=np.zeros(0, np.int64), twin_fraction=np.zeros(0))
    return rvegen.Workload("point", rve, S, C, law, rvegen.uniaxial_path(0.005, steps))


@pytest.mark.parametrize("eta", [1e4, 1e5])
def test_schmid_half_crystal_first_yields_at_twice_tau0(eta):
    """The semi-quantitative check of Section 4's yield stresses: a crystal
    whose ordinary system 3 has the Schmid factor 1/2 along the load (all
    other systems lower ratios tau0/m) stays elastic up to 2 tau0 = 260 MPa
    and is plastic right after, whatever eta; device against the oracle."""
    S = rvegen.table1_systems(True)
    w = _workload(eta, tuple(rvegen.schmid_half_orientation(S, 2)), steps=100)
    R = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, rk4_M=1).run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12, M=1)).run(w.path)
    assert np.abs(R["Sigma"] - ref.Sigma).max() <= 1e-9 * np.abs(ref.Sigma).max()
    k = int(np.argmax(R["mean_v"] > 0))
    print("eta", eta, "onset between", R["Sigma"][k - 1, 0], R["Sigma"][k, 0], flush=True)
    assert k > 0 and R["Sigma"][k - 1, 0] <= 260.0 < R["Sigma"][k, 0]
    assert k == int(np.argmax(ref.mean_v > 0))


@pytest.mark.parametrize("eta", [5e3, 1e4, 1e5])
def test_yield_stress_matches_oracle(eta):
    w = _workload(eta)
    R = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, rk4_M=1).run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12, M=1)).run(w.path)
    y = yield_offset(R["E"][:, 0], R["Sigma"][:, 0])
    yo = yield_offset(ref.E[:, 0], ref.Sigma[:, 0])
    print("eta", eta, "yield", y, yo, flush=True)
    assert y == pytest.approx(yo, rel=1e-9)
    assert np.abs(R["Sigma"] - ref.Sigma).max() <= 1e-9 * np.abs(ref.Sigma).max()


def test_small_eta_diverges_on_both_sides():
    w = _workload(1e3)
    with pytest.raises(cp.CpfError):
        cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, rk4_M=1).run(w.path)
    with pytest.raises((FloatingPointError, oracle.NotConverged)):
        oracle.solver_for(w, oracle.Options(tol=1e-12, M=1)).run(w.path)


def test_yield_rises_with_eta():
    ys = []
    for eta in (5e3, 1e4, 1e5, 1e6):
        w = _workload(eta)
        R = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, rk4_M=1).run(w.path)
        ys.append(yield_offset(R["E"][:, 0], R["Sigma"][:, 0]))
    assert all(b > a for a, b in zip(ys, ys[1:])), ys
