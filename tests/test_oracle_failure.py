"""Failure handling of the oracle: the local-stress count of Section 4's
condition (|sigma_{n+1} - sigma_n|_F > E0 |E_{n+1} - E_n|_F) in closed
form, and the step cut-back (a load step that diverges is retried as two
half steps).  CPU only."""
import numpy as np
import pytest

import oracle
import rvegen


def _iso(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return rvegen.cubic_stiffness(lam + 2 * mu, lam, mu), lam, mu


def _elastic_solver(C, shape=(4, 4, 4)):
    _, law = rvegen.config_law()
    S = rvegen.config_systems(False)
    labels = np.zeros(shape, np.int32)
    eul = np.array([[0.4, 1.1, 2.0]])
    return oracle.Solver(labels, eul, C, S.n_miller, S.l_miller, S.family, np.full(12, 1e9), law,
                         oracle.Options(tol=1e-12))


@pytest.mark.parametrize("nu", [0.2, 0.3, 0.45])
def test_symptom_count_closed_forms(nu):
    """Homogeneous isotropic elastic RVE (the reference medium is the
    material itself): under uniaxial stress |dsigma| = E |dE11| < E
    |dE|_F (lateral contraction), no voxel is counted; under uniaxial
    strain (every component prescribed) |dsigma| = |dE11| sqrt((lam +
    2 mu)^2 + 2 lam^2) > E |dE11|, every voxel is."""
    E = 150000.0
    C, lam, mu = _iso(E, nu)
    s = _elastic_solver(C)
    assert s.mu0 == pytest.approx(mu, rel=1e-12) and s.lam0 == pytest.approx(lam, rel=1e-12)
    R = s.run(rvegen.uniaxial_path(3e-3, 3))
    assert np.array_equal(R.n_symptom, np.zeros(3, np.int64))
    assert np.sqrt((lam + 2 * mu) ** 2 + 2 * lam ** 2) > E
    s = _elastic_solver(C)
    t = np.linspace(0.0, 3.0, 4)
    target = np.zeros((3, 6))
    target[:, 0] = [1e-3, 2e-3, 3e-3]
    path = rvegen.LoadPath(t=t, strain_ctrl=np.ones((3, 6), np.uint8), target=target)
    R = s.run(path)
    assert np.array_equal(R.n_symptom, np.full(3, 64))
    assert R.Sigma[-1, 1] == pytest.approx(lam * 3e-3, rel=1e-10)


def _stiff_step_workload(strain=2e-3):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve((4, 4, 4), 3, 4)
    S = rvegen.config_systems(with_twins=False)
    return rvegen.Workload("cb", rve, S, C, law, rvegen.uniaxial_path(strain, 1))


def test_diverging_step_is_reported_and_cut_back():
    """One RK4 substep over a 2 s load step of 0.2 % diverges (non-finite
    residual); with cut-back the step completes in half steps, each of
    which converges, and a retry without halvings left reports the error."""
    w = _stiff_step_workload()
    with pytest.raises(FloatingPointError):
        oracle.solver_for(w, oracle.Options(tol=1e-10, M=1)).run(w.path)
    s = oracle.solver_for(w, oracle.Options(tol=1e-10, M=1, cutback=6))
    R = s.run(w.path)
    assert R.cutbacks[0] >= 1 and np.all(np.isfinite(R.Sigma))
    assert R.E[0, 0] == pytest.approx(2e-3, rel=1e-12)
    assert abs(R.Sigma[0, 1]) < 1e-8 * abs(R.Sigma[0, 0])       # lateral stress at its target
    with pytest.raises(FloatingPointError):
        oracle.solver_for(w, oracle.Options(tol=1e-10, M=1, cutback=1)).run(w.path)
