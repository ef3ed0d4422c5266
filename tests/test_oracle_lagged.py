"""Pins of the oracle's lagged regularization (option reg='lagged': the
yield stress of a load step raised by eta times the slip rate of the
previous step, the rate itself from the plain Norton law).  A
one-system single crystal under an imposed shear strain rate (every
component prescribed, linear Norton law n = 1, no hardening) has closed
forms: at steady state both readings give tau = tau0 + (K + eta) gdot with
gdot = 2 dE12/dt; with eta < K the lagged steps converge to it, with eta
much larger than K they alternate between purely elastic steps and steps
that slip at twice the imposed rate (the behaviour Section 4 describes);
with eta = 0 the two readings coincide.  CPU only."""
import numpy as np
import pytest

import oracle
import rvegen

E_, NU = 150000.0, 0.3
LAM = E_ * NU / ((1 + NU) * (1 - 2 * NU))
MU = E_ / (2 * (1 + NU))
RATE = 1e-3            # dE12/dt (tensor component); the slip rate is twice that


def _run(K, eta, reg, steps=60, n=1.0):
    C = rvegen.cubic_stiffness(LAM + 2 * MU, LAM, MU)
    fam = rvegen.FamilyLaw(Q=0.0, b=10.0, c=0.0, d=0.0, K=K, n=n, q_self=1.0, q_latent=1.0)
    law = rvegen.Law(slip=fam, twin=rvegen.FamilyLaw(**vars(fam)), eta=eta)
    S = rvegen.SystemSet(np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]),
                         np.array([0], np.int32), ["o"], np.array([50.0]))
    t = np.linspace(0.0, steps * 0.5, steps + 1)
    target = np.zeros((steps, 6))
    target[:, 5] = RATE * t[1:]
    path = rvegen.LoadPath(t=t, strain_ctrl=np.ones((steps, 6), np.uint8), target=target)
    s = oracle.Solver(np.zeros((2, 2, 2), np.int32), np.array([[0.0, 0.0, 0.0]]), C, S.n_miller, S.l_miller,
                      S.family, S.tau0, law, oracle.Options(tol=1e-12, M=4, reg=reg))
    return s.run(path)


def test_lagged_reaches_the_implicit_steady_state_when_eta_is_below_K():
    K, eta = 20000.0, 4000.0
    closed = 50.0 + (K + eta) * 2 * RATE
    for reg in ("implicit", "lagged"):
        R = _run(K, eta, reg)
        assert R.Sigma[-1, 5] == pytest.approx(closed, rel=1e-9), reg
        rate = np.diff(R.mean_v)[-5:] / 0.5
        assert np.allclose(rate, 2 * RATE, rtol=1e-9), reg


@pytest.mark.parametrize("eta", [2e5, 2e6])
def test_lagged_alternates_elastic_and_plastic_steps_when_eta_dominates(eta):
    R = _run(20000.0, eta, "lagged")
    dv = np.diff(np.concatenate([[0.0], R.mean_v]))[-20:]
    rate = dv / 0.5
    zero, slip = rate[0::2], rate[1::2]
    if zero[0] > slip[0]:
        zero, slip = slip, zero
    assert np.all(zero == 0.0)
    assert np.allclose(slip, 4 * RATE, rtol=1e-9)
    # the two-step mean is the imposed rate; the implicit reading does not alternate
    Ri = _run(20000.0, eta, "implicit")
    assert np.all(np.diff(Ri.mean_v)[-20:] > 0.0)


def test_lagged_equals_implicit_without_regularization():
    # eta = 0: no raised resistance in either reading (a stable K for explicit RK4)
    Ra = _run(20000.0, 0.0, "implicit", steps=12)
    Rb = _run(20000.0, 0.0, "lagged", steps=12)
    assert np.array_equal(Ra.Sigma, Rb.Sigma) and np.array_equal(Ra.mean_v, Rb.mean_v)


def test_lagged_option_is_checked():
    w = rvegen.workload(0, n_override=8)
    with pytest.raises(ValueError):
        oracle.solver_for(w, oracle.Options(reg="delayed"))
    with pytest.raises(ValueError):
        oracle.solver_for(w, oracle.Options(reg="lagged", aa_depth=2))
