"""Pins of the oracle's hardening interaction (Section 3, equation 4), the
untwinned-fraction weighting of the slip contribution (equation 1) and the
Section 5 averages <v^s>, <f_beta>.  Each expected value is a closed form
of the steady state of the law under constant imposed plastic shear, or a
number worked out by hand, so that a wrong interaction coefficient,
hardening across families, a dropped (1 - sum f) factor or a twin fraction
taken without the twinning shear fails here.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import rvegen

SQ2 = math.sqrt(2.0)
MU = 200000.0 / 2.6                                  # shear modulus of _iso()


def _iso(E=200000.0, nu=0.3):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return rvegen.cubic_stiffness(lam + 2 * mu, lam, mu)


def _law(Qs=40.0, Qt=30.0, b=10.0, K=10.0, n=10.0, eta=1e4, qs=1.0, ql=1.4):
    slip = rvegen.FamilyLaw(Q=Qs, b=b, c=0.0, d=0.0, K=K, n=n, q_self=qs, q_latent=ql)
    twin = rvegen.FamilyLaw(Q=Qt, b=b, c=0.0, d=0.0, K=K, n=n, q_self=qs, q_latent=ql)
    return rvegen.Law(slip=slip, twin=twin, eta=eta)


def _drive(mat, y, eps, comp, rate, t_end, dt=1.0, M=20):
    """Engineering shear rate `rate` on tensor shear component `comp`
    (3: 23, 4: 13, 5: 12) of a single point; returns (y, eps, tau_comp)."""
    t = 0.0
    sig = None
    while t < t_end - 1e-12:
        e1 = eps.copy()
        e1[comp] += SQ2 * 0.5 * rate * dt            # Mandel sqrt2 * eps_ij, eps_ij = gamma / 2
        y, sig = mat.update([0], eps, e1, y, dt, M)
        eps, t = e1, t + dt
    return y, eps, sig[0, comp] / SQ2


def test_latent_hardening_within_a_family_closed_form():
    """Two slip systems with the same Schmid tensor (planes and directions
    swapped) share a constant imposed shear rate g equally.  At saturation
    (b v >> 1) equation 4 gives r = tau0 + Q (q_self + q_latent), so the
    steady resolved shear stress is tau0 + Q (q_self + q_latent)
    + K (g/2)^(1/n) + eta g / 2."""
    tau0, Q, qs, ql, K, n, eta, g = 50.0, 40.0, 1.0, 1.4, 10.0, 10.0, 1e4, 0.02
    law = _law(Qs=Q, qs=qs, ql=ql, K=K, n=n, eta=eta)
    mat = oracle.Material([[0, 0, 0]], _iso(), [[0, 1, 0], [1, 0, 0]], [[1, 0, 0], [0, 1, 0]],
                          [0, 0], [tau0, tau0], law)
    y, eps, tau = _drive(mat, np.zeros((1, mat.state_dim)), np.zeros(6), 5, g, 600.0)
    expect = tau0 + Q * (qs + ql) + K * (g / 2) ** (1 / n) + eta * g / 2
    assert tau == pytest.approx(expect, rel=1e-9)
    # the two systems slipped alike, and together by the imposed shear less
    # its elastic part tau / mu
    assert y[0, 6] == pytest.approx(y[0, 7], rel=1e-12)
    assert y[0, 6] + y[0, 7] == pytest.approx(g * 600.0 - tau / MU, rel=1e-12)
    # a different latent coefficient moves the steady state by Q * dq
    law2 = _law(Qs=Q, qs=qs, ql=2.0, K=K, n=n, eta=eta)
    mat2 = oracle.Material([[0, 0, 0]], _iso(), [[0, 1, 0], [1, 0, 0]], [[1, 0, 0], [0, 1, 0]],
                           [0, 0], [tau0, tau0], law2)
    _, _, tau2 = _drive(mat2, np.zeros((1, mat.state_dim)), np.zeros(6), 5, g, 600.0)
    assert tau2 - tau == pytest.approx(Q * (2.0 - ql), rel=1e-8)


def test_latent_hardening_by_an_inactive_system_of_the_family():
    """Slip on system a only (system b's Schmid tensor is orthogonal to the
    load) hardens b by Q q_latent (1 - exp(-b v_a)); loading b afterwards at
    a slow rate then yields it above tau0 + Q q_latent: the steady state of
    b is tau0 + Q (q_self + q_latent) + K g^(1/n) + eta g once both
    saturate, and before b accumulates slip its first yield lies at
    tau0 + Q q_latent + (rate terms)."""
    tau0, Q, qs, ql, K, n, eta, g = 50.0, 40.0, 1.0, 1.4, 10.0, 10.0, 1e4, 0.02
    law = _law(Qs=Q, qs=qs, ql=ql, K=K, n=n, eta=eta)
    # a: shear 12, b: shear 13
    mat = oracle.Material([[0, 0, 0]], _iso(), [[0, 1, 0], [0, 0, 1]], [[1, 0, 0], [1, 0, 0]],
                          [0, 0], [tau0, tau0], law)
    y, eps, tau_a = _drive(mat, np.zeros((1, mat.state_dim)), np.zeros(6), 5, g, 600.0)
    assert y[0, 7] == 0.0                          # b never slipped
    assert tau_a == pytest.approx(tau0 + Q * qs + K * g ** (1 / n) + eta * g, rel=1e-9)
    # unload a (its stress to zero) and load b to saturation
    e1 = eps.copy()
    e1[5] = y[0, 5]
    y, _ = mat.update([0], eps, e1, y, 1.0, 20)
    eps = e1
    y, eps, tau_b = _drive(mat, y, eps, 4, g, 600.0)
    assert tau_b == pytest.approx(tau0 + Q * (qs + ql) + K * g ** (1 / n) + eta * g, rel=1e-9)


def _slip_twin_material(twin_mode=rvegen.TWIN_NORTON, gamma_T=1.0 / SQ2):
    """Slip system on shear 12, twin system on shear 13 (orthogonal Schmid
    tensors), identity orientation, isotropic stiffness."""
    law = _law(Qs=40.0, Qt=30.0)
    law.twin_mode = twin_mode
    law.gamma_T = gamma_T
    law.K_c, law.f_m = 1.45, 0.8
    return oracle.Material([[0, 0, 0]], _iso(), [[0, 1, 0], [0, 0, 1]], [[1, 0, 0], [1, 0, 0]],
                           [0, 1], [50.0, 60.0], law)


@pytest.mark.parametrize("twin_mode", [rvegen.TWIN_NORTON, rvegen.TWIN_PAPER])
def test_frozen_twin_fraction_scales_the_slip_contribution(twin_mode):
    """Twin first (shear 13) to a fraction f = v_beta / gamma_T, then unload
    the twin exactly (its resolved stress becomes zero, below r_beta, so
    f stays frozen) and shear along 12 at the engineering rate g.  Equation
    1 weights the slip contribution by (1 - f): at steady state the slip
    rate is g / (1 - f).  Equation 4 sums within the slip family only, so
    the twin's accumulated slip does not harden the slip system: the steady
    resolved stress is tau0_s + Q_s q_self + K (g/(1-f))^(1/n) + eta g/(1-f)."""
    mat = _slip_twin_material(twin_mode)
    law = mat.law
    y, eps, _ = _drive(mat, np.zeros((1, mat.state_dim)), np.zeros(6), 4, 0.02, 12.0, dt=0.5, M=10)
    v_beta = y[0, 7]
    assert 0.05 < v_beta < 0.5
    e1 = eps.copy()
    e1[4] = y[0, 4]                                  # eps13 = eps_p13: sigma13 = 0
    y, _ = mat.update([0], eps, e1, y, 1.0, 20)
    eps = e1
    f = y[0, 7] / law.gamma_T
    assert 0.05 < f < 0.6
    g = 0.02
    y2, eps2, tau = _drive(mat, y, eps, 5, g, 600.0)
    assert y2[0, 7] == y[0, 7]                       # the fraction stayed frozen
    gs = g / (1.0 - f)
    expect = 50.0 + 40.0 * 1.0 + 10.0 * gs ** 0.1 + 1e4 * gs
    assert tau == pytest.approx(expect, rel=1e-9)
    # the slip system's accumulated slip is the plastic shear / (1 - f)
    assert y2[0, 6] == pytest.approx((g * 600.0 - tau / MU) / (1.0 - f), rel=1e-12)


def test_twin_steady_state_in_norton_mode():
    """A lone twin system driven at the constant engineering rate g along
    its own shear: its contribution is not weighted, so its rate is g and,
    once its own hardening saturates, tau = tau0_b + Q_b q_self
    + K g^(1/n) + eta g."""
    law = _law(Qt=30.0)
    mat = oracle.Material([[0, 0, 0]], _iso(), [[0, 0, 1]], [[1, 0, 0]], [1], [60.0], law)
    g = 0.02
    y, _, tau = _drive(mat, np.zeros((1, mat.state_dim)), np.zeros(6), 4, g, 600.0)
    assert tau == pytest.approx(60.0 + 30.0 + 10.0 * g ** 0.1 + 1e4 * g, rel=1e-9)


def _tiny_solver(gamma_T):
    S = rvegen.SystemSet(n_miller=np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0], [0, 1, 0]], float),
                         l_miller=np.array([[1, 0, 0], [1, 0, 0], [0, 0, 1], [0, 0, 1]], float),
                         family=np.array([0, 0, 1, 1], np.int32),
                         tau0=np.array([50.0, 50.0, 60.0, 60.0]),
                         kind=["o", "o", "t", "t"])
    law = _law()
    law.gamma_T = gamma_T
    return oracle.Solver(np.zeros((1, 1, 2), np.int32), np.zeros((1, 3)), _iso(), S.n_miller,
                         S.l_miller, S.family, S.tau0, law)


def test_section5_averages_from_a_hand_set_state():
    """<v^s>: mean over slip systems and voxels; <f_beta>: mean over twin
    systems and voxels of f = v_beta / gamma_T; <sigma>_eq: von Mises of the
    mean stress; <sigma_eq>: mean of the local von Mises stress.  Values
    worked out by hand."""
    s = _tiny_solver(1.0 / SQ2)
    # state columns: eps_p[6], v[4] (slip, slip, twin, twin), alpha[4]
    s.y[0, 6:10] = [0.1, 0.3, 0.05, 0.0]
    s.y[1, 6:10] = [0.2, 0.0, 0.01, 0.02]
    # voxel 0 uniaxial 100 MPa, voxel 1 pure shear 50 MPa (tensor comps)
    s.sig[0] = oracle.to_mandel([100.0, 0, 0, 0, 0, 0])
    s.sig[1] = oracle.to_mandel([0, 0, 0, 0, 0, 50.0])
    s.Sigma = np.array([50.0, 0, 0, 0, 0, 25.0])
    seq_mean, mean_seq, mv, mf = s.outputs()
    assert mv == pytest.approx(0.15, rel=1e-15)                    # (0.1+0.3+0.2+0)/4
    assert mf == pytest.approx(0.028284271247461901, rel=1e-14)    # 0.08/4 * sqrt2
    assert mean_seq == pytest.approx(93.301270189221932, rel=1e-14)  # (100 + 50 sqrt3)/2
    assert seq_mean == pytest.approx(66.143782776614765, rel=1e-14)  # sqrt(50^2 + 3 25^2)
    s2 = _tiny_solver(0.5)
    s2.y[:] = s.y
    assert s2.outputs()[3] == pytest.approx(0.04, rel=1e-14)        # 0.02 / 0.5


def test_schmid_half_crystal_first_yields_at_twice_tau0():
    """A single crystal oriented so that ordinary system 3 of Table 1 has the
    Schmid factor 1/2 along the load axis (the largest possible) and every
    other system a larger ratio tau0 / m: under uniaxial tension it is
    elastic while sigma_xx <= 2 tau0 = 260 MPa and slips once above (the
    resolved shear of equation 3 reaches the initial resistance), for any
    eta.  The step that first shows slip brackets 260 MPa."""
    C, law = rvegen.paper_law()
    S = rvegen.table1_systems(True)
    e = rvegen.schmid_half_orientation(S, 2)
    Q = oracle.euler_to_rotation(e)[0]
    mxx = oracle.lab_schmid(oracle.schmid_tensors(S.n_miller, S.l_miller), Q[None]).reshape(-1, 6)[:, 0]
    assert mxx[2] == pytest.approx(0.5, abs=1e-14)
    lim = [S.tau0[i] / abs(mxx[i]) if S.family[i] == 0 else (S.tau0[i] / mxx[i] if mxx[i] > 0 else np.inf)
           for i in range(16) if mxx[i] != 0]
    assert min(lim) == pytest.approx(260.0, rel=1e-14)
    rve = rvegen.Microstructure(labels=np.zeros((2, 2, 2), np.int32), euler=np.array([e]), n_grains=1,
                                twinned=np.zeros(0, np.int64), twin_fraction=np.zeros(0))
    for eta in (1e4, 1e5):
        law.eta = eta
        w = rvegen.Workload("point", rve, S, C, law, rvegen.uniaxial_path(0.005, 100))
        R = oracle.solver_for(w, oracle.Options(tol=1e-12, M=1)).run(w.path)
        k = int(np.argmax(R.mean_v > 0))
        assert k > 0 and R.Sigma[k - 1, 0] <= 260.0 < R.Sigma[k, 0], (eta, R.Sigma[k - 1:k + 1, 0])
        assert np.all(R.mean_v[:k] == 0.0)
