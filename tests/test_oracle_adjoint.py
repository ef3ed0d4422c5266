"""Pins of the oracle's reverse mode: the rate and RK4 vector-Jacobian
products and the discrete adjoint of the whole load-stepped solve against
central finite differences of the forward oracle.  CPU only."""
import copy

import numpy as np
import pytest

import oracle
import rvegen


def _material(law, twins=True, tau0=None):
    C, _ = rvegen.config_law()
    S = rvegen.config_systems(twins)
    rve = rvegen.make_rve((4, 6, 8), 3, 77, twin_share=0.5 if twins else 0.0)
    return rve, S, C, oracle.Material(rve.euler, C, S.n_miller, S.l_miller, S.family,
                                      S.tau0 if tau0 is None else tau0, law)


def _perturbed(law, S, fam, name, h):
    l2 = copy.deepcopy(law)
    t0 = S.tau0.copy()
    if name == "r0":
        t0 = np.where(S.family == fam, t0 + h, t0)
    else:
        F = l2.slip if fam == 0 else l2.twin
        setattr(F, name, getattr(F, name) + h)
    return l2, t0


def _base(law, fam, name):
    if name == "r0":
        return 80.0 if fam == 0 else 120.0
    return getattr(law.slip if fam == 0 else law.twin, name)


def _plastic_point(rng, S):
    e = oracle.to_mandel(np.array([3e-3, -1.2e-3, -1.5e-3, 2e-4, -1e-4, 3e-4]))
    y = np.concatenate([rng.standard_normal(6) * 2e-4, rng.random(S) * 2e-3,
                        rng.standard_normal(S) * 1e-3])
    return e, y


@pytest.mark.parametrize("mode", [rvegen.TWIN_NORTON, rvegen.TWIN_PAPER])
def test_rate_vjp_matches_central_differences(mode):
    _, law = rvegen.config_law()
    law.twin_mode = mode
    if mode == rvegen.TWIN_PAPER:
        law.K_c, law.f_m = 1.45, 0.8
    rve, S, C, mat = _material(law)
    rng = np.random.default_rng(0)
    e, y = _plastic_point(rng, 16)
    D = mat.state_dim
    active = mat.rate(0, e, y)[6:22] > 0
    assert active[:12].sum() >= 2 and active[12:].sum() >= 1
    kb = rng.standard_normal(D)
    yb, eb, th = mat.rate_vjp(0, e, y, kb)
    f = lambda ee, yy, m=mat: kb @ m.rate(0, ee, yy)
    fd_y = np.array([(f(e, y + 1e-7 * np.eye(D)[q]) - f(e, y - 1e-7 * np.eye(D)[q])) / 2e-7
                     for q in range(D)])
    fd_e = np.array([(f(e + 1e-9 * np.eye(6)[q], y) - f(e - 1e-9 * np.eye(6)[q], y)) / 2e-9
                     for q in range(6)])
    assert np.abs(yb - fd_y).max() < 1e-6 * np.abs(fd_y).max()
    assert np.abs(eb - fd_e).max() < 1e-6 * np.abs(fd_e).max()
    for fam in (0, 1):
        for k, name in enumerate(oracle.THETA_NAMES):
            h = 1e-6 * max(abs(_base(law, fam, name)), 1.0)
            mp = oracle.Material(rve.euler, C, S.n_miller, S.l_miller, S.family,
                                 *_perturbed(law, S, fam, name, h)[::-1])
            mm = oracle.Material(rve.euler, C, S.n_miller, S.l_miller, S.family,
                                 *_perturbed(law, S, fam, name, -h)[::-1])
            fd = (kb @ mp.rate(0, e, y) - kb @ mm.rate(0, e, y)) / (2 * h)
            assert th[fam, k] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(fd) + 1e-14), (fam, name)


def test_rk4_vjp_matches_central_differences():
    _, law = rvegen.config_law()
    rve, S, C, mat = _material(law)
    rng = np.random.default_rng(1)
    e0, y0 = _plastic_point(rng, 16)
    e1 = e0 + oracle.to_mandel(np.array([4e-4, -2e-4, -1.5e-4, 0, 5e-5, 0]))
    D = mat.state_dim
    sb = rng.standard_normal(6)
    ybM = rng.standard_normal(D) * 1e3

    def J(a0, a1, yy):
        y1, s1 = mat.update([0], a0, a1, yy[None, :], 0.4, 8)
        return sb @ s1[0] + ybM @ y1[0]

    e0b, e1b, y0b, th = mat.update_vjp([0], e0, e1, y0[None, :], 0.4, 8, sb[None, :], ybM[None, :])
    for i in range(6):
        d = np.eye(6)[i] * 1e-9
        assert e1b[0, i] == pytest.approx((J(e0, e1 + d, y0) - J(e0, e1 - d, y0)) / 2e-9, rel=1e-5, abs=1e-3)
        assert e0b[0, i] == pytest.approx((J(e0 + d, e1, y0) - J(e0 - d, e1, y0)) / 2e-9, rel=1e-5, abs=1e-3)
    for q in (0, 3, 6, 10, 20, 30, 37):
        d = np.eye(D)[q] * 1e-8
        assert y0b[0, q] == pytest.approx((J(e0, e1, y0 + d) - J(e0, e1, y0 - d)) / 2e-8, rel=1e-5, abs=1e-2)


def test_discrete_adjoint_gradient_matches_finite_differences():
    """Loss over 3 load steps of a 4x4x6 twinned RVE; all 14 parameters."""
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    rve = rvegen.make_rve((4, 4, 6), 3, 77, twin_share=0.5)
    path = rvegen.uniaxial_path(0.006, 3, rate=1e-2)
    w = rvegen.Workload("t", rve, S, C, law, path)
    o = oracle.solver_for(w, oracle.Options(tol=1e-12))
    tgt = o.run(path).Sigma[:, 0] * 1.03
    L, grad, _ = o.gradient(path, tgt, adj_tol=1e-12)
    assert L > 0

    def Lof(fam, name, h):
        l2, t0 = _perturbed(law, S, fam, name, h)
        sv = oracle.Solver(rve.labels, rve.euler, C, S.n_miller, S.l_miller, S.family, t0, l2,
                           oracle.Options(tol=1e-12))
        return float(np.sum((sv.run(path).Sigma[:, 0] - tgt) ** 2))

    for fam in (0, 1):
        for k, name in enumerate(oracle.THETA_NAMES):
            h = 1e-6 * max(abs(_base(law, fam, name)), 1.0)
            fd = (Lof(fam, name, h) - Lof(fam, name, -h)) / (2 * h)
            scale = np.abs(grad[fam]).max()
            assert abs(grad[fam, k] - fd) <= 1e-6 * abs(fd) + 1e-5 * scale, (fam, name, grad[fam, k], fd)
    assert np.abs(grad[1]).max() > 0        # the twin family is active


@pytest.mark.parametrize("green", ["continuous", "rotated"])
def test_vjp_general_cotangent_matches_finite_differences(green):
    """J = sum_n Sigma_bar_n . Sigma_n with a cotangent on all six
    components (shear included, tensor components) against central
    differences of the forward solves, for parameters of both families,
    with either Green operator (the adjoint equilibrium uses the same
    operator as the forward solve)."""
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    rve = rvegen.make_rve((4, 4, 6), 3, 77, twin_share=0.5)
    path = rvegen.uniaxial_path(0.006, 3, rate=1e-2)
    w = rvegen.Workload("t", rve, S, C, law, path)
    o = oracle.solver_for(w, oracle.Options(tol=1e-12, green=green))
    sb = np.random.default_rng(3).standard_normal((3, 6))
    grad, Sig = o.vjp(path, sb, adj_tol=1e-12)
    assert np.abs(Sig[:, 3:]).max() > 0      # shear stresses are not zero

    def J(fam, name, h):
        l2, t0 = _perturbed(law, S, fam, name, h)
        sv = oracle.Solver(rve.labels, rve.euler, C, S.n_miller, S.l_miller, S.family, t0, l2,
                           oracle.Options(tol=1e-12, green=green))
        return float(np.sum(sb * sv.run(path).Sigma))

    for fam, name in ((0, "r0"), (0, "K"), (0, "c"), (1, "r0"), (1, "n")):
        k = oracle.THETA_NAMES.index(name)
        h = 1e-6 * max(abs(_base(law, fam, name)), 1.0)
        fd = (J(fam, name, h) - J(fam, name, -h)) / (2 * h)
        scale = np.abs(grad[fam]).max()
        assert abs(grad[fam, k] - fd) <= 1e-6 * abs(fd) + 1e-5 * scale, (fam, name, grad[fam, k], fd)
    # the stress-curve loss is the special cotangent 2 (Sigma_xx - target) e_xx
    tgt = Sig[:, 0] * 1.02
    L, g2, sxx = o.gradient(path, tgt, adj_tol=1e-12)
    cot = np.zeros((3, 6))
    cot[:, 0] = 2 * (Sig[:, 0] - tgt)
    g3, _ = o.vjp(path, cot, adj_tol=1e-12)
    assert np.allclose(g2, g3, rtol=1e-12, atol=1e-12 * np.abs(g2).max())
    assert np.array_equal(sxx, Sig[:, 0])
