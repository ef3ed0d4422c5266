"""Pins of the oracle's Anderson-accelerated fixed point (an option beyond
the paper's basic scheme): it converges to the basic scheme's fixed point,
in fewer iterations, and reduces to the basic scheme at depth 0 and when
the history is degenerate; the mean strain stays the mean of the strain
field.  CPU only."""
import numpy as np
import pytest

import oracle
import rvegen


def _w(shape=(8, 8, 8), steps=4):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve(shape, 5, 3, twin_share=0.5)
    return rvegen.Workload("t", rve, rvegen.config_systems(True), C, law,
                           rvegen.uniaxial_path(0.008, steps, rate=1e-2))


@pytest.mark.parametrize("m", [1, 4, 8])
def test_same_fixed_point_fewer_iterations(m):
    w = _w()
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12)).run(w.path, keep_fields=True)
    s = oracle.solver_for(w, oracle.Options(tol=1e-12, aa_depth=m))
    R = s.run(w.path, keep_fields=True)
    assert np.abs(R.Sigma - ref.Sigma).max() <= 1e-8 * np.abs(ref.Sigma).max()
    assert np.abs(R.E - ref.E).max() <= 1e-9 * np.abs(ref.E).max()
    assert np.abs(R.fields["stress"] - ref.fields["stress"]).max() <= 1e-7 * np.abs(ref.fields["stress"]).max()
    if m >= 4:
        assert R.iters.sum() * 1.5 < ref.iters.sum(), (R.iters, ref.iters)
    # the mixed mean strain is the mean of the strain field
    assert np.allclose(oracle.from_mandel(s.eps).mean(axis=0), s.E, rtol=0, atol=1e-14)


def test_anderson_step_reduces_to_the_basic_step():
    rng = np.random.default_rng(0)
    x, f = rng.standard_normal((5, 6)), rng.standard_normal((5, 6))
    E, dE = rng.standard_normal(6), rng.standard_normal(6)
    hist = []
    xn, En = oracle.Solver._anderson(hist, x, f, E, dE, 4)       # no history yet
    assert np.array_equal(xn, x + f) and np.array_equal(En, E + dE)
    xn2, En2 = oracle.Solver._anderson(hist, x, f, E, dE, 4)     # zero differences: degenerate
    assert np.array_equal(xn2, x + f) and np.array_equal(En2, E + dE)


def test_linear_step_is_the_secant_solution():
    """For an affine step f(x) = b - A x the depth-1 update after two
    iterates removes the component of the residual along the last
    difference (Anderson = a secant method): f at the new iterate is
    orthogonal to dF in the affine case."""
    rng = np.random.default_rng(1)
    n = 12
    A = np.eye(n) * 0.5 + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    f = lambda x: b - A @ x
    hist = []
    x0 = np.zeros((2, 6))
    E = np.zeros(6)
    x1, _ = oracle.Solver._anderson(hist, x0, f(x0.ravel()).reshape(2, 6), E, E, 1)
    x2, _ = oracle.Solver._anderson(hist, x1, f(x1.ravel()).reshape(2, 6), E, E, 1)
    dF = f(x1.ravel()) - f(x0.ravel())
    # the least-squares residual f1 - dF gamma is orthogonal to dF
    f1 = f(x1.ravel())
    gam = (dF @ f1) / (dF @ dF)
    assert abs(dF @ (f1 - gam * dF)) < 1e-12 * np.linalg.norm(f1) * np.linalg.norm(dF)
    dX = (x1 - x0).ravel()
    assert np.allclose(x2.ravel(), x1.ravel() + f1 - gam * (dX + dF), rtol=0, atol=1e-12)
