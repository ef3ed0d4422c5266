"""Pins of the oracle's frozen error-controlled substep counts (an option
beyond the paper's fixed RK4 substeps): the probe reduces to the fixed
count when every point passes, chooses the least passing count (checked
against separate fixed-count integrations), caps at the largest, keeps the
fixed point convergent, and approaches a fine fixed-count reference as the
tolerance falls.  CPU only."""
import numpy as np
import pytest

import oracle
import rvegen


def _w(steps=3):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve((6, 6, 6), 4, 3, twin_share=0.5)
    return rvegen.Workload("t", rve, rvegen.config_systems(True), C, law,
                           rvegen.uniaxial_path(0.006, steps, rate=1e-2))


def _state(w, seed=1):
    S = w.systems.family.shape[0]
    mat = oracle.Material(w.rve.euler, w.C, w.systems.n_miller, w.systems.l_miller, w.systems.family,
                          w.systems.tau0, w.law)
    rng = np.random.default_rng(seed)
    n = w.rve.labels.size
    e0 = rng.standard_normal((n, 6)) * 1e-3
    e1 = e0 + rng.standard_normal((n, 6)) * 2e-3
    y0 = np.zeros((n, 6 + 2 * S))
    y0[:, 6:6 + S] = rng.random((n, S)) * 1e-3
    return mat, w.rve.labels.ravel(), e0, e1, y0


def _err2(a, b, S):
    f = np.sum((a[:, :6] - b[:, :6]) ** 2, axis=1)
    m = np.max((a[:, 6:] - b[:, 6:]) ** 2, axis=1)
    return np.maximum(f, m)


def test_probe_reduces_to_the_fixed_count():
    w = _w()
    mat, lab, e0, e1, y0 = _state(w)
    y, s, j = mat.probe(lab, e0, e1, y0, 0.4, 8, 1.0, 4)
    yf, sf = mat.update(lab, e0, e1, y0, 0.4, 8)
    assert np.all(j == 0) and np.array_equal(y, yf) and np.array_equal(s, sf)
    y2, s2 = mat.update_j(lab, e0, e1, y0, 0.4, 8, np.full(lab.size, 2))
    y3, s3 = mat.update(lab, e0, e1, y0, 0.4, 32)
    assert np.array_equal(y2, y3) and np.array_equal(s2, s3)


@pytest.mark.parametrize("tol", [1e-5, 1e-6])
def test_probe_takes_the_least_passing_count(tol):
    w = _w()
    mat, lab, e0, e1, y0 = _state(w)
    S = w.systems.family.shape[0]
    M, maxd = 2, 4
    y, s, j = mat.probe(lab, e0, e1, y0, 0.4, M, tol, maxd)
    ys = [mat.update(lab, e0, e1, y0, 0.4, M << k)[0] for k in range(maxd + 1)]
    lim = (15 * tol) ** 2
    passes = np.stack([_err2(ys[k], ys[k + 1], S) <= lim for k in range(maxd)], axis=1)
    first = np.where(passes.any(axis=1), passes.argmax(axis=1), maxd)
    assert np.array_equal(j, first)
    assert len(np.unique(j)) >= 2                    # points differ in their counts
    for k in range(maxd + 1):
        sel = j == k
        assert np.array_equal(y[sel], ys[k][sel])


def test_probe_caps_at_the_largest_count():
    w = _w()
    mat, lab, e0, e1, y0 = _state(w)
    y, s, j = mat.probe(lab, e0, e1, y0, 0.4, 2, 1e-15, 3)
    plastic = np.abs(mat.update(lab, e0, e1, y0, 0.4, 2)[0][:, :6] - y0[:, :6]).max(axis=1) > 0
    assert np.all(j[plastic] == 3)


def test_solve_converges_and_approaches_the_fine_reference():
    w = _w()
    ref = oracle.solver_for(w, oracle.Options(tol=1e-11, M=64)).run(w.path)
    errs = []
    for tol in (1e-6, 1e-7, 1e-8):
        s = oracle.solver_for(w, oracle.Options(tol=1e-11, rk_tol=tol))
        R = s.run(w.path)                      # converges to 1e-11 (raises otherwise)
        errs.append(np.abs(R.Sigma - ref.Sigma).max())
    fixed = np.abs(oracle.solver_for(w, oracle.Options(tol=1e-11)).run(w.path).Sigma - ref.Sigma).max()
    assert errs[0] <= fixed * (1 + 1e-12) and errs[2] < errs[0] and errs[2] < 0.2 * fixed
