"""Pins of the oracle's von Mises stress and its histogram (the statistic
of the paper's probability density of sigma_eq): closed forms of uniaxial,
shear and hydrostatic states, invariance under rotation and added
pressure, and the placement of values at and around bin edges."""
import numpy as np

import oracle


def _tensor_to_comps(T):
    return np.array([T[0, 0], T[1, 1], T[2, 2], T[1, 2], T[0, 2], T[0, 1]])


def test_closed_forms():
    a = np.array([250.0, -37.5, 1e-3])
    z = np.zeros_like(a)
    assert np.allclose(oracle.von_mises_field([a, z, z, z, z, z]), np.abs(a), rtol=2e-16, atol=0)
    assert np.allclose(oracle.von_mises_field([z, a, z, z, z, z]), np.abs(a), rtol=2e-16, atol=0)
    tau = np.array([10.0, -4.0])
    z2 = np.zeros_like(tau)
    assert np.allclose(oracle.von_mises_field([z2, z2, z2, z2, z2, tau]), np.sqrt(3) * np.abs(tau), rtol=4e-16)
    assert np.allclose(oracle.von_mises_field([z2, z2, z2, tau, z2, z2]), np.sqrt(3) * np.abs(tau), rtol=4e-16)
    p = np.array([100.0, -3.0])
    assert np.all(oracle.von_mises_field([p, p, p, z2, z2, z2]) == 0.0)
    # equal biaxial = uniaxial of the same magnitude
    assert np.allclose(oracle.von_mises_field([tau, tau, z2, z2, z2, z2]), np.abs(tau), rtol=4e-16)


def test_invariance_under_rotation_and_pressure():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3)) * 100
    T = 0.5 * (A + A.T)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    q0 = oracle.von_mises_field(_tensor_to_comps(T)[:, None])
    q1 = oracle.von_mises_field(_tensor_to_comps(Q @ T @ Q.T)[:, None])
    q2 = oracle.von_mises_field(_tensor_to_comps(T + 321.0 * np.eye(3))[:, None])
    assert abs(q1[0] - q0[0]) < 1e-12 * q0[0] and abs(q2[0] - q0[0]) < 1e-12 * q0[0]
    # via the deviatoric principal values: sqrt(3/2) |eigs(dev T)|
    dev = T - np.trace(T) / 3 * np.eye(3)
    assert abs(q0[0] - np.sqrt(1.5 * np.sum(np.linalg.eigvalsh(dev) ** 2))) < 1e-12 * q0[0]


def test_histogram_bins_and_edges():
    lo, hi, nb = 100.0, 250.0, 6           # width 25: edges 100, 125, ..., 250
    vals = np.array([99.0, 100.0, 112.5, 124.999, 125.0, 249.999, 250.0, 400.0, np.nan])
    z = np.zeros_like(vals)
    c = oracle.von_mises_histogram([np.stack([vals, z, z, z, z, z])], nb, lo, hi)
    # uniaxial s11 = v gives sigma_eq = v for these values exactly
    assert list(c) == [1, 3, 1, 0, 0, 0, 1, 3]
    assert int(c.sum()) == vals.size
    # several fields accumulate
    c2 = oracle.von_mises_histogram([np.stack([vals, z, z, z, z, z])] * 2, nb, lo, hi)
    assert np.array_equal(c2, 2 * c)


def test_histogram_range_below_zero():
    """Edges at or below zero lie below every von Mises stress."""
    vals = np.array([0.0, 10.0, 24.9, 30.0, 60.0])
    z = np.zeros_like(vals)
    c = oracle.von_mises_histogram([np.stack([vals, z, z, z, z, z])], 4, -50.0, 50.0)
    # bins [-50,-25), [-25,0), [0,25), [25,50)
    assert list(c) == [0, 0, 0, 3, 1, 1]
