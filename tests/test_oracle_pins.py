"""Pins of the CPU oracle against facts that do not come from the oracle:
the paper's printed table, brute-force transforms, closed forms of the law,
exact laminate solutions, bounds and symmetries.  CPU only."""
import math
import os

import numpy as np
import pytest

import oracle
import rvegen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _iso_voigt(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return rvegen.cubic_stiffness(lam + 2 * mu, lam, mu), lam, mu


def _law(Q=0.0, b=10.0, c=0.0, d=0.0, K=10.0, n=10.0, eta=1e4, qs=1.0, ql=1.4):
    fam = rvegen.FamilyLaw(Q=Q, b=b, c=c, d=d, K=K, n=n, q_self=qs, q_latent=ql)
    return rvegen.Law(slip=fam, twin=rvegen.FamilyLaw(**vars(fam)), eta=eta)


# ---------------------------------------------------------------------------
# Table 1
# ---------------------------------------------------------------------------
def test_table1_as_printed_and_the_system9_reading():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_systems.txt"))
            if l.strip() and not l.startswith("#")]
    printed = np.array([[int(v) for v in r[2:8]] for r in rows], dtype=float)
    kinds = [r[1] for r in rows]
    # every printed plane is a {111} and every pair is orthogonal
    assert np.all(np.abs(printed[:, :3]) == 1)
    assert np.all(np.einsum("ij,ij->i", printed[:, :3], printed[:, 3:]) == 0)
    # the printed system 9 duplicates system 7
    assert np.array_equal(printed[6], printed[8])
    S = rvegen.table1_systems()
    assert [k for k in S.kind] == kinds
    same = np.all(np.hstack([S.n_miller, S.l_miller]) == printed, axis=1)
    assert same.sum() == 15 and not same[8]
    # read direction: the in-plane [1 +-1 0] of (1-11), like systems 3, 6, 12
    assert np.dot(S.n_miller[8], S.l_miller[8]) == 0
    assert S.l_miller[8][2] == 0
    for s in (2, 5, 11):
        assert S.l_miller[s][2] == 0 and abs(S.l_miller[s]).sum() == 2
    # twins: 4 distinct planes, <112> directions
    assert len({tuple(r) for r in S.n_miller[12:]}) == 4
    assert np.all(np.sort(np.abs(S.l_miller[12:]), axis=1) == [1, 1, 2])


# ---------------------------------------------------------------------------
# DFT and Green operator
# ---------------------------------------------------------------------------
def test_fft_matches_brute_force_dft():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((2, 3, 4, 6))
    nz, ny, nx = f.shape[1:]
    ref = np.zeros(f.shape, dtype=complex)
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                for z in range(nz):
                    for y in range(ny):
                        for x in range(nx):
                            w = np.exp(-2j * np.pi * (kz * z / nz + ky * y / ny + kx * x / nx))
                            ref[:, kz, ky, kx] += f[:, z, y, x] * w
    assert np.allclose(oracle.fft3(f), ref, rtol=0, atol=1e-12)
    assert np.allclose(oracle.ifft3_real(oracle.fft3(f)), f, atol=1e-14)


def _gamma_matrix(xi, lam0, mu0):
    """6x6 matrix of the oracle's Gamma0 at one frequency, in Mandel form."""
    shape = (1, 1, 1)
    G = np.zeros((6, 6))
    for J in range(6):
        e = np.zeros(6)
        e[J] = 1.0 / oracle.MANDEL_W[J]          # Mandel unit vector -> tensor comps
        tau = e.reshape(6, 1, 1, 1).astype(complex)
        out = oracle.gamma0_apply(tau, lam0, mu0, xi.reshape(3, 1, 1, 1),
                                  np.ones(shape, bool))
        G[:, J] = (out.reshape(6) * oracle.MANDEL_W).real
    return G


def test_gamma0_is_a_c0_projector_of_rank_3():
    lam0, mu0 = 57583.3, 79625.0
    C0 = oracle.iso_stiffness(lam0, mu0)
    rng = np.random.default_rng(2)
    for _ in range(5):
        xi = rng.standard_normal(3)
        xi /= np.linalg.norm(xi)
        G = _gamma_matrix(xi, lam0, mu0)
        assert np.allclose(G, G.T, atol=1e-18)
        assert np.allclose(G @ C0 @ G, G, rtol=0, atol=1e-16)
        assert np.linalg.matrix_rank(G, tol=1e-12 / mu0) == 3
        # compatible strains sym(xi (x) u) are reproduced: Gamma0 C0 e = e
        u = rng.standard_normal(3)
        e = oracle.to_mandel(oracle.mat_to_sym(0.5 * (np.outer(xi, u) + np.outer(u, xi))))
        assert np.allclose(G @ C0 @ e, e, atol=1e-14)
        # divergence-free stresses (sigma . xi = 0) are annihilated
        a, b = np.linalg.svd(xi.reshape(1, 3))[2][1:]
        s = oracle.to_mandel(oracle.mat_to_sym(np.outer(a, a) + 0.3 * np.outer(a, b)
                                               + 0.3 * np.outer(b, a)))
        assert np.allclose(G @ s, 0, atol=1e-18)
        # evenness in xi
        assert np.allclose(_gamma_matrix(-xi, lam0, mu0), G)


def test_green_convolution_recovers_a_compatible_field():
    """eps = sym grad u of a periodic u (Fourier synthesis without Nyquist
    content): Gamma0 * (C0 : eps) = eps - <eps> on the grid."""
    shape = (6, 8, 10)
    lam0, mu0 = 1.1e5, 8.0e4
    rng = np.random.default_rng(3)
    xi_hat, ctrl = oracle.frequency_directions(shape)
    nz, ny, nx = shape
    ms = [np.where(np.arange(N) <= N // 2, np.arange(N), np.arange(N) - N) / N
          for N in (nx, ny, nz)]
    MZ, MY, MX = np.meshgrid(ms[2], ms[1], ms[0], indexing="ij")
    xi = np.stack([MX, MY, MZ])
    u = np.fft.fftn(rng.standard_normal((3,) + shape), axes=(1, 2, 3))
    u = np.where(ctrl, u, 0)
    grad = 1j * 2 * np.pi * xi[:, None] * u[None, :]        # d u_j / d x_i
    eps_hat = 0.5 * (grad + np.swapaxes(grad, 0, 1))
    eps = np.fft.ifftn(eps_hat, axes=(2, 3, 4)).real
    eps6 = np.stack([eps[i, j] for (i, j) in oracle.VOIGT_PAIRS]) + 1e-3  # add a mean
    C0 = oracle.iso_stiffness(lam0, mu0)
    sig = np.einsum("ij,j...->i...", C0, eps6)
    out = oracle.ifft3_real(oracle.gamma0_apply(oracle.fft3(sig), lam0, mu0))
    assert np.abs(out.mean(axis=(1, 2, 3))).max() < 1e-15 * np.abs(out).max()
    assert np.allclose(out, eps6 - 1e-3, rtol=0, atol=1e-13 * np.abs(eps6).max())


def _rotated_gradient(u):
    """Rotated-scheme derivatives of a field u[..., nz, ny, nx] given at the
    voxel corners (node (i,j,k) is the lower corner of voxel (i,j,k)): the
    derivative along an axis at a voxel centre is the mean of the four
    differences along the voxel edges parallel to that axis.  Returns
    [3 (d/dx, d/dy, d/dz), ...]."""
    ax = {0: -1, 1: -2, 2: -3}
    out = []
    for d in range(3):
        diff = np.roll(u, -1, axis=ax[d]) - u
        o1, o2 = [ax[e] for e in range(3) if e != d]
        acc = 0.0
        for a in (0, 1):
            for b in (0, 1):
                acc = acc + np.roll(np.roll(diff, -a, axis=o1), -b, axis=o2)
        out.append(0.25 * acc)
    return np.stack(out)


def _rotated_divergence(T):
    """Transpose of the rotated-scheme gradient applied to a voxel-centred
    tensor field T[i, j, nz, ny, nx]: sum_j D_j^T T_ij at the corners, with
    (D_j^T f)(n) = 1/4 sum over the four voxels around each edge through n
    parallel to j of f(voxel below along j) - f(voxel above)."""
    ax = {0: -1, 1: -2, 2: -3}
    out = np.zeros((3,) + T.shape[2:])
    for i in range(3):
        for d in range(3):
            f = T[i, d]
            diff = np.roll(f, 1, axis=ax[d]) - f
            o1, o2 = [ax[e] for e in range(3) if e != d]
            for a in (0, 1):
                for b in (0, 1):
                    out[i] += 0.25 * np.roll(np.roll(diff, a, axis=o1), b, axis=o2)
    return out


def _as_tensor(s6):
    T = np.empty((3, 3) + s6.shape[1:])
    for c, (i, j) in enumerate(oracle.VOIGT_PAIRS):
        T[i, j] = T[j, i] = s6[c]
    return T


@pytest.mark.parametrize("shape", [(6, 8, 10), (4, 5, 6), (3, 4, 9)])
def test_rotated_green_recovers_a_rotated_scheme_compatible_field(shape):
    """eps = sym grad_h u of a random corner displacement field, grad_h the
    rotated finite differences written out in real space: the rotated
    operator reproduces it, Gamma0 * (C0 : eps) = eps - <eps>, also with
    Nyquist content (the continuous operator does not)."""
    lam0, mu0 = 1.1e5, 8.0e4
    rng = np.random.default_rng(4)
    u = rng.standard_normal((3,) + shape)
    g = _rotated_gradient(u)                       # g[i, j] = d u_j / d x_i
    eps = 0.5 * (g + np.swapaxes(g, 0, 1))
    eps6 = np.stack([eps[i, j] for (i, j) in oracle.VOIGT_PAIRS]) + 1e-3
    C0 = oracle.iso_stiffness(lam0, mu0)
    sig = np.einsum("ij,j...->i...", C0, eps6)
    xi, ctrl = oracle.frequency_directions_rotated(shape)
    out = oracle.ifft3_real(oracle.gamma0_apply(oracle.fft3(sig), lam0, mu0, xi, ctrl))
    assert np.allclose(out, eps6 - 1e-3, rtol=0, atol=1e-13 * np.abs(eps6).max())
    cont = oracle.ifft3_real(oracle.gamma0_apply(oracle.fft3(sig), lam0, mu0))
    assert np.abs(cont - (eps6 - 1e-3)).max() > 1e-3 * np.abs(eps6).max()
    # for any polarization tau, sigma = C0 : (-Gamma0 * tau) + tau is in
    # equilibrium under the rotated divergence (the transposed stencil)
    tau = rng.standard_normal((6,) + shape)
    e = -oracle.ifft3_real(oracle.gamma0_apply(oracle.fft3(tau), lam0, mu0, xi, ctrl))
    sg = np.einsum("ij,j...->i...", C0, e) + tau
    div = _rotated_divergence(_as_tensor(sg))
    assert np.abs(div).max() < 1e-12 * np.abs(tau).max()
    ec = -oracle.ifft3_real(oracle.gamma0_apply(oracle.fft3(tau), lam0, mu0))
    div_c = _rotated_divergence(_as_tensor(np.einsum("ij,j...->i...", C0, ec) + tau))
    assert np.abs(div_c).max() > 1e-3 * np.abs(tau).max()


def test_rotated_directions_special_frequencies():
    """s / |s| at a single Nyquist component is the axis itself; with two
    or more Nyquist components (and at zero) s vanishes; at low frequency
    the direction tends to the continuous one."""
    shape = (4, 6, 8)
    xi, ctrl = oracle.frequency_directions_rotated(shape)
    assert np.allclose(xi[:, 0, 0, 4], [1, 0, 0]) and ctrl[0, 0, 4]
    assert np.allclose(xi[:, 0, 3, 0], [0, 1, 0]) and ctrl[0, 3, 0]
    assert np.allclose(xi[:, 2, 0, 0], [0, 0, 1]) and ctrl[2, 0, 0]
    assert np.abs(xi[:, 1, 3, 4]).max() == 0 and not ctrl[1, 3, 4]
    assert np.abs(xi[:, 2, 2, 4]).max() == 0 and not ctrl[2, 2, 4]
    assert not ctrl[0, 0, 0] and not ctrl[2, 3, 4]
    assert int((~ctrl).sum()) == 1 + (4 + 6 + 8 - 2)
    # (1, 1, 1) of a 256^3 grid vs the continuous direction
    xr = oracle.frequency_directions_rotated((256, 256, 256))[0][:, 1, 2, 3]
    xc = oracle.frequency_directions((256, 256, 256))[0][:, 1, 2, 3]
    assert np.allclose(xr, xc, atol=1e-4) and not np.allclose(xr, xc, atol=1e-7)


def test_reference_medium_closed_form_for_cubic():
    C = rvegen.cubic_stiffness(183000.0, 74500.0, 105000.0)
    lam0, mu0 = oracle.reference_medium(C)
    k0 = (183000.0 + 2 * 74500.0) / 3
    assert math.isclose(mu0, 0.5 * ((183000.0 - 74500.0) / 2 + 105000.0), rel_tol=1e-13)
    assert math.isclose(lam0, k0 - 2 * mu0 / 3, rel_tol=1e-13)


# ---------------------------------------------------------------------------
# Rotations
# ---------------------------------------------------------------------------
def test_rotations_of_stiffness_and_schmid():
    C = rvegen.tetragonal_stiffness(183000.0, 170000.0, 74000.0, 70000.0, 105000.0, 78000.0)
    Q0 = oracle.euler_to_rotation([[0, 0, 0]])
    assert np.allclose(Q0[0], np.eye(3))
    CM = oracle.mandel_of_tensor4(oracle.stiffness_tensor(C))
    assert np.allclose(oracle.lab_stiffness(C, Q0)[0], CM)
    # 90 degrees about x maps crystal axis 3 onto lab axis 2: c33 -> C22
    Qx = oracle.euler_to_rotation([[0, math.pi / 2, 0]])
    Cl = oracle.lab_stiffness(C, Qx)[0]
    assert math.isclose(Cl[1, 1], 170000.0, rel_tol=1e-12)
    assert math.isclose(Cl[2, 2], 183000.0, rel_tol=1e-12)
    # isotropic stiffness is invariant under any rotation
    Ci, lam, mu = _iso_voigt(200000.0, 0.3)
    Qr = rvegen.bunge_to_matrix(np.random.default_rng(4).random((3, 3)) * 3)
    assert np.allclose(oracle.lab_stiffness(Ci, Qr), oracle.iso_stiffness(lam, mu), atol=1e-9)
    # Schmid tensors are traceless with |m|^2 = 1/2
    m = oracle.schmid_tensors(rvegen.table1_systems().n_miller, rvegen.table1_systems().l_miller)
    assert np.allclose(np.trace(m, axis1=1, axis2=2), 0)
    assert np.allclose(np.sum(m * m, axis=(1, 2)), 0.5)


# ---------------------------------------------------------------------------
# Local law
# ---------------------------------------------------------------------------
def test_regularized_rate_solves_its_equation():
    for (o, A, K, n, eta) in [(10.0, 1.0, 10.0, 10.0, 1e4), (150.0, 1.0, 104.0, 6.42, 1e4),
                              (0.5, 0.3, 10.0, 10.0, 1e4), (40.0, 1.0, 10.0, 10.0, 1.0),
                              (3.0, 1.0, 10.0, 3.0, 1e3)]:
        g = oracle.reg_rate(o, A, K, n, eta)
        # g = A < (o - eta g)/K >^n, checked by bisection on the same equation
        lo, hi = 0.0, o / eta
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid - A * max(0.0, (o - eta * mid) / K) ** n > 0:
                hi = mid
            else:
                lo = mid
        assert math.isclose(g, lo, rel_tol=1e-12), (o, g, lo)
    assert oracle.reg_rate(-1.0, 1.0, 10.0, 10.0, 1e4) == 0.0
    assert oracle.reg_rate(5.0, 1.0, 10.0, 10.0, 0.0) == pytest.approx(0.5 ** 10, rel=1e-14)
    # linear viscosity (n = 1) has the closed form g = A o / (K + eta A)
    assert oracle.reg_rate(5.0, 0.7, 10.0, 1.0, 1e4) == pytest.approx(0.7 * 5 / (10 + 7e3), rel=1e-14)


def _one_system_material(law, tau0=50.0, family=0, n=(0, 1, 0), l=(1, 0, 0)):
    C, lam, mu = _iso_voigt(200000.0, 0.3)
    mat = oracle.Material([[0, 0, 0]], C, [n], [l], [family], [tau0], law)
    return mat, mu


def _drive_shear(mat, rate, t_end, dt, M, sign=1.0):
    y = np.zeros((1, mat.state_dim))
    eps = np.zeros(6)
    t = 0.0
    hist = []
    while t < t_end - 1e-12:
        e1 = eps.copy()
        e1[5] += sign * math.sqrt(2.0) * 0.5 * rate * dt      # Mandel sqrt2*eps12
        y, sig = mat.update([0], eps, e1, y, dt, M)
        eps, t = e1, t + dt
        hist.append((t, sig[0, 5] / math.sqrt(2.0), y[0].copy()))
    return hist


@pytest.mark.parametrize("Q,c,d", [(0.0, 0.0, 0.0), (40.0, 1e4, 300.0)])
def test_single_slip_steady_state_closed_form(Q, c, d):
    """One slip system in simple shear at constant rate: at steady state the
    slip rate equals the imposed rate and tau = r_sat + x_sat + K g^(1/n) + eta g."""
    law = _law(Q=Q, b=10.0, c=c, d=d, K=10.0, n=10.0, eta=1e4)
    mat, mu = _one_system_material(law, tau0=50.0)
    g = 0.02
    hist = _drive_shear(mat, g, 400.0, 1.0, 20)
    tau = hist[-1][1]
    expect = 50.0 + Q * 1.0 + (c / d if d else 0.0) + 10.0 * g ** 0.1 + 1e4 * g
    assert tau == pytest.approx(expect, rel=1e-9)
    # accumulated slip equals the plastic shear, plastic strain is traceless
    y = hist[-1][2]
    assert y[6] == pytest.approx(2 * y[5] / math.sqrt(2.0), rel=1e-12)
    assert abs(y[0] + y[1] + y[2]) < 1e-18


def test_elastic_point_is_exact_and_rk4_is_fourth_order():
    law = _law(Q=40.0, c=1e4, d=300.0)
    mat = oracle.Material([[0.3, 0.7, 1.1]], rvegen.cubic_stiffness(183000.0, 74500.0, 105000.0),
                          rvegen.table1_systems().n_miller, rvegen.table1_systems().l_miller,
                          rvegen.table1_systems().family, np.full(16, 80.0), law)
    e1 = oracle.to_mandel([2e-4, -5e-5, -5e-5, 1e-5, 0, 2e-5])
    y, sig = mat.update([0], np.zeros(6), e1, np.zeros((1, mat.state_dim)), 0.2, 4)
    assert np.all(y == 0)
    assert np.allclose(sig[0], mat.C_lab[0] @ e1, rtol=1e-15, atol=1e-12)
    # plastic increment: error against a fine reference drops ~16x per halving
    e0 = oracle.to_mandel([3e-3, -1.5e-3, -1.5e-3, 0, 0, 0])
    y0, _ = mat.update([0], np.zeros(6), e0, np.zeros((1, mat.state_dim)), 3.0, 400)
    e1 = oracle.to_mandel([4e-3, -2e-3, -2e-3, 0, 0, 0])
    ref, _ = mat.update([0], e0, e1, y0, 1.0, 2048)
    errs = []
    for M in (16, 32, 64):
        yM, _ = mat.update([0], e0, e1, y0, 1.0, M)
        errs.append(np.abs(yM - ref).max())
    assert errs[0] > 0 and 10 < errs[0] / errs[1] < 22 and 10 < errs[1] / errs[2] < 22
    assert abs(ref[0, :3].sum()) < 1e-18 * 100


def test_twinning_is_unidirectional_and_saturates():
    law = _law(Q=0.0, K=104.0, n=6.42, eta=1e4)
    law.twin_mode = rvegen.TWIN_PAPER
    law.K_c, law.f_m = 1.45, 0.8
    mat, mu = _one_system_material(law, tau0=130.0, family=1)
    neg = _drive_shear(mat, 0.05, 20.0, 0.5, 10, sign=-1.0)
    assert neg[-1][2][6] == 0.0                       # no twinning under reversed shear
    pos = _drive_shear(mat, 0.05, 200.0, 0.5, 10)
    f = np.array([h[2][6] for h in pos]) / law.gamma_T
    # the fraction rises monotonically to f_m (explicit RK4 may overshoot it
    # slightly once the rate prefactor becomes stiff; it then stops)
    assert np.all(np.diff(f) >= 0) and f[-1] == pytest.approx(0.8, abs=2e-3)
    # norton mode: no saturation, same sign rule
    law.twin_mode = rvegen.TWIN_NORTON
    mat2, _ = _one_system_material(law, tau0=130.0, family=1)
    assert _drive_shear(mat2, 0.05, 20.0, 0.5, 10, sign=-1.0)[-1][2][6] == 0.0


# ---------------------------------------------------------------------------
# Fixed-point solver
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(4, 4, 6), (2, 6, 4), (3, 4, 4)])
def test_nyquist_formula_is_the_real_part_of_the_full_inverse(shape):
    """With nyquist='formula', Gamma0 * tau is the real part of the inverse
    DFT, summed here by brute force, of the formula applied at every nonzero
    frequency with Nyquist components at +N/2 (directions built here from
    the indices); on an odd grid there is nothing to differ from 'zero'."""
    lam0, mu0 = 57583.3, 79625.0
    rng = np.random.default_rng(11)
    tau = rng.standard_normal((6,) + shape)
    nz, ny, nx = shape
    th = oracle.fft3(tau)
    ref = np.zeros((6,) + shape, dtype=complex)
    grid = np.stack(np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij"))
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                m = np.array([kx if 2 * kx <= nx else kx - nx, ky if 2 * ky <= ny else ky - ny,
                              kz if 2 * kz <= nz else kz - nz], float) / np.array([nx, ny, nz])
                if not m.any():
                    continue
                G = _gamma_matrix(m / np.linalg.norm(m), lam0, mu0)
                e = (G @ (th[:, kz, ky, kx] * oracle.MANDEL_W)) / oracle.MANDEL_W
                ph = np.exp(2j * np.pi * (kz * grid[0] / nz + ky * grid[1] / ny + kx * grid[2] / nx))
                ref += e[:, None, None, None] * ph[None] / tau[0].size
    xi, ctrl = oracle.frequency_directions(shape, "formula")
    out = oracle.ifft3_real(oracle.gamma0_apply(th, lam0, mu0, xi, ctrl))
    assert np.allclose(out, ref.real, rtol=0, atol=1e-13 * np.abs(ref).max())
    assert np.abs(ref.imag).max() > 1e-6 * np.abs(ref.real).max()   # the formula is not Hermitian there
    xz, cz = oracle.frequency_directions(shape, "zero")
    assert not np.allclose(oracle.ifft3_real(oracle.gamma0_apply(th, lam0, mu0, xz, cz)), out)
    xo, co = oracle.frequency_directions((3, 5, 7), "formula")
    xe, ce = oracle.frequency_directions((3, 5, 7), "zero")
    assert np.array_equal(co, ce) and np.array_equal(xo, xe)


def _solver(labels, euler, C, law, systems=None, **kw):
    S = systems or rvegen.config_systems(False)
    return oracle.Solver(labels, euler, C, S.n_miller, S.l_miller, S.family,
                         kw.pop("tau0", S.tau0), law, oracle.Options(**kw))


def test_homogeneous_reference_medium_converges_in_one_iteration():
    C, lam, mu = _iso_voigt(200000.0, 0.3)
    C0 = rvegen.cubic_stiffness(lam + 2 * mu, lam, mu)
    labels = np.zeros((4, 6, 8), np.int32)
    s = _solver(labels, [[0.1, 0.2, 0.3]], C0, _law(), tau0=np.full(12, 1e9), tol=1e-12)
    path = rvegen.uniaxial_path(1e-3, 2)
    R = s.run(path)
    E, nu = 200000.0, 0.3
    assert np.allclose(R.Sigma[:, 0], E * path.target[:, 0], rtol=1e-12)
    assert np.allclose(R.E[:, 1], -nu * path.target[:, 0], rtol=1e-12)
    assert R.iters[0] <= 2


@pytest.mark.parametrize("green,nyquist,lo,hi", [("continuous", "zero", 4, 10), ("rotated", "zero", 4, 10),
                                                ("rotated", "zero", 3, 10), ("continuous", "formula", 3, 10),
                                                ("continuous", "formula", 4, 10)])
def test_two_phase_laminate_closed_form(green, nyquist, lo, hi):
    """Layers normal to x of two orientations of a cubic crystal, elastic.
    Exact solution: piecewise constant fields with continuous traction
    sigma.e_x and continuous in-plane strain; solved here as an 11x11
    linear system independent of the oracle's operator.  Layer widths 6
    and 10 have no Nyquist content; 7 and 9 do, which the rotated operator
    and the continuous one applied at Nyquist frequencies control (the
    direction at (m_x, 0, 0) is e_x for every m_x != 0, Nyquist included),
    so the exact solution is their fixed point too."""
    n = 16
    C = rvegen.cubic_stiffness(183000.0, 74500.0, 105000.0)
    eul = np.array([[0.3, 0.9, 0.2], [1.7, 2.1, 0.5]])
    labels = np.zeros((4, 4, n), np.int32)
    labels[..., lo:hi] = 1
    f2 = (hi - lo) / n
    s = _solver(labels, eul, C, _law(), tau0=np.full(12, 1e9), tol=1e-13, green=green, nyquist=nyquist)
    path = rvegen.uniaxial_path(1e-3, 1)
    R = s.run(path, keep_fields=True)
    Cm = [oracle.lab_stiffness(C, oracle.euler_to_rotation(eul[i:i + 1]))[0] for i in range(2)]
    Ct = [np.diag(1 / oracle.MANDEL_W) @ c @ np.diag(oracle.MANDEL_W) for c in Cm]  # tensor comps
    # unknowns: a1, a2 = (e11, e13, e12) of each phase; t = (e22, e33, e23) common; e13m, e12m
    N_ = [0, 4, 5]
    T_ = [1, 2, 3]
    A = np.zeros((11, 11))
    r = np.zeros(11)

    def strain(p):
        M = np.zeros((6, 11))
        for k, i in enumerate(N_):
            M[i, 3 * p + k] = 1
        for k, i in enumerate(T_):
            M[i, 6 + k] = 1
        return M

    S1, S2 = Ct[0] @ strain(0), Ct[1] @ strain(1)
    row = 0
    for i in N_:                                 # traction continuity
        A[row] = S1[i] - S2[i]; row += 1
    for k, i in enumerate(N_):                   # mean of normal components
        A[row, k] = 1 - f2; A[row, 3 + k] = f2
        if i == 0:
            r[row] = 1e-3
        else:
            A[row, 9 + (k - 1)] = -1
        row += 1
    Sm = (1 - f2) * S1 + f2 * S2
    for i in [1, 2, 3, 4, 5]:                    # zero mean stress except 11
        A[row] = Sm[i]; row += 1
    x = np.linalg.solve(A, r)
    sig_exact = Sm @ x
    assert np.allclose(R.Sigma[0], sig_exact, rtol=0, atol=1e-8 * abs(sig_exact[0]))
    e_field = R.fields["strain"]
    e1 = strain(0) @ x
    e2 = strain(1) @ x
    assert np.allclose(e_field[:, 0, 0, 0], e1, atol=1e-13)
    assert np.allclose(e_field[:, 0, 0, lo], e2, atol=1e-13)


def _elastic_polycrystal(n=8, grains=6, seed=7, tol=1e-12):
    rve = rvegen.make_rve(n, grains, seed)
    C = rvegen.cubic_stiffness(183000.0, 74500.0, 105000.0)
    return rve, C, _solver(rve.labels, rve.euler, C, _law(), tau0=np.full(12, 1e9), tol=tol)


def test_voigt_reuss_bounds_and_hill_mandel():
    rve, C, s = _elastic_polycrystal()
    R = s.run(rvegen.uniaxial_path(1e-3, 1), keep_fields=True)
    E_app = R.Sigma[0, 0] / R.E[0, 0]
    Cm = s.mat.C_lab[rve.labels.ravel()]
    C_voigt_avg = Cm.mean(axis=0)
    S_reuss_avg = np.linalg.inv(Cm).mean(axis=0)
    E_upper = 1 / np.linalg.inv(C_voigt_avg)[0, 0]
    E_lower = 1 / S_reuss_avg[0, 0]
    assert E_lower < E_app < E_upper
    sig, eps = R.fields["stress"], R.fields["strain"]
    hm = np.mean(np.sum(oracle.FROB_W[:, None, None, None] * sig * eps, axis=0))
    assert hm == pytest.approx(np.sum(oracle.FROB_W * R.Sigma[0] * R.E[0]), rel=1e-11)
    # the per-step statistics: von Mises of the mean stress and mean of the
    # local von Mises, here from full 3x3 tensors sqrt(3/2 dev:dev)
    def vm(t):
        T = np.array([[t[0], t[5], t[4]], [t[5], t[1], t[3]], [t[4], t[3], t[2]]])
        D = T - np.trace(T) / 3 * np.eye(3)
        return np.sqrt(1.5 * np.sum(D * D))
    assert R.sig_eq_of_mean[0] == pytest.approx(vm(R.Sigma[0]), rel=1e-13)
    local = [vm(sig[:, z, y, x]) for z in range(8) for y in range(8) for x in range(8)]
    assert R.mean_sig_eq[0] == pytest.approx(np.mean(local), rel=1e-13)
    assert R.mean_sig_eq[0] > R.sig_eq_of_mean[0]     # convexity, heterogeneous field


def test_axis_permutation_and_shift_invariance():
    """A cyclic relabelling of the lab axes (a proper rotation) applied to the
    microstructure, the orientations and the load axis permutes the
    response; a periodic shift leaves the mean response unchanged."""
    rve = rvegen.make_rve((6, 8, 10), 5, 11)
    C, law = rvegen.config_law()
    kw = dict(tol=1e-12)
    base = _solver(rve.labels, rve.euler, C, law, **kw)
    path = rvegen.uniaxial_path(0.003, 3)
    R0 = base.run(path)
    assert R0.mean_v[-1] > 0           # plastic by the last step
    # new axes (x', y', z') = old (y, z, x)
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0.0]])
    Qp = P @ rvegen.bunge_to_matrix(rve.euler)
    perm = _solver(np.ascontiguousarray(np.transpose(rve.labels, (2, 0, 1))),
                   rvegen.matrix_to_bunge(Qp), C, law, **kw)
    R1 = perm.run(rvegen.uniaxial_path(0.003, 3, axis=2))
    idx = [2, 0, 1, 5, 3, 4]
    assert np.allclose(R1.Sigma[:, idx], R0.Sigma, rtol=0, atol=1e-9)
    assert np.array_equal(R1.iters, R0.iters)
    shifted = _solver(np.roll(rve.labels, (2, 3, 1), axis=(0, 1, 2)), rve.euler, C, law, **kw)
    R2 = shifted.run(path)
    assert np.allclose(R2.Sigma, R0.Sigma, rtol=0, atol=1e-9)


def test_single_orientation_rve_equals_material_point():
    """A one-orientation RVE has uniform fields: its mean response must equal
    a 0-D material point whose lateral strains make the lateral stresses
    vanish (solved here by Newton on the point law)."""
    C, law = rvegen.config_law()
    eul = np.array([[0.4, 0.8, 1.3]])
    s = _solver(np.zeros((4, 4, 4), np.int32), eul, C, law, tol=1e-12)
    path = rvegen.uniaxial_path(0.004, 4)
    R = s.run(path)
    mat = s.mat
    y = np.zeros((1, mat.state_dim))
    eps = np.zeros(6)
    for n in range(4):
        dt = path.t[n + 1] - path.t[n]
        M = oracle.substeps(dt, 0.05)
        e = eps.copy()
        e[0] = path.target[n, 0]

        def resid(lat):
            ee = e.copy(); ee[1:] = lat
            return mat.update([0], eps, ee, y, dt, M)

        lat = e[1:].copy()
        for _ in range(30):
            y1, sig = resid(lat)
            F = sig[0, 1:]
            if np.abs(F).max() < 1e-10:
                break
            J = np.zeros((5, 5))
            for j in range(5):
                d = np.zeros(5); d[j] = 1e-9
                J[:, j] = (resid(lat + d)[1][0, 1:] - resid(lat - d)[1][0, 1:]) / 2e-9
            lat = lat - np.linalg.solve(J, F)
        e[1:] = lat
        y, eps = y1, e
        assert R.Sigma[n, 0] == pytest.approx(sig[0, 0], rel=1e-8)
        assert np.allclose(oracle.to_mandel(R.E[n]), eps, atol=1e-12)
    assert R.mean_v[-1] > 0
