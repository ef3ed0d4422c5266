"""CPU ORACLE -- test infrastructure only.

A plain, slow, FP64 CPU implementation of what the GPU path computes: the
paper's Green-operator FFT fixed point for a voxelized periodic polycrystal
with the regularized Meric-Cailletaud law (Sections 3 and 4 of the paper).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU
library; the two are fed from the same seeded input generator only.

The local law (``cp_law.c``) is plain C on Mandel 6-vectors; this module
adds the per-label setup (rotations), the Green operator, the fixed-point
iteration with mixed macroscopic conditions, and the per-step outputs.  The
FFT is ``numpy.fft`` (a library primitive serving as one step).

Readings of points the paper leaves open (each is listed with its reason in
the design notes of the repository):

* Green operator: the continuous isotropic Gamma0 of a reference medium
  (lam0, mu0); frequencies xi_j = m_j / N_j with m_j in (-N_j/2, N_j/2];
  Gamma0 = 0 at xi = 0 and at every frequency with a Nyquist component
  (m_j = N_j/2, N_j even), which keeps the real field real.  Option
  nyquist='formula': the formula at every nonzero frequency (Nyquist
  components taken as +N_j/2) and the real part of the inverse transform,
  with those frequencies in the residual.
* Discrete variant (option): the Green operator of the rotated
  finite-difference scheme, the continuous formula at the unit vector of
  s_j = sin(q_j/2) prod_{l != j} cos(q_l/2); zero where s = 0.
* Reference medium: k0 = (1/9) 1:C:1 (Voigt bulk), mu0 = mean of the
  extreme deviatoric shear moduli of C, lam0 = k0 - 2 mu0 / 3.
* Basic scheme: eps^{k+1} = eps^k - Gamma0 * sigma^k + dE^k, with the
  stress-controlled mean strain corrected by the reference compliance.
* Convergence: err_eq = sqrt(sum_xi |sigma_hat(xi) . xi_hat|^2) / |sigma_hat(0)|
  over controlled frequencies, err_bc = |P_S(Sigma - Sigma*)| / |Sigma|.
* Local integration: total strain linear in time within a load step;
  RK4 with M = ceil(dt / h_max) equal substeps.
* Regularization (equation "regu", Section 4): by default the resistance
  is raised by eta times the rate being solved for.  Option reg='lagged':
  by eta times each system's mean slip rate over the previous load step,
  (v_n - v_{n-1}) / dt, with the plain Norton rate in the step (the reading
  under which elastoplastic and purely elastic steps alternate).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import time
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SQ2 = math.sqrt(2.0)
# tensor-component order of every 6-vector at the interfaces: 11,22,33,23,13,12
VOIGT_PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
MANDEL_W = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])
FROB_W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])   # |A|^2 in tensor comps


# ---------------------------------------------------------------------------
# C library
# ---------------------------------------------------------------------------
class _Material(ctypes.Structure):
    _fields_ = [
        ("n_sys", ctypes.c_int), ("n_labels", ctypes.c_int),
        ("C_lab", ctypes.POINTER(ctypes.c_double)),
        ("m_lab", ctypes.POINTER(ctypes.c_double)),
        ("family", ctypes.POINTER(ctypes.c_int)),
        ("tau0", ctypes.POINTER(ctypes.c_double)),
        ("Q", ctypes.c_double * 2), ("b", ctypes.c_double * 2),
        ("c", ctypes.c_double * 2), ("d", ctypes.c_double * 2),
        ("K", ctypes.c_double * 2), ("n", ctypes.c_double * 2),
        ("q_self", ctypes.c_double * 2), ("q_lat", ctypes.c_double * 2),
        ("twin_mode", ctypes.c_int),
        ("K_c", ctypes.c_double), ("f_m", ctypes.c_double),
        ("gamma_T", ctypes.c_double), ("eta", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("CP_ORACLE_LIB") or os.path.join(_HERE, "_cp_law.so")
        if os.environ.get("CP_ORACLE_LIB") and not os.path.exists(path):
            raise FileNotFoundError("CP_ORACLE_LIB names a missing library: " + path)
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_reg_rate.restype = ctypes.c_double
        L.orc_reg_rate.argtypes = [ctypes.c_double] * 5
        L.orc_rate.restype = None
        L.orc_rate.argtypes = [ctypes.POINTER(_Material), ctypes.c_int, dp, dp, dp]
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_cp_probe.restype = ctypes.c_int
        L.orc_cp_probe.argtypes = [ctypes.POINTER(_Material), ctypes.c_long, ip, dp, dp, dp, dp, dp,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, ip]
        L.orc_cp_update_j.restype = ctypes.c_int
        L.orc_cp_update_j.argtypes = [ctypes.POINTER(_Material), ctypes.c_long, ip, dp, dp, dp, dp, dp,
                                      ctypes.c_double, ctypes.c_int, ip]
        L.orc_cp_update_lagged.restype = ctypes.c_int
        L.orc_cp_update_lagged.argtypes = [ctypes.POINTER(_Material), ctypes.c_long,
                                           ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp, dp, dp,
                                           ctypes.c_double, ctypes.c_int]
        L.orc_cp_update.restype = ctypes.c_int
        L.orc_cp_update.argtypes = [ctypes.POINTER(_Material), ctypes.c_long,
                                    ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp, dp,
                                    ctypes.c_double, ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_rate_vjp_point.restype = None
        L.orc_rate_vjp_point.argtypes = [ctypes.POINTER(_Material), ctypes.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_vjp_grid.restype = ctypes.c_int
        L.orc_vjp_grid.argtypes = [ctypes.POINTER(_Material), ctypes.c_long, ctypes.POINTER(ctypes.c_int),
                                   dp, dp, dp, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def threads() -> int:
    return lib().orc_max_threads()


def set_threads(n: int) -> None:
    """Thread count of the C law loops (the FFTs are numpy's, one thread)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------------------
# Tensor bookkeeping
# ---------------------------------------------------------------------------
def to_mandel(t: np.ndarray) -> np.ndarray:
    """tensor components (.., 6) -> Mandel (.., 6)"""
    return np.asarray(t, dtype=np.float64) * MANDEL_W


def from_mandel(m: np.ndarray) -> np.ndarray:
    return np.asarray(m) / MANDEL_W


def sym_to_mat(v: np.ndarray) -> np.ndarray:
    """tensor components (..., 6) -> (..., 3, 3)"""
    out = np.empty(v.shape[:-1] + (3, 3), dtype=v.dtype)
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        out[..., i, j] = v[..., I]
        out[..., j, i] = v[..., I]
    return out


def mat_to_sym(a: np.ndarray) -> np.ndarray:
    return np.stack([a[..., i, j] for (i, j) in VOIGT_PAIRS], axis=-1)


def von_mises(t: np.ndarray) -> np.ndarray:
    """von Mises equivalent of tensor-component 6-vectors: sqrt(3/2 s:s)."""
    t = np.asarray(t, dtype=np.float64)
    p = (t[..., 0] + t[..., 1] + t[..., 2]) / 3.0
    s = t.copy()
    s[..., :3] -= p[..., None]
    return np.sqrt(1.5 * np.sum(FROB_W * s * s, axis=-1))


def frob(t: np.ndarray) -> float:
    return float(np.sqrt(np.sum(FROB_W * np.asarray(t) ** 2)))


# ---------------------------------------------------------------------------
# Per-label setup (orientation, stiffness and Schmid tensors in the lab frame)
# ---------------------------------------------------------------------------
def euler_to_rotation(euler: np.ndarray) -> np.ndarray:
    """Bunge angles (phi1, Phi, phi2) -> Q = Rz(phi1) Rx(Phi) Rz(phi2),
    active, so that v_lab = Q v_crystal."""
    e = np.atleast_2d(np.asarray(euler, dtype=np.float64))

    def rz(a):
        R = np.zeros(a.shape + (3, 3))
        R[..., 0, 0] = np.cos(a); R[..., 0, 1] = -np.sin(a)
        R[..., 1, 0] = np.sin(a); R[..., 1, 1] = np.cos(a)
        R[..., 2, 2] = 1.0
        return R

    def rx(a):
        R = np.zeros(a.shape + (3, 3))
        R[..., 0, 0] = 1.0
        R[..., 1, 1] = np.cos(a); R[..., 1, 2] = -np.sin(a)
        R[..., 2, 1] = np.sin(a); R[..., 2, 2] = np.cos(a)
        return R

    return rz(e[:, 0]) @ rx(e[:, 1]) @ rz(e[:, 2])


def stiffness_tensor(C_voigt: np.ndarray) -> np.ndarray:
    """Voigt 6x6 (engineering shear) -> fourth-order C_ijkl."""
    C4 = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            for (a, b) in {(i, j), (j, i)}:
                for (c, d) in {(k, l), (l, k)}:
                    C4[a, b, c, d] = C_voigt[I, J]
    return C4


def mandel_of_tensor4(C4: np.ndarray) -> np.ndarray:
    M = np.empty(C4.shape[:-4] + (6, 6))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            M[..., I, J] = MANDEL_W[I] * MANDEL_W[J] * C4[..., i, j, k, l]
    return M


def lab_stiffness(C_voigt: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """C'_ijkl = Q_ia Q_jb Q_kc Q_ld C_abcd for each rotation, in Mandel form."""
    C4 = stiffness_tensor(np.asarray(C_voigt, dtype=np.float64))
    C4r = np.einsum("nia,njb,nkc,nld,abcd->nijkl", Q, Q, Q, Q, C4)
    return mandel_of_tensor4(C4r)


def schmid_tensors(n_miller: np.ndarray, l_miller: np.ndarray) -> np.ndarray:
    """Equation 2: m = (n (x) l + l (x) n) / 2 with unit n and l."""
    n = np.asarray(n_miller, dtype=np.float64)
    l = np.asarray(l_miller, dtype=np.float64)
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    l = l / np.linalg.norm(l, axis=1, keepdims=True)
    return 0.5 * (n[:, :, None] * l[:, None, :] + l[:, :, None] * n[:, None, :])


def lab_schmid(m_crys: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """m_lab = Q m Q^T for each label and system, as Mandel vectors [L,S,6]."""
    mr = np.einsum("nia,sab,njb->nsij", Q, m_crys, Q)
    return to_mandel(mat_to_sym(mr))


def reference_medium(C_voigt: np.ndarray) -> tuple[float, float]:
    """Isotropic reference medium (lam0, mu0) of a crystal stiffness.

    k0 = (1/9) 1:C:1; mu0 = (mu_min + mu_max)/2 with 2*mu the extreme
    eigenvalues of C restricted to deviatoric tensors; lam0 = k0 - 2 mu0/3.
    """
    CM = mandel_of_tensor4(stiffness_tensor(np.asarray(C_voigt, dtype=np.float64)))
    one = np.array([1.0, 1, 1, 0, 0, 0])
    k0 = float(one @ CM @ one) / 9.0
    # orthonormal basis of the deviatoric subspace in Mandel space
    P = np.eye(6) - np.outer(one, one) / 3.0
    w, V = np.linalg.eigh(P)
    B = V[:, w > 0.5]                       # 6 x 5
    ev = np.linalg.eigvalsh(B.T @ CM @ B)
    mu0 = 0.25 * (ev[0] + ev[-1])
    return k0 - 2.0 * mu0 / 3.0, mu0


def iso_stiffness(lam: float, mu: float) -> np.ndarray:
    """Isotropic stiffness acting on tensor-component 6-vectors
    (identical to its Mandel matrix)."""
    K = np.zeros((6, 6))
    K[:3, :3] = lam
    for i in range(3):
        K[i, i] = lam + 2 * mu
    for i in range(3, 6):
        K[i, i] = 2 * mu
    return K


def substeps(dt: float, h_max: float) -> int:
    """Number of equal RK4 substeps in a load step of length dt."""
    return max(1, int(math.ceil(dt / h_max * (1.0 - 1e-12))))


# ---------------------------------------------------------------------------
# Material-point law (wraps the C code)
# ---------------------------------------------------------------------------
class Material:
    """Per-label lab-frame data plus law parameters for the C oracle."""

    def __init__(self, euler, C_voigt, n_miller, l_miller, family, tau0, law):
        self.Q = euler_to_rotation(euler)
        self.C_lab = np.ascontiguousarray(lab_stiffness(C_voigt, self.Q))
        self.m_crys = schmid_tensors(n_miller, l_miller)
        self.m_lab = np.ascontiguousarray(lab_schmid(self.m_crys, self.Q))
        self.family = np.ascontiguousarray(np.asarray(family, dtype=np.int32))
        self.tau0 = np.ascontiguousarray(np.asarray(tau0, dtype=np.float64))
        self.n_sys = int(self.family.shape[0])
        self.n_labels = int(self.Q.shape[0])
        self.law = law
        s = _Material()
        s.n_sys, s.n_labels = self.n_sys, self.n_labels
        s.C_lab, s.m_lab = _dp(self.C_lab), _dp(self.m_lab)
        s.family = self.family.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        s.tau0 = _dp(self.tau0)
        for k, fam in enumerate((law.slip, law.twin)):
            for name in ("Q", "b", "c", "d", "K", "n"):
                getattr(s, name)[k] = float(getattr(fam, name))
            s.q_self[k] = float(fam.q_self)
            s.q_lat[k] = float(fam.q_latent)
        s.twin_mode = int(law.twin_mode)
        s.K_c, s.f_m, s.gamma_T = float(law.K_c), float(law.f_m), float(law.gamma_T)
        s.eta = float(law.eta)
        self._s = s

    @property
    def state_dim(self) -> int:
        return 6 + 2 * self.n_sys

    def rate(self, label: int, eps_mandel, y) -> np.ndarray:
        e = np.ascontiguousarray(eps_mandel, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        dy = np.zeros(self.state_dim)
        lib().orc_rate(ctypes.byref(self._s), int(label), _dp(e), _dp(y), _dp(dy))
        return dy

    def update(self, labels, eps0, eps1, y0, dt, M):
        """Integrate every point over one load increment (Mandel in/out)."""
        labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).ravel())
        n = labels.shape[0]
        eps0 = np.ascontiguousarray(np.broadcast_to(eps0, (n, 6)), dtype=np.float64)
        eps1 = np.ascontiguousarray(np.broadcast_to(eps1, (n, 6)), dtype=np.float64)
        y0 = np.ascontiguousarray(y0, dtype=np.float64)
        y1 = np.empty_like(y0)
        sig = np.empty((n, 6))
        rc = lib().orc_cp_update(ctypes.byref(self._s), n,
                                 labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 _dp(eps0), _dp(eps1), _dp(y0), _dp(y1), _dp(sig),
                                 float(dt), int(M))
        if rc != 0:
            raise ValueError("orc_cp_update rejected its input")
        return y1, sig


    def update_lagged(self, labels, eps0, eps1, y0, dr, dt, M):
        """update() with the lagged regularization: dr [n][S] = eta |gdot| of
        the previous load step raises each system's resistance, and the
        rate is the plain Norton law."""
        labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).ravel())
        n = labels.shape[0]
        eps0 = np.ascontiguousarray(np.broadcast_to(eps0, (n, 6)), dtype=np.float64)
        eps1 = np.ascontiguousarray(np.broadcast_to(eps1, (n, 6)), dtype=np.float64)
        y0 = np.ascontiguousarray(y0, dtype=np.float64)
        dr = np.ascontiguousarray(np.broadcast_to(dr, (n, self.n_sys)), dtype=np.float64)
        y1 = np.empty_like(y0)
        sig = np.empty((n, 6))
        rc = lib().orc_cp_update_lagged(ctypes.byref(self._s), n,
                                        labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                        _dp(eps0), _dp(eps1), _dp(y0), _dp(dr), _dp(y1), _dp(sig),
                                        float(dt), int(M))
        if rc != 0:
            raise ValueError("orc_cp_update_lagged rejected its input")
        return y1, sig

    def _prep(self, labels, eps0, eps1, y0):
        labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).ravel())
        n = labels.shape[0]
        eps0 = np.ascontiguousarray(np.broadcast_to(eps0, (n, 6)), dtype=np.float64)
        eps1 = np.ascontiguousarray(np.broadcast_to(eps1, (n, 6)), dtype=np.float64)
        y0 = np.ascontiguousarray(y0, dtype=np.float64)
        return labels, n, eps0, eps1, y0

    def probe(self, labels, eps0, eps1, y0, dt, M, tol, maxd):
        """Frozen error-controlled substeps (orc_cp_probe): per point the
        least M 2^j whose result agrees with twice the count; returns
        (y1, sig, j)."""
        labels, n, eps0, eps1, y0 = self._prep(labels, eps0, eps1, y0)
        y1 = np.empty_like(y0)
        sig = np.empty((n, 6))
        j = np.zeros(n, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        rc = lib().orc_cp_probe(ctypes.byref(self._s), n, labels.ctypes.data_as(ip), _dp(eps0), _dp(eps1),
                                _dp(y0), _dp(y1), _dp(sig), float(dt), int(M), float(tol), int(maxd),
                                j.ctypes.data_as(ip))
        if rc != 0:
            raise ValueError("orc_cp_probe rejected its input")
        return y1, sig, j

    def update_j(self, labels, eps0, eps1, y0, dt, M, j):
        """``update`` with per-point substep counts M 2^j."""
        labels, n, eps0, eps1, y0 = self._prep(labels, eps0, eps1, y0)
        y1 = np.empty_like(y0)
        sig = np.empty((n, 6))
        j = np.ascontiguousarray(j, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        rc = lib().orc_cp_update_j(ctypes.byref(self._s), n, labels.ctypes.data_as(ip), _dp(eps0), _dp(eps1),
                                   _dp(y0), _dp(y1), _dp(sig), float(dt), int(M), j.ctypes.data_as(ip))
        if rc != 0:
            raise ValueError("orc_cp_update_j rejected its input")
        return y1, sig

    # -- reverse mode -------------------------------------------------------
    def rate_vjp(self, label: int, eps_mandel, y, kbar):
        """Cotangents (y_bar, eps_bar, theta_bar[2][7]) of dy/dt = F(eps, y)
        for the cotangent kbar of its output; theta = (r0, Q, b, c, d, K, n)
        per family (slip, twin)."""
        e = np.ascontiguousarray(eps_mandel, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        kb = np.ascontiguousarray(kbar, dtype=np.float64)
        yb = np.zeros(self.state_dim)
        eb = np.zeros(6)
        th = np.zeros(14)
        lib().orc_rate_vjp_point(ctypes.byref(self._s), int(label), _dp(e), _dp(y), _dp(kb),
                                 _dp(yb), _dp(eb), _dp(th))
        return yb, eb, th.reshape(2, 7)

    def update_vjp(self, labels, eps0, eps1, y0, dt, M, sig_bar, y_bar):
        """Reverse of :meth:`update`: cotangents of eps0, eps1, y0 (per
        point, Mandel) and of theta (summed) for cotangents of the end stress
        and end state."""
        labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).ravel())
        n = labels.shape[0]
        D = self.state_dim
        a = [np.ascontiguousarray(np.broadcast_to(x, (n, k)), dtype=np.float64)
             for x, k in ((eps0, 6), (eps1, 6), (y0, D), (sig_bar, 6), (y_bar, D))]
        e0b, e1b, y0b, th = np.empty((n, 6)), np.empty((n, 6)), np.empty((n, D)), np.empty(14)
        rc = lib().orc_vjp_grid(ctypes.byref(self._s), n,
                                labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                _dp(a[0]), _dp(a[1]), _dp(a[2]), float(dt), int(M), _dp(a[3]),
                                _dp(a[4]), _dp(e0b), _dp(e1b), _dp(y0b), _dp(th))
        if rc != 0:
            raise ValueError("orc_vjp_grid rejected its input")
        return e0b, e1b, y0b, th.reshape(2, 7)


THETA_NAMES = ("r0", "Q", "b", "c", "d", "K", "n")


def reg_rate(o, A, K, n, eta) -> float:
    return lib().orc_reg_rate(float(o), float(A), float(K), float(n), float(eta))


# ---------------------------------------------------------------------------
# Green operator (continuous, isotropic reference medium)
# ---------------------------------------------------------------------------
def von_mises_sq(stress: np.ndarray) -> np.ndarray:
    """Square of the local von Mises stress 3/2 dev(s):dev(s) of stresses
    [6][...] in tensor components (Section 5's sigma_eq, squared), FP64,
    in a fixed order of single IEEE operations: m = ((s11 + s22) + s33) / 3,
    d_i = s_ii - m, 1.5 (((d1 d1 + d2 d2) + d3 d3) + 2 ((s23 s23 + s13 s13)
    + s12 s12))."""
    s = [np.asarray(stress[c], dtype=np.float64) for c in range(6)]
    m = ((s[0] + s[1]) + s[2]) / 3.0
    d1, d2, d3 = s[0] - m, s[1] - m, s[2] - m
    nrm = (d1 * d1 + d2 * d2) + d3 * d3
    sh = (s[3] * s[3] + s[4] * s[4]) + s[5] * s[5]
    return 1.5 * (nrm + 2.0 * sh)


def von_mises_field(stress: np.ndarray) -> np.ndarray:
    """Local von Mises stress sqrt(von_mises_sq) of stresses [6][...]."""
    return np.sqrt(von_mises_sq(stress))


def von_mises_histogram(stress_fields, nbins: int, lo: float, hi: float) -> np.ndarray:
    """Counts [nbins + 2] of the von Mises stress over the voxels of all
    given stress fields ([6][...] each) for the bin edges e_k = lo + k w,
    w = (hi - lo) / nbins: below e_0, in [e_k, e_k+1) for k < nbins, and the
    rest (at or above e_nbins, or not finite).  Decided on squares: the
    largest k with e_k^2 <= sigma_eq^2 (edges <= 0 below every value)."""
    w = (float(hi) - float(lo)) / nbins
    e = float(lo) + np.arange(nbins + 1, dtype=np.float64) * w
    q = np.where(e > 0.0, e * e, -1.0)
    counts = np.zeros(nbins + 2, dtype=np.uint64)
    for f in stress_fields:
        x = von_mises_sq(np.asarray(f).reshape(6, -1))
        bad = ~np.isfinite(x)
        j = np.searchsorted(q, x[~bad], side="right") - 1       # largest j with q[j] <= x
        counts += np.bincount(j + 1, minlength=nbins + 2).astype(np.uint64)
        counts[nbins + 1] += np.uint64(np.count_nonzero(bad))
    return counts


def frequency_directions(shape, nyquist: str = "zero"):
    """Unit frequency directions xi_hat [3,nz,ny,nx] (x,y,z order) of the
    frequencies m_j in (-N_j/2, N_j/2] and the mask of controlled
    frequencies: not zero and, with nyquist='zero', no Nyquist component
    (m_j = N_j/2); with nyquist='formula' every nonzero frequency (the
    Nyquist components taken as +N_j/2)."""
    if nyquist not in ("zero", "formula"):
        raise ValueError("nyquist must be 'zero' or 'formula'")
    nz, ny, nx = shape
    ms, nyq = [], []
    for N in (nx, ny, nz):
        k = np.arange(N)
        m = np.where(k <= N // 2, k, k - N).astype(np.float64)
        ms.append(m / N)
        nyq.append((N % 2 == 0) & (k == N // 2))
    MZ, MY, MX = np.meshgrid(ms[2], ms[1], ms[0], indexing="ij")
    NZ, NY, NX = np.meshgrid(nyq[2], nyq[1], nyq[0], indexing="ij")
    xi = np.stack([MX, MY, MZ])
    nrm = np.sqrt(np.sum(xi * xi, axis=0))
    ctrl = (nrm > 0) & ~(NX | NY | NZ) if nyquist == "zero" else nrm > 0
    xi_hat = np.where(ctrl, xi / np.where(nrm > 0, nrm, 1.0), 0.0)
    return xi_hat, ctrl


def frequency_directions_rotated(shape):
    """Directions of the rotated finite-difference scheme (Willot, 2015),
    the discrete variant of the Green operator: [3,nz,ny,nx] and the mask
    of controlled frequencies.

    In that scheme the derivative along j at a voxel centre is the mean of
    the four differences along the voxel edges parallel to j.  Its Fourier
    symbol is 2i exp(i (q1+q2+q3)/2) s_j with q_j = 2 pi m_j / N_j and
      s_j = sin(q_j / 2) prod_{l != j} cos(q_l / 2).
    The common complex factor cancels in Gamma0, which is therefore the
    continuous formula evaluated at the real unit vector s / |s|.  s = 0 at
    the zero frequency and wherever two or more components are at Nyquist
    (cos(pi/2) = 0, set exactly); there Gamma0 is zero and those
    frequencies are not controlled.  A single Nyquist component is
    controlled (unlike the continuous operator)."""
    nz, ny, nx = shape
    sin_h, cos_h = [], []
    for N in (nx, ny, nz):
        k = np.arange(N)
        m = np.where(k <= N // 2, k, k - N).astype(np.float64)
        half = np.pi * m / N                       # q / 2
        nyq = 2 * m == N
        sin_h.append(np.where(nyq, 1.0, np.sin(half)))
        cos_h.append(np.where(nyq, 0.0, np.cos(half)))
    Sx, Sy, Sz = np.meshgrid(sin_h[2], sin_h[1], sin_h[0], indexing="ij")[::-1]
    Cx, Cy, Cz = np.meshgrid(cos_h[2], cos_h[1], cos_h[0], indexing="ij")[::-1]
    s = np.stack([Sx * Cy * Cz, Sy * Cx * Cz, Sz * Cx * Cy])
    nrm = np.sqrt(np.sum(s * s, axis=0))
    ctrl = nrm > 0
    return np.where(ctrl, s / np.where(ctrl, nrm, 1.0), 0.0), ctrl


def green_directions(shape, green: str = "continuous", nyquist: str = "zero"):
    """Unit directions and controlled-frequency mask of the chosen Green
    operator: 'continuous' (the default; nyquist as in
    frequency_directions) or 'rotated'."""
    if green == "continuous":
        return frequency_directions(shape, nyquist)
    if green == "rotated":
        if nyquist != "zero":
            raise ValueError("nyquist='formula' applies to the continuous operator only")
        return frequency_directions_rotated(shape)
    raise ValueError("green must be 'continuous' or 'rotated'")


def gamma0_apply(tau_hat: np.ndarray, lam0: float, mu0: float,
                 xi_hat: Optional[np.ndarray] = None,
                 ctrl: Optional[np.ndarray] = None) -> np.ndarray:
    """eps_hat = Gamma0(xi) : tau_hat(xi) on a full spectrum.

    tau_hat: [6,nz,ny,nx] tensor components.  With a = tau_hat . xi_hat and
    b = xi_hat . tau_hat . xi_hat,
      eps_hat_ij = (xi_i a_j + xi_j a_i) / (2 mu0)
                   - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) * b * xi_i xi_j ,
    and eps_hat = 0 at uncontrolled frequencies.
    """
    if xi_hat is None:
        xi_hat, ctrl = frequency_directions(tau_hat.shape[1:])
    T = sym_to_mat(np.moveaxis(tau_hat, 0, -1))          # [...,3,3]
    x = np.moveaxis(xi_hat, 0, -1)                        # [...,3]
    a = np.einsum("...ij,...j->...i", T, x)
    b = np.einsum("...i,...i->...", x, a)
    coef = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0))
    E = (x[..., :, None] * a[..., None, :] + a[..., :, None] * x[..., None, :]) / (2.0 * mu0) \
        - coef * b[..., None, None] * x[..., :, None] * x[..., None, :]
    E = np.where(ctrl[..., None, None], E, 0.0)
    return np.moveaxis(mat_to_sym(E), -1, 0)


def fft3(field: np.ndarray) -> np.ndarray:
    """Unnormalized forward DFT over the last three axes (z, y, x)."""
    return np.fft.fftn(field, axes=(-3, -2, -1))


def ifft3_real(spec: np.ndarray) -> np.ndarray:
    """Inverse DFT (normalized by 1/N) over the last three axes, real part."""
    return np.fft.ifftn(spec, axes=(-3, -2, -1)).real


def equilibrium_sums(sig_hat: np.ndarray, xi_hat, ctrl) -> float:
    """sum over controlled frequencies of |sigma_hat(xi) . xi_hat|^2."""
    T = sym_to_mat(np.moveaxis(sig_hat, 0, -1))
    x = np.moveaxis(xi_hat, 0, -1)
    a = np.einsum("...ij,...j->...i", T, x)
    return float(np.sum(np.where(ctrl, np.sum(np.abs(a) ** 2, axis=-1), 0.0)))


# ---------------------------------------------------------------------------
# The fixed-point solver
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Options:
    tol: float = 1e-8
    max_iter: int = 1000
    h_max: float = 0.05
    M: Optional[int] = None           # fixed RK4 substeps, overrides h_max
    lam0: Optional[float] = None      # reference medium override
    mu0: Optional[float] = None
    green: str = "continuous"         # or "rotated" (discrete Green operator)
    rk_tol: float = 0.0               # > 0: frozen error-controlled substep counts per load step
    rk_max_doublings: int = 4
    aa_depth: int = 0                 # > 0: Anderson-accelerated fixed point of that depth
    nyquist: str = "zero"             # continuous operator at Nyquist frequencies: 'zero' or 'formula'
    cutback: int = 0                  # > 0: a failed load step is retried as two half steps, recursively
    reg: str = "implicit"             # 'implicit' (equation "regu" with the rate itself) or 'lagged'


class NotConverged(RuntimeError):
    pass


@dataclasses.dataclass
class Result:
    Sigma: np.ndarray          # [n_steps][6] tensor components, MPa
    E: np.ndarray              # [n_steps][6]
    sig_eq_of_mean: np.ndarray  # von Mises of Sigma
    mean_sig_eq: np.ndarray    # mean of local von Mises
    mean_v: np.ndarray         # mean accumulated slip over slip systems
    mean_f: np.ndarray         # mean twin fraction over twin systems
    iters: np.ndarray          # constitutive evaluations per step
    err_eq: np.ndarray
    err_bc: np.ndarray
    wall: float = 0.0
    fields: Optional[dict] = None
    n_symptom: Optional[np.ndarray] = None   # local-stress test count per step (Solver.symptom_count)
    cutbacks: Optional[np.ndarray] = None    # failed attempts retried as half steps


class Solver:
    """Plain FP64 Green-operator fixed point over mixed load steps."""

    def __init__(self, labels, euler, C_voigt, n_miller, l_miller, family,
                 tau0, law, options: Optional[Options] = None):
        self.labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
        self.shape = self.labels.shape
        self.n_vox = int(self.labels.size)
        self.mat = Material(euler, C_voigt, n_miller, l_miller, family, tau0, law)
        self.opts = options or Options()
        lam0, mu0 = reference_medium(C_voigt)
        if self.opts.mu0 is not None:
            lam0, mu0 = self.opts.lam0, self.opts.mu0
        self.lam0, self.mu0 = lam0, mu0
        self.K0 = iso_stiffness(lam0, mu0)
        self.xi_hat, self.ctrl = green_directions(self.shape, self.opts.green, self.opts.nyquist)
        if self.opts.reg not in ("implicit", "lagged"):
            raise ValueError("reg must be 'implicit' or 'lagged'")
        if self.opts.reg == "lagged" and (self.opts.rk_tol > 0 or self.opts.aa_depth > 0):
            raise ValueError("the lagged regularization runs the basic fixed point with fixed substeps")
        self.slip = self.mat.family == 0
        self.twin = self.mat.family == 1
        self.reset()

    def reset(self):
        n, D = self.n_vox, self.mat.state_dim
        self.eps = np.zeros((n, 6))          # Mandel, committed total strain
        self.y = np.zeros((n, D))            # committed internal variables
        self.Sigma = np.zeros(6)             # committed mean stress (tensor)
        self.E = np.zeros(6)                 # committed mean strain (tensor)
        self.sig = np.zeros((n, 6))          # committed stress (Mandel)
        # lagged regularization: eta |gdot| of the previous load step per
        # point and system (zero before the first step)
        self.dr = np.zeros((n, self.mat.n_sys))

    # -- pieces ------------------------------------------------------------
    def errors(self, sig_t: np.ndarray, Sigma: np.ndarray, sidx, target):
        grid = np.moveaxis(sig_t.reshape(self.shape + (6,)), -1, 0)
        sig_hat = fft3(grid)
        num = math.sqrt(equilibrium_sums(sig_hat, self.xi_hat, self.ctrl))
        den = self.n_vox * frob(Sigma)
        err_eq = num / den if den > 0 else (0.0 if num == 0 else math.inf)
        dS = np.where(sidx, Sigma - target, 0.0)
        sn = frob(Sigma)
        err_bc = frob(dS) / sn if sn > 0 else (0.0 if frob(dS) == 0 else math.inf)
        return sig_hat, err_eq, err_bc

    def correction(self, sig_hat: np.ndarray) -> np.ndarray:
        """Gamma0 * sigma in real space, tensor components [n_vox][6]."""
        eh = gamma0_apply(sig_hat, self.lam0, self.mu0, self.xi_hat, self.ctrl)
        corr = ifft3_real(eh)
        return np.moveaxis(corr, 0, -1).reshape(self.n_vox, 6)

    @staticmethod
    def _anderson(hist, x, f, E, dE, m):
        """One Anderson-accelerated update of the fixed point x <- x + f
        (f = -Gamma0 * sigma + dE, the basic scheme's step), depth m (Walker
        and Ni, 2011): with the differences dX_i = x_{i+1} - x_i and
        dF_i = f_{i+1} - f_i of the last (up to) m iterations, gamma solves
        (G + lam I) gamma = dF^T f, G = dF^T dF (Euclidean products of the
        Mandel fields, lam = 1e-14 trace(G) / m_k), and
        x_new = x + f - sum_i gamma_i (dX_i + dF_i); the mean strain E is
        mixed with the same coefficients (its steps are the mean parts
        dE).  A system that is not positive definite (no Cholesky factor)
        takes the basic step."""
        hist.append((x.copy(), f.copy(), E.copy(), dE.copy()))
        if len(hist) > m + 1:
            hist.pop(0)
        mk = len(hist) - 1
        if mk == 0:
            return x + f, E + dE
        dF = np.stack([(hist[i + 1][1] - hist[i][1]).ravel() for i in range(mk)], axis=1)
        dX = np.stack([(hist[i + 1][0] - hist[i][0]).ravel() for i in range(mk)], axis=1)
        G = dF.T @ dF
        tr = np.trace(G)
        if not tr > 0:
            return x + f, E + dE               # degenerate history: the basic step
        lam = 1e-14 * tr / mk
        try:
            L = np.linalg.cholesky(G + lam * np.eye(mk))
        except np.linalg.LinAlgError:
            return x + f, E + dE
        gam = np.linalg.solve(L.T, np.linalg.solve(L, dF.T @ f.ravel()))
        x_new = x.ravel() + f.ravel() - (dX + dF) @ gam
        dEX = np.stack([hist[i + 1][2] - hist[i][2] for i in range(mk)], axis=1)
        ddE = np.stack([hist[i + 1][3] - hist[i][3] for i in range(mk)], axis=1)
        E_new = E + dE - (dEX + ddE) @ gam
        return x_new.reshape(x.shape), E_new

    def _stress_correction(self, sidx, rhs) -> np.ndarray:
        dE = np.zeros(6)
        S = np.nonzero(sidx)[0]
        if S.size:
            dE[S] = np.linalg.solve(self.K0[np.ix_(S, S)], rhs[S])
        return dE

    # -- one load step -----------------------------------------------------
    def step(self, t0: float, t1: float, ctrl_row, target_row):
        o = self.opts
        dt = t1 - t0
        M = o.M if o.M is not None else substeps(dt, o.h_max)
        eidx = np.asarray(ctrl_row, dtype=bool)
        sidx = ~eidx
        target = np.asarray(target_row, dtype=np.float64)
        # initial guess: homogeneous reference-medium prediction
        dE = np.zeros(6)
        dE[eidx] = target[eidx] - self.E[eidx]
        rhs = (target - self.Sigma) - self.K0 @ dE
        dE += self._stress_correction(sidx, rhs)
        E = self.E + dE
        eps = self.eps + to_mandel(dE)
        hist = []                            # Anderson: (x, f, E, dE) of earlier iterations
        for k in range(o.max_iter):
            if o.rk_tol > 0 and k == 0:
                y1, sig, self.substep_j = self.mat.probe(self.labels, self.eps, eps, self.y, dt, M,
                                                         o.rk_tol, o.rk_max_doublings)
            elif o.rk_tol > 0:
                y1, sig = self.mat.update_j(self.labels, self.eps, eps, self.y, dt, M, self.substep_j)
            elif o.reg == "lagged":
                y1, sig = self.mat.update_lagged(self.labels, self.eps, eps, self.y, self.dr, dt, M)
            else:
                y1, sig = self.mat.update(self.labels, self.eps, eps, self.y, dt, M)
            sig_t = from_mandel(sig)
            Sigma = sig_t.mean(axis=0)
            sig_hat, err_eq, err_bc = self.errors(sig_t, Sigma, sidx, target)
            if not (np.isfinite(err_eq) and np.isfinite(err_bc)):
                raise FloatingPointError("non-finite residual at iteration %d" % k)
            if err_eq <= o.tol and err_bc <= o.tol:
                break
            corr = self.correction(sig_hat)
            dE = self._stress_correction(sidx, target - Sigma)
            if o.aa_depth > 0:
                eps, E = self._anderson(hist, eps, -to_mandel(corr) + to_mandel(dE), E, dE, o.aa_depth)
            else:
                E = E + dE
                eps = eps - to_mandel(corr) + to_mandel(dE)
        else:
            raise NotConverged("no convergence in %d iterations" % o.max_iter)
        self.last_symptom = self.symptom_count(sig, E)
        self.last_errors = (err_eq, err_bc)
        if o.reg == "lagged":
            # the step's mean slip rates |gdot| = (v_{n+1} - v_n) / dt
            S = self.mat.n_sys
            self.dr = self.mat.law.eta * (y1[:, 6:6 + S] - self.y[:, 6:6 + S]) / dt
        self.eps, self.y, self.sig = eps, y1, sig
        self.Sigma, self.E = Sigma, E
        return k + 1, err_eq, err_bc

    def symptom_count(self, sig_new: np.ndarray, E_new: np.ndarray) -> int:
        """Voxels whose stress moved by more than E0 |dE| over the load step
        (Section 4's condition under which the basic scheme stops enforcing
        equilibrium locally): |sigma_{n+1} - sigma_n|_F > E0 |E_{n+1} - E_n|_F,
        Frobenius norms (Mandel vectors carry them as Euclidean norms), E0
        the Young's modulus of the reference medium; squares compared."""
        lam0, mu0 = self.lam0, self.mu0
        E0 = mu0 * (3.0 * lam0 + 2.0 * mu0) / (lam0 + mu0)
        dE = np.asarray(E_new) - self.E
        thr2 = E0 * E0 * float(np.sum(FROB_W * dE * dE))
        d = sig_new - self.sig
        return int(np.count_nonzero(np.sum(d * d, axis=1) > thr2))

    def step_cut(self, t0: float, t1: float, ctrl_row, target_row, depth: int):
        """One load step, retried as two half steps when it does not converge
        (or its residual is not finite) and halvings are left; the half
        step's targets are the midpoints between the committed mean strain
        (strain-controlled components) or mean stress (stress-controlled ones)
        and the step's targets.  Returns (iterations of the completed
        sub-steps, failed attempts, local-stress counts summed)."""
        try:
            its, _, _ = self.step(t0, t1, ctrl_row, target_row)
            return its, 0, self.last_symptom
        except (NotConverged, FloatingPointError):
            if depth <= 0:
                raise
        ctrl = np.asarray(ctrl_row, dtype=bool)
        target = np.asarray(target_row, dtype=np.float64)
        mid = 0.5 * (np.where(ctrl, self.E, self.Sigma) + target)
        i0, c0, s0 = self.step_cut(t0, 0.5 * (t0 + t1), ctrl_row, mid, depth - 1)
        i1, c1, s1 = self.step_cut(0.5 * (t0 + t1), t1, ctrl_row, target, depth - 1)
        return i0 + i1, c0 + c1 + 1, s0 + s1

    def outputs(self):
        S = self.mat.n_sys
        v = self.y[:, 6:6 + S]
        sig_t = from_mandel(self.sig)
        mv = float(v[:, self.slip].mean()) if self.slip.any() else 0.0
        mf = float(v[:, self.twin].mean() / self.mat.law.gamma_T) if self.twin.any() else 0.0
        return (float(von_mises(self.Sigma)), float(von_mises(sig_t).mean()), mv, mf)

    def run(self, path, keep_fields: bool = False, n_steps: Optional[int] = None) -> Result:
        ns = path.target.shape[0] if n_steps is None else n_steps
        R = Result(*(np.zeros((ns, 6)) for _ in range(2)),
                   *(np.zeros(ns) for _ in range(4)),
                   np.zeros(ns, dtype=np.int64), np.zeros(ns), np.zeros(ns))
        R.n_symptom = np.zeros(ns, dtype=np.int64)
        R.cutbacks = np.zeros(ns, dtype=np.int64)
        t_start = time.perf_counter()
        for n in range(ns):
            if self.opts.cutback > 0:
                its, R.cutbacks[n], R.n_symptom[n] = self.step_cut(
                    path.t[n], path.t[n + 1], path.strain_ctrl[n], path.target[n], self.opts.cutback)
                ee, eb = self.last_errors
            else:
                its, ee, eb = self.step(path.t[n], path.t[n + 1], path.strain_ctrl[n],
                                        path.target[n])
                R.n_symptom[n] = self.last_symptom
            R.Sigma[n], R.E[n] = self.Sigma, self.E
            (R.sig_eq_of_mean[n], R.mean_sig_eq[n], R.mean_v[n],
             R.mean_f[n]) = self.outputs()
            R.iters[n], R.err_eq[n], R.err_bc[n] = its, ee, eb
        R.wall = time.perf_counter() - t_start
        if keep_fields:
            R.fields = self.fields()
        return R

    # -- discrete adjoint -------------------------------------------------------
    def gradient(self, path, target_xx, adj_tol: float = 1e-12, n_steps: Optional[int] = None):
        """Loss L = sum_n (Sigma_xx,n - target_xx[n])^2 over the load steps and
        its gradient with respect to theta[f] = (r0, Q, b, c, d, K, n) of the
        slip (f = 0) and twin (f = 1) families: the adjoint below with the
        cotangent dL/dSigma_n = 2 (Sigma_xx,n - target_n) e_xx."""
        tgt = np.asarray(target_xx, dtype=np.float64)

        def cot(Sig):
            sb = np.zeros_like(Sig)
            sb[:, 0] = 2.0 * (Sig[:, 0] - tgt[:Sig.shape[0]])
            return sb

        grad, Sig = self._adjoint(path, cot, adj_tol, n_steps)
        L = float(np.sum((Sig[:, 0] - tgt[:Sig.shape[0]]) ** 2))
        return L, grad, Sig[:, 0]

    def vjp(self, path, sigma_bar, adj_tol: float = 1e-12, n_steps: Optional[int] = None):
        """Vector-Jacobian product of the effective stress history: for a
        cotangent sigma_bar[n][6] = dJ/dSigma_n (tensor components), the
        gradient dJ/dtheta [2][7] of J = sum_n sigma_bar_n . Sigma_n, and the
        history Sigma[n][6]."""
        sb = np.asarray(sigma_bar, dtype=np.float64)
        return self._adjoint(path, lambda Sig: sb[:Sig.shape[0]], adj_tol, n_steps)

    def _adjoint(self, path, cotangent, adj_tol, n_steps):
        """Discrete adjoint of the converged load steps.

        Forward: the converged steps, recording (eps_n, y_n, eps_n+1); then
        the cotangent Sigma_bar_n of every step's mean stress.
        Reverse, per step n (last to first), with the cotangents S_bar,
        eps_bar carried from step n+1:
          g  = d/d eps_{n+1} of [sigma_bar_L . sigma + S_bar . S] + eps_bar,
               sigma_bar_L = Sigma_bar_n / N at every voxel (Mandel
               components: divided by the Mandel weights);
          A  = d sigma_{n+1} / d eps_{n+1} per voxel (six reverse sweeps);
          mu in the admissible strain space (compatible, zero mean, free
               mean on stress-controlled components) with A^T mu - g weakly
               equilibrated -- the same Green-operator fixed point as the
               forward problem, tangent transposed, target mean stress 0;
          then one reverse sweep of the local law with cotangents
          (sigma_bar_L - mu, S_bar) gives S_bar_n, eps_bar_n and theta_bar.
        """
        if self.opts.reg != "implicit":
            raise ValueError("the discrete adjoint differentiates the implicit regularization only")
        ns = path.target.shape[0] if n_steps is None else n_steps
        self.reset()
        rec = []
        Sig = np.zeros((ns, 6))
        for n in range(ns):
            e0, y0 = self.eps.copy(), self.y.copy()
            self.step(path.t[n], path.t[n + 1], path.strain_ctrl[n], path.target[n])
            dt = path.t[n + 1] - path.t[n]
            M = self.opts.M if self.opts.M is not None else substeps(dt, self.opts.h_max)
            rec.append((e0, y0, self.eps.copy(), dt, M, np.asarray(path.strain_ctrl[n], bool)))
            Sig[n] = self.Sigma
        Sbar = np.asarray(cotangent(Sig), dtype=np.float64).reshape(ns, 6)
        N = self.n_vox
        D = self.mat.state_dim
        Sb = np.zeros((N, D))
        eb = np.zeros((N, 6))
        grad = np.zeros((2, 7))
        lab = self.labels.ravel()
        eye = np.eye(6)
        self.adj_iters = []
        for n in range(ns - 1, -1, -1):
            e0, y0, e1, dt, M, ectrl = rec[n]
            sigL = np.broadcast_to(Sbar[n] / (N * MANDEL_W), (N, 6)).copy()
            _, g, _, _ = self.mat.update_vjp(lab, e0, e1, y0, dt, M, sigL, Sb)
            g = g + eb
            Arows = np.empty((N, 6, 6))
            zero = np.zeros((N, D))
            for i in range(6):
                _, Arows[:, i, :], _, _ = self.mat.update_vjp(lab, e0, e1, y0, dt, M,
                                                              np.broadcast_to(eye[i], (N, 6)), zero)
            mu = self._adjoint_equilibrium(Arows, g, ~ectrl, adj_tol)
            e0b, _, y0b, th = self.mat.update_vjp(lab, e0, e1, y0, dt, M, sigL - mu, Sb)
            grad += th
            Sb, eb = y0b, e0b
        self.reset()
        return grad, Sig

    def _adjoint_equilibrium(self, Arows, g, sidx, tol):
        """mu (Mandel, per voxel) with A^T mu - g weakly equilibrated, by the
        basic scheme with Gamma0."""
        N = self.n_vox
        gn = math.sqrt(float(np.sum(g * g)))
        mu = np.zeros((N, 6))
        if gn == 0.0:
            self.adj_iters.append(0)
            return mu
        grms = gn / math.sqrt(N)
        for k in range(self.opts.max_iter):
            tau = np.einsum("ni,nij->nj", mu, Arows) - g
            tau_t = from_mandel(tau)
            T = tau_t.mean(axis=0)
            grid = np.moveaxis(tau_t.reshape(self.shape + (6,)), -1, 0)
            th = fft3(grid)
            err_eq = math.sqrt(equilibrium_sums(th, self.xi_hat, self.ctrl)) / (math.sqrt(N) * gn)
            err_bc = frob(np.where(sidx, T, 0.0)) / grms
            if err_eq <= tol and err_bc <= tol:
                self.adj_iters.append(k + 1)
                return mu
            corr = self.correction(th)
            dM = self._stress_correction(sidx, -T)
            mu = mu - to_mandel(corr) + to_mandel(dM)
        raise NotConverged("adjoint equilibrium: no convergence in %d iterations" % self.opts.max_iter)

    def fields(self) -> dict:
        """Committed local fields, tensor components, grid-shaped [6][nz][ny][nx]."""
        S = self.mat.n_sys

        def grid(a):
            return np.moveaxis(a.reshape(self.shape + (a.shape[-1],)), -1, 0)

        return {
            "stress": grid(from_mandel(self.sig)),
            "strain": grid(from_mandel(self.eps)),
            "plastic_strain": grid(from_mandel(self.y[:, :6])),
            "acc_slip": grid(self.y[:, 6:6 + S]),
            "back_strain": grid(self.y[:, 6 + S:]),
        }


def solver_for(workload, options: Optional[Options] = None) -> Solver:
    """Convenience: an oracle solver for an ``rvegen.Workload``-like object."""
    w = workload
    return Solver(w.rve.labels, w.rve.euler, w.C, w.systems.n_miller,
                  w.systems.l_miller, w.systems.family, w.systems.tau0, w.law,
                  options)
