"""Seeded synthetic inputs for the FFT crystal-plasticity solver.

This module only *generates inputs*: voxel label grids, per-label Bunge
Euler angles, the slip/twin system table, law parameter sets and
macroscopic loading paths.  It contains none of the solver's arithmetic
(no constitutive law, no Green operator, no FFT), so that both the CPU
oracle and the GPU path can be fed from it without sharing code.

Microstructures stand in for the paper's stochastic RVEs (Section 2: a
periodic Voronoi tessellation, uniformly random orientations, twins).
The paper's own Matern hard-core realizations and EBSD data are not
available; the recipes below are synthetic analogues of the same shape:

* grains: periodic Voronoi cells of ``n_grains`` i.i.d. uniform seeds
  (a fixed-count binomial pattern), assigned over voxel centres with the
  minimum-image distance (Section 2.1, the tessellation equation);
* orientations: Haar-uniform on SO(3) (Section 2.2);
* twins (a cubic stand-in for the tetragonal twin law of Section 2.2):
  a grain is cut by a plane normal to one of its four crystal {111}
  normals; the part beyond the (1 - f) quantile of the signed distance
  becomes a twin domain whose orientation is the parent's rotated by 180
  degrees about that normal.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.spatial import cKDTree

# ---------------------------------------------------------------------------
# Table 1 of the paper: 12 dislocation slip systems and 4 twinning
# pseudo-slip systems, Miller indices in the (pseudo-cubic) crystal frame.
# The table prints system 9 with the same plane and direction as system 7;
# the ordinary ("o") direction on (1-11) is read as [110], the only <110]
# direction with zero third index lying in that plane.
# ---------------------------------------------------------------------------
_TABLE1 = [
    # plane          direction       kind
    ((1, 1, -1), (0, 1, 1), "s"),
    ((1, 1, -1), (1, 0, 1), "s"),
    ((1, 1, -1), (1, -1, 0), "o"),
    ((-1, 1, 1), (0, -1, 1), "s"),
    ((-1, 1, 1), (-1, 0, -1), "s"),
    ((-1, 1, 1), (-1, -1, 0), "o"),
    ((1, -1, 1), (0, 1, 1), "s"),
    ((1, -1, 1), (1, 0, -1), "s"),
    ((1, -1, 1), (1, 1, 0), "o"),   # printed as [011]; see note above
    ((1, 1, 1), (0, 1, -1), "s"),
    ((1, 1, 1), (1, 0, -1), "s"),
    ((1, 1, 1), (1, -1, 0), "o"),
    # twinning pseudo-slip systems (unidirectional)
    ((1, 1, -1), (1, 1, 2), "t"),
    ((-1, 1, 1), (-1, 1, -2), "t"),
    ((1, -1, 1), (1, -1, -2), "t"),
    ((1, 1, 1), (1, 1, -2), "t"),
]

FAMILY_SLIP = 0
FAMILY_TWIN = 1


@dataclasses.dataclass
class SystemSet:
    """Slip/twin systems: Miller plane normals, directions, family, tau0."""
    n_miller: np.ndarray   # [S,3] float64
    l_miller: np.ndarray   # [S,3] float64
    family: np.ndarray     # [S] int32, 0 slip, 1 twin
    kind: list             # 'o', 's' or 't' per system
    tau0: np.ndarray       # [S] float64, MPa


def schmid_half_orientation(systems: "SystemSet", index: int = 0) -> np.ndarray:
    """Bunge angles of a crystal whose lab x-axis is the crystal direction
    (n + l)/|n + l| of system `index` (plane normal n, direction l, unit
    pseudo-cubic vectors): under uniaxial stress along x that system has
    the largest possible Schmid factor, 1/2.  The lab y-axis is
    (l - n)/|l - n|."""
    n = np.asarray(systems.n_miller[index], dtype=np.float64)
    l = np.asarray(systems.l_miller[index], dtype=np.float64)
    n = n / np.linalg.norm(n)
    l = l / np.linalg.norm(l)
    a = (n + l) / np.linalg.norm(n + l)
    b = (l - n) / np.linalg.norm(l - n)
    Q = np.stack([a, b, np.cross(a, b)])      # rows: lab axes in the crystal frame
    return matrix_to_bunge(Q)


def table1_systems(with_twins: bool = True, tau0_o: float = 130.0,
                   tau0_s: float = 200.0, tau0_t: float = 130.0) -> SystemSet:
    """Systems of Table 1 with per-kind initial resistances (MPa).

    Defaults are the paper's values (Section 3, plastic parameters):
    tau0 = 130 MPa for ordinary dislocations and twins, 200 MPa for
    superdislocations.
    """
    rows = _TABLE1 if with_twins else _TABLE1[:12]
    n = np.array([r[0] for r in rows], dtype=np.float64)
    l = np.array([r[1] for r in rows], dtype=np.float64)
    kind = [r[2] for r in rows]
    fam = np.array([FAMILY_TWIN if k == "t" else FAMILY_SLIP for k in kind],
                   dtype=np.int32)
    t0 = np.array([{"o": tau0_o, "s": tau0_s, "t": tau0_t}[k] for k in kind])
    return SystemSet(n, l, fam, kind, t0)


def config_systems(with_twins: bool, r0_slip: float = 80.0,
                   r0_twin: float = 120.0) -> SystemSet:
    """Table 1 systems with a single r0 per family (the synthetic configs)."""
    return table1_systems(with_twins, r0_slip, r0_slip, r0_twin)


# ---------------------------------------------------------------------------
# Law parameter sets
# ---------------------------------------------------------------------------
TWIN_NORTON = 0   # twins follow the slip-type regularized Norton rate, >= 0
TWIN_PAPER = 1    # twin-fraction rate with K_c (f_m - sum f) prefactor


@dataclasses.dataclass
class FamilyLaw:
    Q: float
    b: float
    c: float
    d: float
    K: float
    n: float
    q_self: float
    q_latent: float


@dataclasses.dataclass
class Law:
    slip: FamilyLaw
    twin: FamilyLaw
    twin_mode: int = TWIN_NORTON
    K_c: float = 0.0
    f_m: float = 1.0
    gamma_T: float = 1.0 / math.sqrt(2.0)
    eta: float = 1.0e4


def cubic_stiffness(c11: float, c12: float, c44: float) -> np.ndarray:
    """Voigt 6x6 (order 11,22,33,23,13,12; engineering shear), MPa."""
    C = np.zeros((6, 6))
    C[:3, :3] = c12
    np.fill_diagonal(C[:3, :3], c11)
    C[3, 3] = C[4, 4] = C[5, 5] = c44
    return C


def tetragonal_stiffness(c11, c33, c12, c13, c44, c66) -> np.ndarray:
    """Voigt 6x6 of a tetragonal crystal with c along x3, MPa."""
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = c11
    C[2, 2] = c33
    C[0, 1] = C[1, 0] = c12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = c13
    C[3, 3] = C[4, 4] = c44
    C[5, 5] = c66
    return C


def config_law() -> tuple[np.ndarray, Law]:
    """Stiffness and law of the synthetic configurations (cubic, MPa, s)."""
    C = cubic_stiffness(183000.0, 74500.0, 105000.0)
    fam = FamilyLaw(Q=40.0, b=10.0, c=1.0e4, d=300.0, K=10.0, n=10.0,
                    q_self=1.0, q_latent=1.4)
    return C, Law(slip=fam, twin=dataclasses.replace(fam), eta=1.0e4)


def paper_law(b: float = 10.0, q_latent: float = 1.0) -> tuple[np.ndarray, Law]:
    """The paper's gamma-TiAl set (Section 3).  b and q are not given there
    and must be supplied; kinematic hardening is absent (c = d = 0)."""
    C = tetragonal_stiffness(183000.0, 183000.0, 74000.0, 74000.0,
                             105000.0, 78000.0)
    slip = FamilyLaw(Q=9.57, b=b, c=0.0, d=0.0, K=104.0, n=6.42,
                     q_self=1.0, q_latent=q_latent)
    twin = FamilyLaw(Q=10.5, b=b, c=0.0, d=0.0, K=104.0, n=6.42,
                     q_self=1.0, q_latent=q_latent)
    return C, Law(slip=slip, twin=twin, twin_mode=TWIN_PAPER, K_c=1.45,
                  f_m=0.8, gamma_T=1.0 / math.sqrt(2.0), eta=1.0e4)


# ---------------------------------------------------------------------------
# Orientations
# ---------------------------------------------------------------------------
def _quat_to_matrix(q: np.ndarray) -> np.ndarray:
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - z * w)
    R[..., 0, 2] = 2 * (x * z + y * w)
    R[..., 1, 0] = 2 * (x * y + z * w)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - x * w)
    R[..., 2, 0] = 2 * (x * z - y * w)
    R[..., 2, 1] = 2 * (y * z + x * w)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def matrix_to_bunge(R: np.ndarray) -> np.ndarray:
    """Euler angles (phi1, Phi, phi2) with R = Rz(phi1) Rx(Phi) Rz(phi2)
    (active rotations, v_lab = R v_crystal)."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty(R.shape[:-2] + (3,))
    c = np.clip(R[..., 2, 2], -1.0, 1.0)
    Phi = np.arccos(c)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    regular = s > 1e-10
    phi1 = np.where(regular, np.arctan2(R[..., 0, 2], -R[..., 1, 2]),
                    np.arctan2(R[..., 1, 0], R[..., 0, 0]))
    phi2 = np.where(regular, np.arctan2(R[..., 2, 0], R[..., 2, 1]), 0.0)
    out[..., 0] = np.mod(phi1, 2 * np.pi)
    out[..., 1] = Phi
    out[..., 2] = np.mod(phi2, 2 * np.pi)
    return out


def bunge_to_matrix(e: np.ndarray) -> np.ndarray:
    """Inverse of :func:`matrix_to_bunge` (used by the twin construction)."""
    e = np.asarray(e, dtype=np.float64)
    c1, s1 = np.cos(e[..., 0]), np.sin(e[..., 0])
    c, s = np.cos(e[..., 1]), np.sin(e[..., 1])
    c2, s2 = np.cos(e[..., 2]), np.sin(e[..., 2])
    R = np.empty(e.shape[:-1] + (3, 3))
    R[..., 0, 0] = c1 * c2 - s1 * c * s2
    R[..., 0, 1] = -c1 * s2 - s1 * c * c2
    R[..., 0, 2] = s1 * s
    R[..., 1, 0] = s1 * c2 + c1 * c * s2
    R[..., 1, 1] = -s1 * s2 + c1 * c * c2
    R[..., 1, 2] = -c1 * s
    R[..., 2, 0] = s * s2
    R[..., 2, 1] = s * c2
    R[..., 2, 2] = c
    return R


def haar_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotation matrices uniform on SO(3) (Shoemake's quaternion method)."""
    u = rng.random((n, 3))
    a, b = np.sqrt(1 - u[:, 0]), np.sqrt(u[:, 0])
    q = np.stack([a * np.sin(2 * np.pi * u[:, 1]), a * np.cos(2 * np.pi * u[:, 1]),
                  b * np.sin(2 * np.pi * u[:, 2]), b * np.cos(2 * np.pi * u[:, 2])],
                 axis=1)
    return _quat_to_matrix(q)


# ---------------------------------------------------------------------------
# Periodic Voronoi tessellation on voxel centres
# ---------------------------------------------------------------------------
def voronoi_labels(shape: tuple[int, int, int], seeds: np.ndarray) -> np.ndarray:
    """Label grid [nz][ny][nx] (x fastest) of the periodic Voronoi cells.

    ``shape`` is (nz, ny, nx); ``seeds`` are (x, y, z) in voxel units in the
    box [0,nx)x[0,ny)x[0,nz).  Voxel (i,j,k) has centre (i+1/2, j+1/2, k+1/2).
    """
    nz, ny, nx = shape
    box = np.array([nx, ny, nz], dtype=np.float64)
    tree = cKDTree(np.mod(seeds, box), boxsize=box)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    pts = np.stack([x.ravel() + 0.5, y.ravel() + 0.5, z.ravel() + 0.5], axis=1)
    _, idx = tree.query(pts, k=1)
    return idx.astype(np.int32).reshape(shape)


_CUBIC_111 = np.array([[1, 1, 1], [-1, 1, 1], [1, -1, 1], [1, 1, -1]],
                      dtype=np.float64) / math.sqrt(3.0)


@dataclasses.dataclass
class Microstructure:
    labels: np.ndarray      # [nz][ny][nx] int32
    euler: np.ndarray       # [n_labels][3] float64, radians
    n_grains: int
    twinned: np.ndarray     # indices of twinned grains
    twin_fraction: np.ndarray

    @property
    def shape(self):
        return self.labels.shape

    @property
    def n_labels(self):
        return self.euler.shape[0]


def make_rve(n: int | tuple, n_grains: int, seed: int,
             twin_share: float = 0.0, f_range=(0.2, 0.5)) -> Microstructure:
    """Seeded periodic Voronoi RVE with Haar orientations and optional twins.

    ``twin_share`` is the fraction of grains split into a twin pair
    (1.0: every grain; 0.5: a random half).  A twinned grain g receives the
    extra label n_grains + j, j being its rank among the twinned grains.
    """
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    box = np.array([nx, ny, nz], dtype=np.float64)
    seeds = rng.random((n_grains, 3)) * box
    labels = voronoi_labels(shape, seeds)
    R = haar_rotations(rng, n_grains)
    n_tw = int(round(twin_share * n_grains))
    twinned = np.sort(rng.choice(n_grains, size=n_tw, replace=False)) if n_tw else \
        np.zeros(0, dtype=np.int64)
    fracs = rng.uniform(f_range[0], f_range[1], size=n_tw)
    normals = rng.integers(0, 4, size=n_tw)
    eul = [matrix_to_bunge(R)]
    if n_tw:
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                              indexing="ij")
        centres = np.stack([x + 0.5, y + 0.5, z + 0.5], axis=-1)
        R_tw = np.empty((n_tw, 3, 3))
        flat = labels.reshape(-1)
        cflat = centres.reshape(-1, 3)
        for j, g in enumerate(twinned):
            nc = _CUBIC_111[normals[j]]
            R_tw[j] = R[g] @ (2.0 * np.outer(nc, nc) - np.eye(3))
            sel = np.nonzero(flat == g)[0]
            if sel.size == 0:
                continue
            d = cflat[sel] - seeds[g]
            d -= box * np.round(d / box)
            h = d @ (R[g] @ nc)
            thr = np.quantile(h, 1.0 - fracs[j])
            flat[sel[h > thr]] = n_grains + j
        labels = flat.reshape(shape)
        eul.append(matrix_to_bunge(R_tw))
    return Microstructure(labels=labels, euler=np.concatenate(eul, axis=0),
                          n_grains=n_grains, twinned=twinned, twin_fraction=fracs)


# ---------------------------------------------------------------------------
# Loading paths (mixed: strain-controlled or stress-controlled components)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class LoadPath:
    t: np.ndarray            # [n_steps+1] s
    strain_ctrl: np.ndarray  # [n_steps][6] uint8; 1 = mean strain prescribed
    target: np.ndarray       # [n_steps][6] strain (if ctrl) else stress, MPa

    @property
    def n_steps(self):
        return self.target.shape[0]


def uniaxial_path(total_strain: float, n_steps: int, rate: float = 1.0e-3,
                  axis: int = 0) -> LoadPath:
    """Uniaxial loading along ``axis`` at constant mean strain rate with the
    other five mean stress components held at zero.  Components follow the
    order 11, 22, 33, 23, 13, 12 (tensor components)."""
    dt = abs(total_strain) / abs(rate) / n_steps
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    ctrl = np.zeros((n_steps, 6), dtype=np.uint8)
    ctrl[:, axis] = 1
    tgt = np.zeros((n_steps, 6))
    tgt[:, axis] = np.sign(total_strain) * abs(rate) * t[1:]
    return LoadPath(t=t, strain_ctrl=ctrl, target=tgt)


# ---------------------------------------------------------------------------
# The five synthetic workloads.  Seeds: workload i uses 20240215 + i; batch
# member j uses 20240300 + j.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    rve: Microstructure
    systems: SystemSet
    C: np.ndarray
    law: Law
    path: LoadPath


def workload(i: int, n_override: Optional[int] = None,
             steps_override: Optional[int] = None) -> Workload:
    """Workload ``i`` (0..2, 4) as a single-RVE problem."""
    C, law = config_law()
    if i == 0:
        n, g, tw, strain, steps, twins = 16, 8, 0.0, 0.005, 10, False
        name = "16^3 untwinned, 12 slip systems, 0.5% in 10 steps"
    elif i in (1, 4):
        n, g, tw, strain, steps, twins = 64, 100, 1.0, 0.02, 50, True
        name = "64^3 fully twinned, 12+4 systems, 2% in 50 steps"
    elif i == 2:
        n, g, tw, strain, steps, twins = 128, 500, 0.5, 0.02, 100, True
        name = "128^3 half twinned, 12+4 systems, 2% in 100 steps"
    else:
        raise ValueError("workload index must be 0, 1, 2 or 4")
    seed = 20240215 + (1 if i == 4 else i)
    if n_override is not None:
        n = n_override
    per_step = strain / steps
    if steps_override is not None:
        steps = steps_override
    rve = make_rve(n, g, seed, twin_share=tw)
    systems = config_systems(with_twins=twins)
    path = uniaxial_path(per_step * steps, steps)
    return Workload(name=name, rve=rve, systems=systems, C=C, law=law, path=path)


def batch_members(count: int = 32, sizes=(32, 48, 64, 96)) -> list[Microstructure]:
    """Batch workload: uneven grid sizes, 50-300 grains, twinned iff j even."""
    out = []
    for j in range(count):
        rng = np.random.default_rng(20240300 + j)
        n = int(rng.choice(sizes))
        g = int(rng.integers(50, 301))
        out.append(make_rve(n, g, 20240300 + j + 1000,
                            twin_share=0.5 if j % 2 == 0 else 0.0))
    return out
