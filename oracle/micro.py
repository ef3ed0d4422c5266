"""CPU ORACLE of the stochastic microstructure model -- test infrastructure
only (``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may use it).  Plain, slow code written from Section 2
of the paper; it shares no code with the GPU library.

Pipeline (Section 2.1, then 2.2):

1. Primary points: a Poisson number of i.i.d. uniform points in the
   periodic window W, on a lattice of 1/q voxel (integer coordinates).
2. Matern hard-core thinning, type II with the generation order as the
   mark: a point is kept iff no earlier point lies within distance r
   (periodic minimum image).  The kept points, in order, are the
   generators s_0 .. s_{N_W - 1}.
3. Periodic Voronoi tessellation on the voxel centres (the tessellation
   equation of Section 2.1); a centre equidistant from several generators
   goes to the lowest index.  Distances are exact integers.
4. Grain graph: grains sharing a voxel face (periodic) are neighbours;
   grain volumes in voxels.
5. Neighbouring twins: N_neigh ~ Poisson(p_neigh N_W / 2) conditioned on
   N_neigh <= N_W / 2 (the rejection of Section 2.2.1); pairs are drawn
   until N_neigh pairs exist or no free grain has a free neighbour.  The
   first grain's orientation is uniform under the condition that a habit
   plane lies on the joint facet; the second's is the first's rotated by
   theta about [100] or [010].
6. The other grains: Haar-uniform orientations.
7. Inclusion twins: with probability p_incl per grain, a slab of thickness
   delta through a random point of the grain boundary, parallel to a habit
   plane, becomes a new grain whose orientation is the parent's rotated by
   theta about the matching axis.

Random numbers come from one SplitMix64 stream (Steele, Lea and Flood,
2014), consumed in the order the steps above name; see ``generate``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


# ---------------------------------------------------------------------------
# Random stream
# ---------------------------------------------------------------------------
def splitmix64(state: int) -> tuple[int, int]:
    """One SplitMix64 step: (new state, output)."""
    state = (state + GAMMA) & MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return state, z ^ (z >> 31)


class Stream:
    """Sequential draws: u64, uniform doubles in [0, 1) from the top 53
    bits, integers in [0, m) by the high 32 bits times m, shifted."""

    def __init__(self, seed: int):
        self.state = seed & MASK
        self.count = 0

    def u64(self) -> int:
        self.state, z = splitmix64(self.state)
        self.count += 1
        return z

    def uniform(self) -> float:
        return (self.u64() >> 11) * 2.0 ** -53

    def below(self, m: int) -> int:
        assert 0 < m < 2 ** 32
        return ((self.u64() >> 32) * m) >> 32


def poisson_inverse(u: float, mu: float, kmax: int) -> int:
    """Smallest k with P(N <= k) > u for N ~ Poisson(mu) conditioned on
    N <= kmax (inversion).  The weights mu^k / k! are taken relative to the
    mode m = min(floor(mu), kmax), built outwards from w_m = 1 by the ratio
    w_k / w_{k-1} = mu / k, and summed in ascending k."""
    if mu <= 0.0 or kmax <= 0:
        return 0
    m = min(int(mu), kmax)
    w = [0.0] * (kmax + 1)
    w[m] = 1.0
    for k in range(m + 1, kmax + 1):
        w[k] = w[k - 1] * mu / k
    for k in range(m - 1, -1, -1):
        w[k] = w[k + 1] * (k + 1) / mu
    T = 0.0
    for k in range(kmax + 1):
        T += w[k]
    target = u * T
    acc = 0.0
    for k in range(kmax + 1):
        acc += w[k]
        if acc > target:
            return k
    return kmax


def poisson_kmax(mu: float) -> int:
    """Upper end of the primary count's support used by the inversion
    (beyond it the weights are below 1e-80 of the mode's)."""
    return int(mu + 20.0 * math.sqrt(mu) + 20.0)


# ---------------------------------------------------------------------------
# Point process and tessellation (Section 2.1)
# ---------------------------------------------------------------------------
def periodic_d2(a: np.ndarray, b: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Squared minimum-image distance of integer points (exact int64)."""
    d = np.abs(np.asarray(a, np.int64) - np.asarray(b, np.int64))
    d = np.minimum(d, L - d)
    return np.sum(d * d, axis=-1)


def matern_ii_keep(pts: np.ndarray, L: np.ndarray, r_q: float) -> np.ndarray:
    """Keep flags of Matern type II thinning with marks = order: i is kept
    iff no j < i has minimum-image distance <= r_q (lattice units)."""
    n = pts.shape[0]
    keep = np.ones(n, dtype=bool)
    r2 = r_q * r_q
    for i in range(1, n):
        d2 = periodic_d2(pts[:i], pts[i][None, :], L)
        if np.any(d2.astype(np.float64) <= r2):
            keep[i] = False
    return keep


def voxel_centres(shape, q: int) -> np.ndarray:
    """Integer centres (q i + q/2, ...) of all voxels, [nvox][3] (x, y, z),
    x fastest."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.int64) * q + q // 2


def voronoi_labels_at(centres: np.ndarray, seeds: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Label of each given centre: the generator at the smallest squared
    minimum-image distance, the lowest index among equals."""
    out = np.empty(centres.shape[0], dtype=np.int32)
    step = max(1, 4_000_000 // max(1, seeds.shape[0]))
    for a in range(0, centres.shape[0], step):
        c = centres[a:a + step]
        d2 = periodic_d2(c[:, None, :], seeds[None, :, :], L)
        out[a:a + step] = np.argmin(d2, axis=1)     # first minimum = lowest index
    return out


def voronoi_labels(shape, seeds: np.ndarray, q: int) -> np.ndarray:
    nz, ny, nx = shape
    L = np.array([nx, ny, nz], np.int64) * q
    return voronoi_labels_at(voxel_centres(shape, q), seeds, L).reshape(shape)


def grain_graph(labels: np.ndarray, n: int):
    """Neighbour sets (face-adjacent voxels with different labels, periodic)
    as a boolean matrix [n][n], and voxel counts [n]."""
    adj = np.zeros((n, n), dtype=bool)
    for ax in range(3):
        a = labels
        b = np.roll(labels, -1, axis=ax)
        m = a != b
        adj[a[m], b[m]] = True
        adj[b[m], a[m]] = True
    vol = np.bincount(labels.ravel(), minlength=n).astype(np.int64)
    return adj, vol


# ---------------------------------------------------------------------------
# Orientations (Section 2.2)
# ---------------------------------------------------------------------------
def axis_rotation(axis: np.ndarray, angle: float) -> np.ndarray:
    """Right-handed rotation by ``angle`` about the unit vector ``axis``
    (Rodrigues)."""
    k = np.asarray(axis, dtype=np.float64)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def habit_normal(axis_index: int, theta: float) -> np.ndarray:
    """Crystal-frame unit normal of the habit plane that goes with a twin
    rotation about [100] (axis_index 0: plane (011)) or [010] (1: plane
    (101)), for a tetragonal lattice with a / c = tan(theta / 2) (the
    twin angle theta = 2 atan(a / c))."""
    ac = math.tan(0.5 * theta)
    v = np.array([0.0, 1.0, ac]) if axis_index == 0 else np.array([1.0, 0.0, ac])
    return v / math.sqrt(float(v @ v))


def twin_rotation(O: np.ndarray, axis_index: int, theta: float) -> np.ndarray:
    """Orientation of the twin: O rotated by theta about its crystal [100]
    (axis_index 0) or [010] (1), O R.  The sense of each rotation is the one
    that carries the parent's habit plane onto one of the twin's (so that
    both grains have a habit plane on the joint facet): right-handed about
    [100] (the (011) normal becomes the twin's (0-11)-type normal
    (0, 1, -a/c)) and left-handed about [010] (the (101) normal becomes
    (1, 0, -a/c))."""
    if axis_index == 0:
        return O @ axis_rotation(np.array([1.0, 0.0, 0.0]), theta)
    return O @ axis_rotation(np.array([0.0, 1.0, 0.0]), -theta)


def align(h: np.ndarray, f: np.ndarray) -> np.ndarray:
    """The rotation of least angle taking unit h to unit f."""
    v = np.cross(h, f)
    s = math.sqrt(float(v @ v))
    c = float(h @ f)
    if s < 1e-15:
        if c > 0:
            return np.eye(3)
        # half turn about any axis normal to h
        p = np.array([1.0, 0.0, 0.0]) if abs(h[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        p = p - (p @ h) * h
        return axis_rotation(p / math.sqrt(float(p @ p)), math.pi)
    return axis_rotation(v / s, math.atan2(s, c))


def haar_rotation(u1: float, u2: float, u3: float) -> np.ndarray:
    """Uniform rotation from three uniforms (Shoemake's unit quaternion)."""
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    w, x, y, z = (a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2),
                  b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def facet_normal(si: np.ndarray, sj: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Unit normal of the Voronoi facet between generators si and sj (the
    bisector plane of the minimum-image difference), lattice units."""
    d = np.asarray(sj, np.int64) - np.asarray(si, np.int64)      # in (-L, L)
    d = np.where(d > L / 2, d - L, np.where(d < -L / 2, d + L, d))  # |d| = L/2 stays
    v = d.astype(np.float64)
    return v / math.sqrt(float(v @ v))


def boundary_point(g: int, seeds: np.ndarray, L: np.ndarray, direction: np.ndarray) -> np.ndarray:
    """Point where the ray from generator g along ``direction`` leaves the
    (continuous, periodic) Voronoi cell of g: the smallest t over all other
    generators and periodic images m of |m - s_g|^2 / (2 (m - s_g) . d)
    among those ahead of the ray.  Lattice units."""
    sg = seeds[g].astype(np.float64)
    tbest = math.inf
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                shift = L * np.array([sx, sy, sz])
                diff = (seeds + shift - seeds[g]).astype(np.float64)
                if sx == sy == sz == 0:
                    diff = np.delete(diff, g, axis=0)
                den = diff @ direction
                num = np.sum(diff * diff, axis=1)
                ok = den > 0
                if np.any(ok):
                    tbest = min(tbest, float(np.min(num[ok] / (2.0 * den[ok]))))
    return sg + tbest * direction


def wrap_point(x: np.ndarray, L: np.ndarray) -> np.ndarray:
    """x - L floor(x / L), componentwise."""
    x = np.asarray(x, np.float64)
    return x - L * np.floor(x / L)


def slab_members(labels: np.ndarray, g: int, normal: np.ndarray, x0: np.ndarray, half: float,
                 q: int) -> np.ndarray:
    """Voxels of grain g whose centre y has |n . (y - x0)| <= half, with
    x0 wrapped into the window (x0 - L floor(x0 / L)) and y - x0 taken as
    the minimum image (shifted by L where it exceeds L/2 in magnitude); the
    dot product in the fixed order (n0 d0 + n1 d1) + n2 d2 of single double
    operations.  Lattice units."""
    nz, ny, nx = labels.shape
    L = np.array([nx, ny, nz], np.float64) * q
    x0 = wrap_point(x0, L)
    idx = np.nonzero(labels.ravel() == g)[0]
    c = voxel_centres(labels.shape, q)[idx].astype(np.float64)
    d = c - x0
    d = np.where(d > L / 2, d - L, np.where(d < -L / 2, d + L, d))
    t = (normal[0] * d[:, 0] + normal[1] * d[:, 1]) + normal[2] * d[:, 2]
    return idx[np.abs(t) <= half]


# ---------------------------------------------------------------------------
# The whole model
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    shape: tuple                  # (nz, ny, nx)
    lam: float                    # primary intensity per voxel^3
    r: float                      # hard-core radius, voxels
    p_neigh: float = 0.0
    p_incl: float = 0.0
    delta: tuple = (0.1, 0.3)     # relative inclusion thickness bounds
    theta: float = math.radians(69.79)
    seed: int = 1
    q: int = 16                   # lattice points per voxel edge


@dataclasses.dataclass
class Micro:
    labels: np.ndarray            # [nz][ny][nx] int32
    rotations: np.ndarray         # [n_labels][3][3], crystal -> lab
    n_primary: int
    points: np.ndarray            # primary points [n_primary][3], lattice units
    keep: np.ndarray
    seeds: np.ndarray             # generators [N_W][3]
    adjacency: np.ndarray
    volumes: np.ndarray
    n_neigh_drawn: int
    pairs: list                   # (k, l, axis_index)
    inclusions: list              # (parent, child label, axis_index, half, normal, x0)
    draws: int


def generate(p: Params, labels_only: bool = False) -> Micro:
    """The model of Section 2 with the draws in this order:
    1 uniform: primary count (Poisson inversion, support up to poisson_kmax);
    3 per point: x, y, z lattice coordinates (below(q n_x), ...);
    [p_neigh > 0] 1 uniform: N_neigh; per pair: first grain (below(number
    of free grains with a free neighbour), ascending), its partner
    (below(number of its free neighbours), ascending), the axis (below(2)),
    the angle psi about the facet normal (2 pi uniform);
    3 uniforms per remaining grain, ascending: Haar orientation;
    [p_incl > 0] per grain, ascending: 1 uniform (selected iff < p_incl);
    if selected: the axis (below(2)), the ray direction (2 uniforms: z =
    1 - 2 u, phi = 2 pi u), the relative thickness (1 uniform)."""
    nz, ny, nx = p.shape
    q = p.q
    L = np.array([nx, ny, nz], np.int64) * q
    st = Stream(p.seed)
    mu = p.lam * nx * ny * nz
    n_p = poisson_inverse(st.uniform(), mu, poisson_kmax(mu))
    pts = np.zeros((n_p, 3), np.int64)
    for i in range(n_p):
        pts[i] = [st.below(int(L[0])), st.below(int(L[1])), st.below(int(L[2]))]
    keep = matern_ii_keep(pts, L, p.r * q)
    seeds = pts[keep]
    nw = seeds.shape[0]
    labels = voronoi_labels(p.shape, seeds, q) if nw else np.zeros(p.shape, np.int32)
    adj, vol = grain_graph(labels, nw)
    if labels_only:
        return Micro(labels, np.zeros((0, 3, 3)), n_p, pts, keep, seeds, adj, vol, 0, [], [], st.count)

    rot = np.zeros((nw, 3, 3))
    assigned = np.zeros(nw, dtype=bool)
    pairs = []
    n_neigh = 0
    if p.p_neigh > 0 and nw >= 2:
        n_neigh = poisson_inverse(st.uniform(), p.p_neigh * nw / 2.0, nw // 2)
        while len(pairs) < n_neigh:
            free = ~assigned
            cand = [k for k in range(nw) if free[k] and np.any(adj[k] & free)]
            if not cand:
                break
            k = cand[st.below(len(cand))]
            nb = [m for m in range(nw) if adj[k, m] and free[m]]
            l = nb[st.below(len(nb))]
            a = st.below(2)
            psi = 2.0 * math.pi * st.uniform()
            f = facet_normal(seeds[k], seeds[l], L)
            h = habit_normal(a, p.theta)
            Ok = axis_rotation(f, psi) @ align(h, f)
            rot[k] = Ok
            rot[l] = twin_rotation(Ok, a, p.theta)
            assigned[k] = assigned[l] = True
            pairs.append((k, l, a))
    for g in range(nw):
        if not assigned[g]:
            rot[g] = haar_rotation(st.uniform(), st.uniform(), st.uniform())
    inclusions = []
    out = labels.ravel().copy()
    extra = []
    if p.p_incl > 0:
        for g in range(nw):
            if not st.uniform() < p.p_incl:
                continue
            a = st.below(2)
            zc = 1.0 - 2.0 * st.uniform()
            phi = 2.0 * math.pi * st.uniform()
            rho = math.sqrt(max(0.0, 1.0 - zc * zc))
            d = np.array([rho * math.cos(phi), rho * math.sin(phi), zc])
            u = st.uniform()
            x0 = boundary_point(g, seeds, L, d)
            ved = (6.0 * float(vol[g]) / math.pi) ** (1.0 / 3.0)
            delta = (p.delta[0] + (p.delta[1] - p.delta[0]) * u) * ved
            half = 0.5 * delta * q
            n = rot[g] @ habit_normal(a, p.theta)
            child = nw + len(inclusions)
            out[slab_members(labels, g, n, x0, half, q)] = child
            extra.append(twin_rotation(rot[g], a, p.theta))
            inclusions.append((g, child, a, half, n, x0))
    if extra:
        rot = np.concatenate([rot, np.array(extra)], axis=0)
    return Micro(out.reshape(p.shape).astype(np.int32), rot, n_p, pts, keep, seeds, adj, vol,
                 n_neigh, pairs, inclusions, st.count)
