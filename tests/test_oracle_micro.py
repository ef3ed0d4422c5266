"""Pins of the oracle's microstructure model (Section 2) against facts
that do not come from it: the published SplitMix64 outputs, scipy's Poisson
distribution and periodic k-d tree, closed forms (Matern II intensity, cube
cells, slab voxel counts, the twin angle of a tetragonal lattice) and
invariants of the generated structure.  CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.spatial import cKDTree

import oracle.micro as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
THETA = math.radians(69.79)


def test_splitmix64_published_outputs():
    ref = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if not x.startswith("#")]
    s = M.Stream(0)
    assert [s.u64() for _ in range(len(ref))] == ref


def test_stream_uniform_and_below_are_uniform():
    s = M.Stream(12345)
    u = np.array([s.uniform() for _ in range(20000)])
    assert u.min() >= 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    k = np.array([s.below(7) for _ in range(14000)])
    chi2 = stats.chisquare(np.bincount(k, minlength=7)).pvalue
    assert k.min() == 0 and k.max() == 6 and chi2 > 1e-4


@pytest.mark.parametrize("mu,kmax", [(3.5, 60), (10.0, 6), (930.0, 905), (1920.0, M.poisson_kmax(1920.0))])
def test_poisson_inverse_matches_scipy(mu, kmax):
    """Quantiles on a grid of u against scipy's (conditioned on N <= kmax:
    the rejection until N <= kmax of Section 2.2.1)."""
    top = stats.poisson.cdf(kmax, mu)
    for u in (np.arange(400) + 0.5) / 400:
        k = M.poisson_inverse(float(u), mu, kmax)
        assert 0 <= k <= kmax
        assert stats.poisson.cdf(k, mu) / top > u * (1 - 1e-12)
        if k > 0:
            assert stats.poisson.cdf(k - 1, mu) / top <= u * (1 + 1e-12)
    assert M.poisson_inverse(0.3, 0.0, 5) == 0


def test_matern_ii_definition_and_intensity():
    """Kept points are more than r apart; every removed point has an
    earlier point (kept or not) within r; the kept intensity matches the
    type II closed form (1 - exp(-lam V_r)) / V_r within 4 sigma."""
    n, q, r = 256, 16, 5.0
    lam = 1920 / n ** 3
    s = M.Stream(3)
    mu = lam * n ** 3
    n_p = M.poisson_inverse(s.uniform(), mu, M.poisson_kmax(mu))
    L = np.array([n * q] * 3)
    pts = np.array([[s.below(n * q) for _ in range(3)] for _ in range(n_p)])
    keep = M.matern_ii_keep(pts, L, r * q)
    tree = cKDTree(pts[keep].astype(float), boxsize=L.astype(float))
    assert len(tree.query_pairs(r * q)) == 0
    full = cKDTree(pts.astype(float), boxsize=L.astype(float))
    for i in np.nonzero(~keep)[0]:
        near = full.query_ball_point(pts[i].astype(float), r * q)
        assert any(j < i for j in near)
    Vr = 4 / 3 * math.pi * r ** 3
    expect = (1 - math.exp(-lam * Vr)) / Vr * n ** 3
    assert abs(keep.sum() - expect) < 4 * math.sqrt(expect)


def test_voronoi_labels_against_periodic_kdtree():
    shape, q = (12, 16, 20), 16
    nz, ny, nx = shape
    L = np.array([nx, ny, nz]) * q
    rng = np.random.default_rng(5)
    seeds = np.stack([rng.integers(0, L[i], 25) for i in range(3)], axis=1)
    lab = M.voronoi_labels(shape, seeds, q)
    c = M.voxel_centres(shape, q).astype(float)
    d, idx = cKDTree(seeds.astype(float), boxsize=L.astype(float)).query(c, k=2)
    chosen = M.periodic_d2(c.astype(np.int64), seeds[lab.ravel()], L)
    assert np.allclose(chosen, d[:, 0] ** 2, rtol=1e-12)
    clear = d[:, 1] ** 2 - d[:, 0] ** 2 > 0.5
    assert np.array_equal(lab.ravel()[clear], idx[clear, 0])


def test_voronoi_tie_goes_to_the_lowest_index():
    q = 16
    # two generators symmetric about the centre of voxel (2, 0, 0)
    seeds = np.array([[40 + 24, 8, 8], [40 - 24, 8, 8], [120, 8, 8]])
    lab = M.voronoi_labels((1, 1, 8), seeds, q)
    assert lab[0, 0, 2] == 0
    seeds2 = seeds[[1, 0, 2]]
    assert M.voronoi_labels((1, 1, 8), seeds2, q)[0, 0, 2] == 0


def test_grain_graph_closed_forms():
    lab = np.zeros((3, 4, 8), np.int32)
    for i in range(8):
        lab[..., i] = i // 2                 # slabs along x, periodic ring 0-1-2-3-0
    adj, vol = M.grain_graph(lab, 4)
    ring = np.zeros((4, 4), bool)
    for a in range(4):
        ring[a, (a + 1) % 4] = ring[(a + 1) % 4, a] = True
    assert np.array_equal(adj, ring) and np.all(vol == 24)
    cb = np.arange(8, dtype=np.int32).reshape(2, 2, 2)   # 2x2x2 cells, one voxel each
    adj, vol = M.grain_graph(cb, 8)
    assert np.all(adj.sum(axis=1) == 3) and np.all(vol == 1)
    assert not np.any(np.diag(adj))


def test_twin_geometry_of_the_tetragonal_lattice():
    """theta = 2 atan(a/c): the twin rotation about [100] by theta maps the
    parent's (011) normal onto the child's (0-11)-type normal (0, 1, -a/c),
    so both grains have a habit plane on the joint facet; likewise [010]
    with (101).  The misorientation angle is theta."""
    ac = math.tan(THETA / 2)
    rng = np.random.default_rng(1)
    O = M.haar_rotation(*rng.random(3))
    assert np.allclose(O @ O.T, np.eye(3), atol=1e-14) and np.linalg.det(O) == pytest.approx(1)
    for a in (0, 1):
        h = M.habit_normal(a, THETA)
        Ot = M.twin_rotation(O, a, THETA)
        cosang = (np.trace(O.T @ Ot) - 1) / 2
        assert math.degrees(math.acos(cosang)) == pytest.approx(69.79, abs=1e-10)
        h_child = np.array([0.0, 1.0, -ac]) if a == 0 else np.array([1.0, 0.0, -ac])
        h_child /= np.linalg.norm(h_child)
        assert np.allclose(Ot @ h_child, O @ h, atol=1e-14)
    f = np.array([0.3, -0.4, 0.866])
    f /= np.linalg.norm(f)
    h = M.habit_normal(0, THETA)
    assert np.allclose(M.align(h, f) @ h, f, atol=1e-14)
    assert np.allclose(M.align(h, -h) @ h, -h, atol=1e-14)


def test_haar_rotation_mean_is_zero():
    s = M.Stream(9)
    R = np.array([M.haar_rotation(s.uniform(), s.uniform(), s.uniform()) for _ in range(4000)])
    assert np.abs(R.mean(axis=0)).max() < 4 * math.sqrt(1 / 3 / 4000)


def test_boundary_point_of_cubic_cells():
    """Generators on a 2x2x2 lattice of spacing 32 (box 64): the cells are
    cubes of side 32, so a ray from a generator leaves at t = 16 / max|d_i|."""
    g = np.array([[16 + 32 * i, 16 + 32 * j, 16 + 32 * k] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    L = np.array([64, 64, 64])
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        x = M.boundary_point(5, g, L, d)
        assert np.allclose(x, g[5] + 16.0 / np.abs(d).max() * d, rtol=0, atol=1e-12)


def test_slab_members_closed_form():
    lab = np.zeros((10, 6, 5), np.int32)
    q = 16
    for c, half in ((37.0, 20.0), (8.0, 8.0), (150.0, 41.0), (-30.0, 25.0)):
        idx = M.slab_members(lab, 0, np.array([0.0, 0.0, 1.0]), np.array([3.0, 7.0, c]), half, q)
        zc = np.arange(10) * q + q // 2
        dz = (zc - (c % 160)) % 160
        dz = np.where(dz > 80, dz - 160, dz)
        assert idx.size == 30 * int(np.sum(np.abs(dz) <= half))


@pytest.mark.parametrize("p_neigh,p_incl", [(1.0, 0.0), (0.0, 1.0), (0.0, 0.0), (1.0, 0.5)])
def test_generated_structure_invariants(p_neigh, p_incl):
    p = M.Params(shape=(24, 28, 32), lam=45 / (24 * 28 * 32), r=2.5, p_neigh=p_neigh,
                 p_incl=p_incl, delta=(0.2, 0.4), seed=11)
    m = M.generate(p)
    nw = m.seeds.shape[0]
    assert m.rotations.shape[0] == nw + len(m.inclusions)
    assert np.allclose(np.einsum("nij,nkj->nik", m.rotations, m.rotations), np.eye(3), atol=1e-13)
    base = M.voronoi_labels(p.shape, m.seeds, p.q)
    L = np.array(p.shape[::-1]) * p.q
    used = set()
    assert m.n_neigh_drawn <= nw // 2 and len(m.pairs) <= m.n_neigh_drawn
    for k, l, a in m.pairs:
        assert m.adjacency[k, l] and k not in used and l not in used
        used |= {k, l}
        f = M.facet_normal(m.seeds[k], m.seeds[l], L)
        assert np.allclose(m.rotations[k] @ M.habit_normal(a, p.theta), f, atol=1e-13)
        hc = np.array([0.0, 1.0, -math.tan(p.theta / 2)]) if a == 0 else \
            np.array([1.0, 0.0, -math.tan(p.theta / 2)])
        assert np.allclose(m.rotations[l] @ (hc / np.linalg.norm(hc)), f, atol=1e-13)
    if p_neigh > 0:
        assert len(m.pairs) > 0
    for g, child, a, half, n, x0 in m.inclusions:
        mine = m.labels == child
        assert np.all(base[mine] == g)           # inside the parent
        assert half > 0
    if p_incl == 1.0:
        assert len(m.inclusions) == nw
    assert np.array_equal(m.labels[m.labels < nw], base[m.labels < nw])
    m2 = M.generate(p)
    assert np.array_equal(m.labels, m2.labels) and np.array_equal(m.rotations, m2.rotations)
