"""The microstructure model of Section 2 on the device (include/cpfft_micro.h)
against the oracle: Matern thinning, Voronoi labels, grain graph and slabs
bit-exact on identical inputs (ragged tiles, ties, overflowing candidate
lists, a 256^3 window on sampled voxels); the whole generator with the
same draws, pair choices and counts, rotations to rounding, and labels
equal wherever the slab decision is not within rounding of its edge."""
import math

import numpy as np
import pytest

import oracle.micro as M
import rvegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
cp = pytest.importorskip("paper_2402_09996_amd")

THETA = math.radians(69.79)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cp._lib.lib()
    yield


def _p4(a):
    out = np.zeros((a.shape[0], 4), np.int32)
    out[:, :3] = a
    return torch.from_numpy(out).cuda()


@pytest.mark.parametrize("n,L,r", [(500, (320, 384, 256), 40.0), (2000, (4096, 4096, 4096), 80.0), (1, (16, 16, 16), 3.0)])
def test_thin_matches_oracle(n, L, r):
    rng = np.random.default_rng(n)
    pts = np.stack([rng.integers(0, L[i], n) for i in range(3)], axis=1)
    pts[: n // 10] = np.stack([rng.integers(L[i] - 20, L[i], n // 10) for i in range(3)], axis=1)  # near the wrap
    keep = cp.micro_thin(_p4(pts), L, r).cpu().numpy().astype(bool)
    ref = M.matern_ii_keep(pts, np.array(L), r)
    assert np.array_equal(keep, ref)


@pytest.mark.parametrize("shape,n,q", [((16, 16, 16), 30, 16), ((20, 24, 28), 45, 16), ((9, 13, 5), 7, 4),
                                       ((16, 16, 16), 3000, 16), ((1, 1, 8), 3, 16)])
def test_labels_match_oracle(shape, n, q):
    print("case", shape, n, q, flush=True)
    nz, ny, nx = shape
    L = np.array([nx, ny, nz]) * q
    rng = np.random.default_rng(7)
    seeds = np.stack([rng.integers(0, L[i], n) for i in range(3)], axis=1)
    if shape == (1, 1, 8):
        seeds = np.array([[64, 8, 8], [16, 8, 8], [120, 8, 8]])     # a tie at voxel 2: lowest index
    lab, fb = cp.micro_label(shape, q, _p4(seeds))
    ref = M.voronoi_labels(shape, seeds, q)
    assert np.array_equal(lab.cpu().numpy(), ref)
    if n == 3000:
        assert int(fb.item()) > 0          # the candidate lists overflowed: full search
    else:
        assert int(fb.item()) == 0


def test_labels_256_cube_sampled():
    """The 256^3 window of Section 2.3 (lambda = 1920 / 256^3, r = 5):
    labels of 20000 sampled voxels against the oracle's."""
    n, q = 256, 16
    s = M.Stream(3)
    mu = 1920.0
    n_p = M.poisson_inverse(s.uniform(), mu, M.poisson_kmax(mu))
    L = np.array([n * q] * 3)
    pts = np.array([[s.below(n * q) for _ in range(3)] for _ in range(n_p)])
    keep = M.matern_ii_keep(pts, L, 5.0 * q)
    seeds = pts[keep]
    lab, fb = cp.micro_label((n, n, n), q, _p4(seeds))
    lab = lab.cpu().numpy().ravel()
    idx = np.random.default_rng(1).integers(0, n ** 3, 20000)
    c = M.voxel_centres((n, n, n), q)[idx]
    assert np.array_equal(lab[idx], M.voronoi_labels_at(c, seeds, L))
    assert int(fb.item()) == 0


@pytest.mark.parametrize("shape,n", [((16, 16, 16), 30), ((20, 24, 28), 45), ((4, 3, 2), 5)])
def test_graph_matches_oracle(shape, n):
    nz, ny, nx = shape
    q = 16
    L = np.array([nx, ny, nz]) * q
    rng = np.random.default_rng(11)
    seeds = np.stack([rng.integers(0, L[i], n) for i in range(3)], axis=1)
    ref_lab = M.voronoi_labels(shape, seeds, q)
    adj, vol = cp.micro_graph(torch.from_numpy(ref_lab).cuda(), n)
    bits = adj.cpu().numpy().view(np.uint32)
    A = np.array([[(bits[g, m >> 5] >> (m & 31)) & 1 for m in range(n)] for g in range(n)], bool)
    ref_adj, ref_vol = M.grain_graph(ref_lab, n)
    assert np.array_equal(A, ref_adj)
    assert np.array_equal(vol.cpu().numpy(), ref_vol)


def test_slabs_match_oracle():
    shape, q, n = (20, 24, 28), 16, 12
    nz, ny, nx = shape
    L = np.array([nx, ny, nz]) * q
    rng = np.random.default_rng(13)
    seeds = np.stack([rng.integers(0, L[i], n) for i in range(3)], axis=1)
    lab = M.voronoi_labels(shape, seeds, q)
    slab_of = np.full(n, -1, np.int32)
    slabs, ref = [], lab.ravel().copy()
    for j, g in enumerate([0, 3, 4, 7, 11]):
        v = rng.standard_normal(3)
        nrm = v / np.linalg.norm(v)
        x0 = rng.uniform(-50, 500, 3)
        half = float(rng.uniform(5, 60))
        slab_of[g] = j
        xw = M.wrap_point(x0, L.astype(float))
        slabs.append([*nrm, *xw, half, n + j])
        ref[M.slab_members(lab, g, nrm, x0, half, q)] = n + j
    out = cp.micro_slabs(torch.from_numpy(lab.copy()).cuda(), q, n, torch.from_numpy(slab_of).cuda(),
                         torch.tensor(slabs, dtype=torch.float64).cuda())
    assert np.array_equal(out.cpu().numpy().ravel(), ref)


def _slab_band(m_ref, base, p):
    """Voxels whose slab decision lies within 1e-9 of its edge (where the
    two sides' rounding of the slab geometry may differ)."""
    band = np.zeros(base.size, bool)
    nz, ny, nx = p.shape
    L = np.array([nx, ny, nz], float) * p.q
    c = M.voxel_centres(p.shape, p.q).astype(float)
    for g, child, a, half, n, x0 in m_ref.inclusions:
        idx = np.nonzero(base.ravel() == g)[0]
        d = c[idx] - M.wrap_point(x0, L)
        d = np.where(d > L / 2, d - L, np.where(d < -L / 2, d + L, d))
        t = np.abs(d @ n)
        band[idx[np.abs(t - half) < 1e-9 * L.max()]] = True
    return band


@pytest.mark.parametrize("p_neigh,p_incl,seed", [(1.0, 0.0, 11), (0.0, 1.0, 11), (0.0, 0.0, 5), (1.0, 0.5, 21)])
def test_generate_matches_oracle(p_neigh, p_incl, seed):
    print("case", p_neigh, p_incl, seed, flush=True)
    p = M.Params(shape=(24, 28, 32), lam=45 / (24 * 28 * 32), r=2.5, p_neigh=p_neigh, p_incl=p_incl,
                 delta=(0.2, 0.4), theta=THETA, seed=seed)
    ref = M.generate(p)
    g = cp.generate_microstructure(p.shape, p.lam, p.r, p_neigh, p_incl, p.delta, THETA, seed, p.q)
    assert g["n_primary"] == ref.n_primary
    assert g["n_grains"] == ref.seeds.shape[0]
    assert g["n_neigh_drawn"] == ref.n_neigh_drawn
    assert g["draws"] == ref.draws
    assert [tuple(r) for r in g["pairs"]] == [tuple(r) for r in ref.pairs]
    assert g["n_inclusions"] == len(ref.inclusions) and g["n_labels"] == ref.rotations.shape[0]
    assert np.abs(g["rotations"] - ref.rotations).max() < 1e-12
    Q = rvegen.bunge_to_matrix(g["euler"])
    assert np.abs(Q - ref.rotations).max() < 1e-9
    lab = g["labels"].cpu().numpy().ravel()
    base = M.voronoi_labels(p.shape, ref.seeds, p.q)
    bad = lab != ref.labels.ravel()
    assert not np.any(bad & ~_slab_band(ref, base, p)), int(bad.sum())


def test_generated_rve_solves():
    """A generated twinned RVE goes straight into the solver (Bunge angles
    from the generator): two load steps converge."""
    shape = (32, 32, 32)
    g = cp.generate_microstructure(shape, 60 / 32 ** 3, 2.0, 1.0, 0.5, (0.1, 0.3), THETA, 4)
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    prob = cp.Problem(g["labels"].cpu().numpy(), g["euler"], C, S.n_miller, S.l_miller, S.family, S.tau0, law)
    R = cp.Solver(prob, precision="fp32", tol=1e-5, stag_tol=1e-4).run(rvegen.uniaxial_path(0.004, 2))
    assert np.all(R["status"] == 0) and R["Sigma"][-1, 0] > 0


def test_micro_argument_errors():
    with pytest.raises(cp.CpfError):
        cp.generate_microstructure((8, 8, 8), 1e-2, 1.0, p_neigh=1.5)
    with pytest.raises(cp.CpfError):
        cp.generate_microstructure((8, 8, 8), 1e-2, 1.0, q=3)
    with pytest.raises(cp.CpfError):
        cp.generate_microstructure((8, 8, 8), 0.0, 1.0)         # no generator at all
