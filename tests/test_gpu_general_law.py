"""The general law path (run-time Schmid tensors and stiffness: any system
set that is not the Table 1 set in its order) against the oracle: the
local law alone and whole solves, with the twin systems interleaved among
the slip systems (family from the mask), and with 24 systems (the largest
instantiation, 32 systems, whose FP64 x pass must fit the LDS of a
block)."""
import numpy as np
import pytest

import oracle
import rvegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
cp = pytest.importorskip("paper_2402_09996_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cp._lib.lib()
    yield


def _relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _systems(kind):
    """'interleaved': the 16 Table 1 systems with the twins moved among the
    slip systems; 'many': Table 1 plus 8 random slip systems (24)."""
    S = rvegen.config_systems(True)
    if kind == "interleaved":
        order = [12, 0, 1, 13, 2, 3, 4, 14, 5, 6, 7, 8, 15, 9, 10, 11]
        return rvegen.SystemSet(S.n_miller[order], S.l_miller[order], S.family[order],
                                [S.kind[i] for i in order], S.tau0[order])
    rng = np.random.default_rng(5)
    n = rng.standard_normal((8, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    l = rng.standard_normal((8, 3))
    l -= np.sum(l * n, axis=1, keepdims=True) * n
    return rvegen.SystemSet(np.vstack([S.n_miller, n]), np.vstack([S.l_miller, l]),
                            np.concatenate([S.family, np.zeros(8, np.int32)]), S.kind + ["o"] * 8,
                            np.concatenate([S.tau0, np.full(8, 90.0)]))


def _wl(shape, kind, steps=3, strain_per_step=1e-3):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve(shape, 5, 31, twin_share=0.5)
    return rvegen.Workload("general", rve, _systems(kind), C, law,
                           rvegen.uniaxial_path(strain_per_step * steps, steps))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["interleaved", "many"])
def test_general_local_law_matches_oracle(kind, precision):
    print("case", kind, precision, flush=True)
    shape = (8, 8, 16)
    w = _wl(shape, kind)
    S = w.systems.family.shape[0]
    s = cp.Solver(cp.Problem.from_workload(w), precision=precision)
    rng = np.random.default_rng(9)
    nv = int(np.prod(shape))
    e0 = rng.standard_normal((nv, 6)) * 1e-3
    e1 = e0 + rng.standard_normal((nv, 6)) * 4e-4
    ep = rng.standard_normal((nv, 6)) * 2e-4
    ep[:, :3] -= ep[:, :3].mean(axis=1, keepdims=True)
    v = rng.random((nv, S)) * 2e-3
    al = rng.standard_normal((nv, S)) * 1e-3
    dt, M = 0.4, 8
    mat = oracle.Material(w.rve.euler, w.C, w.systems.n_miller, w.systems.l_miller, w.systems.family,
                          w.systems.tau0, w.law)
    y1, sig = mat.update(w.rve.labels.ravel(), oracle.to_mandel(e0), oracle.to_mandel(e1),
                         np.hstack([oracle.to_mandel(ep), v, al]), dt, M)
    assert (np.abs(y1[:, 6:6 + S] - v).max(axis=1) > 0).mean() > 0.5     # plastic

    def grid(a):
        return torch.from_numpy(np.ascontiguousarray(a.T.reshape((a.shape[1],) + shape)))

    st1, sg = s.constitutive(grid(e0), grid(e1), grid(np.hstack([ep, v, al])), dt, M)
    st1 = st1.cpu().numpy().reshape(6 + 2 * S, nv).T
    sg = sg.cpu().numpy().reshape(6, nv).T
    tol = 1e-11 if precision == "fp64" else 2e-5
    assert _relerr(sg, oracle.from_mandel(sig)) < tol
    assert _relerr(st1[:, :6], oracle.from_mandel(y1[:, :6])) < tol * 10
    assert _relerr(st1[:, 6:], y1[:, 6:]) < tol * 10


@pytest.mark.parametrize("kind", ["interleaved", "many"])
def test_general_solve_fp64_parity(kind):
    print("case", kind, flush=True)
    w = _wl((6, 8, 12), kind)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-12)).run(w.path, keep_fields=True)
    assert np.all(R["status"] == 0)
    assert _relerr(R["Sigma"], ref.Sigma) < 1e-10
    assert _relerr(R["mean_v"], ref.mean_v) < 1e-9
    assert np.array_equal(R["iters"], ref.iters), (R["iters"], ref.iters)
    for name in ("stress", "plastic_strain", "acc_slip"):
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-10, name
    assert ref.mean_v[-1] > 0


def test_general_many_systems_fp32_against_fp64_oracle():
    w = _wl((8, 8, 16), "many", steps=4)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp32", tol=1e-6, stag_tol=1e-4)
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-10)).run(w.path)
    assert np.all(R["status"] == 0)
    assert np.abs(R["Sigma"][:, 0] - ref.Sigma[:, 0]).max() / np.abs(ref.Sigma[:, 0]).max() < 1e-4
