"""The continuous Green operator applied at Nyquist frequencies too
(nyquist='formula') on the device, through the C-ABI, against the oracle:
the operator alone (the real part of the inverse of the formula at every
nonzero frequency), whole solves (FP64 to 1e-10 with the same iteration
counts), a batch of uneven members against solo solves, the
vector-Jacobian product, and the option checks."""
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


def _wl(shape, grains, seed, twins=False, steps=3, strain_per_step=5e-4):
    C, law = rvegen.config_law()
    rve = rvegen.make_rve(shape, grains, seed, twin_share=0.5 if twins else 0.0)
    S = rvegen.config_systems(with_twins=twins)
    return rvegen.Workload("nyq", rve, S, C, law, rvegen.uniaxial_path(strain_per_step * steps, steps))


def _relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 16, 24), (6, 18, 32), (4, 2, 3), (9, 6, 27), (64, 128, 256)])
def test_green_operator_matches_oracle(shape, precision):
    print("case formula", shape, precision, flush=True)
    w = _wl(shape, 3, 6)
    s = cp.Solver(cp.Problem.from_workload(w), precision=precision, nyquist="formula")
    lam0, mu0 = oracle.reference_medium(w.C)
    f = np.random.default_rng(2).standard_normal((6,) + shape) * 100.0
    full = oracle.fft3(f)
    xi, ctrl = oracle.frequency_directions(shape, "formula")
    ref = oracle.ifft3_real(oracle.gamma0_apply(full, lam0, mu0, xi, ctrl))
    ref_err2 = oracle.equilibrium_sums(full, xi, ctrl)
    out, err2 = s.green(torch.from_numpy(full[..., : shape[2] // 2 + 1]))
    tol = 1e-13 if precision == "fp64" else 3e-6
    assert _relerr(out.cpu().numpy(), ref) < tol
    assert err2 == pytest.approx(ref_err2, rel=tol * 10)
    if shape[2] % 2 == 0:
        xz, cz = oracle.frequency_directions(shape, "zero")
        assert _relerr(oracle.ifft3_real(oracle.gamma0_apply(full, lam0, mu0, xz, cz)), ref) > 1e-6


@pytest.mark.parametrize("shape,twins", [((6, 12, 18), True), ((8, 8, 8), False), ((6, 8, 9), True)])
def test_solve_fp64_parity(shape, twins):
    """tol 1e-5: with the formula at Nyquist frequencies the fixed point
    contracts far more slowly (hundreds of iterations per load step here
    against tens with the default), so the tolerance is kept loose; the
    iterates are compared to 1e-10 all the same."""
    print("case formula solve", shape, twins, flush=True)
    w = _wl(shape, 5, 21, twins=twins, steps=3, strain_per_step=1e-3)
    gs = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-5, nyquist="formula")
    R = gs.run(w.path)
    ref = oracle.solver_for(w, oracle.Options(tol=1e-5, nyquist="formula")).run(w.path, keep_fields=True)
    assert np.all(R["status"] == 0)
    for k in ("Sigma", "E", "mean_sig_eq", "mean_v"):
        assert _relerr(R[k], getattr(ref, k)) < 1e-10, k
    assert np.array_equal(R["iters"], ref.iters), (R["iters"], ref.iters)
    for name in ("stress", "strain", "plastic_strain", "acc_slip"):
        assert _relerr(gs.field(name).cpu().numpy(), ref.fields[name]) < 1e-10, name
    assert ref.mean_v[-1] > 0
    z = oracle.solver_for(w, oracle.Options(tol=1e-5)).run(w.path)
    assert ref.iters.sum() > 2 * z.iters.sum()


def test_batch_members_match_solo_solves():
    """Uneven members (even and odd nx) in one batch give their solo results."""
    ws = [_wl((8, 8, 8), 4, 3, twins=True, steps=3, strain_per_step=1e-3),
          _wl((6, 8, 9), 5, 4, twins=True, steps=3, strain_per_step=1e-3)]
    probs = [cp.Problem.from_workload(x) for x in ws]
    b = cp.Solver(probs, precision="fp64", tol=1e-7, nyquist="formula")
    outs = [[] for _ in ws]
    for n in range(ws[0].path.n_steps):
        for i, o in enumerate(b.step_batch(ws[0].path, n)):
            outs[i].append(o["Sigma"])
    for i, p in enumerate(probs):
        Rs = cp.Solver(p, precision="fp64", tol=1e-7, nyquist="formula").run(ws[0].path)
        assert _relerr(np.array(outs[i]), Rs["Sigma"]) < 1e-12


def test_vjp_matches_oracle():
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    rve = rvegen.make_rve((4, 4, 6), 3, 77, twin_share=0.5)
    path = rvegen.uniaxial_path(0.006, 3, rate=1e-2)
    w = rvegen.Workload("adj", rve, S, C, law, path)
    sb = np.random.default_rng(3).standard_normal((3, 6))
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp64", tol=1e-12, max_iter=3000, nyquist="formula")
    g, sig = s.vjp(path, sb, checkpoint_every=2, adj_tol=1e-12)
    go, so = oracle.solver_for(w, oracle.Options(tol=1e-12, max_iter=3000, nyquist="formula")).vjp(
        path, sb, adj_tol=1e-12)
    assert np.abs(sig - so).max() <= 1e-10 * np.abs(so).max()
    for f in (0, 1):
        assert np.abs(g[f] - go[f]).max() <= 1e-9 * np.abs(go[f]).max(), (f, g[f], go[f])


def test_nyquist_option_is_checked():
    w = _wl((4, 4, 4), 2, 1)
    with pytest.raises(ValueError):
        cp.Solver(cp.Problem.from_workload(w), nyquist="keep")
    with pytest.raises(cp.CpfError):
        cp.Solver(cp.Problem.from_workload(w), nyquist="formula", green="rotated")
