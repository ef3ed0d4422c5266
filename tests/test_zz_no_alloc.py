"""The allocation-free histogram entry point (cpf_seq_histogram_field, its
counts in the library's fixed device array) gives, count for count, what
cpf_seq_histogram gives for the same committed stress, on two calls in a
row with the second on a smaller field (the array keeps the first call's
contents), in both precisions; an empty field gives zero counts."""
import numpy as np
import pytest

import rvegen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
cp = pytest.importorskip("paper_2402_09996_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cp._lib.lib()
    yield


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_histogram_field_equals_solver_histogram(precision):
    C, law = rvegen.config_law()
    S = rvegen.config_systems(True)
    path = rvegen.uniaxial_path(0.008, 6)
    # member 0 larger than member 1: the second call sees a smaller input
    wl = [rvegen.Workload("nh%d" % i, rvegen.make_rve(sh, 6, 70 + i, twin_share=0.5), S, C, law, path)
          for i, sh in enumerate([(16, 24, 32), (8, 12, 16)])]
    kw = dict(tol=1e-10 if precision == "fp64" else 1e-6, stag_tol=0.0 if precision == "fp64" else 1e-4)
    s = cp.Solver([cp.Problem.from_workload(w) for w in wl], precision=precision, **kw)
    for n in range(path.n_steps):
        out = s.step_batch(path, n)
    assert all(o["mean_v"] > 0 for o in out)
    for nb, span in ((4096, 1.0), (37, 0.5)):
        for i in range(2):
            f = s.field_of(i, "stress")
            seq = torch.sqrt(1.5 * ((f[:3] - f[:3].mean(0)) ** 2).sum(0) + 3.0 * (f[3:] ** 2).sum(0))
            lo, hi = float(seq.min()) * (1 - 0.1 * span), float(seq.max()) * (1 + 0.1 * span)
            print("precision", precision, "member", i, "voxels", f[0].numel(), "bins", nb, flush=True)
            got = cp.von_mises_histogram_field(f.reshape(6, -1), nb, lo, hi)
            ref = s.von_mises_histogram(nb, lo, hi, rve=i)
            assert int(ref.sum()) == f[0].numel()
            assert np.array_equal(got, ref)
    torch.cuda.synchronize()


def test_histogram_field_of_an_empty_field():
    empty = torch.empty((6, 0), dtype=torch.float64, device="cuda:0")
    got = cp.von_mises_histogram_field(empty, 10, 0.0, 1.0)
    assert got.shape == (12,) and not got.any()
