"""Write the oracle's expected values for the full-size parity tests.

Every value stored here comes from ``oracle/`` (FP64) on inputs from
``rvegen`` (seeded); nothing is read from the device path.  The runs take
tens of minutes to hours on a few CPU cores, so their results are kept as
``.npz`` files beside this script:

* ``cfg1_64cube_oracle.npz``: the 64^3 fully twinned RVE (100 grains, 12
  slip + 4 twin systems), uniaxial tension to 2 % in 50 load steps, tol
  1e-8: per-step mean stress and strain, the Section 5 averages, iteration
  counts, and the local stress, strain, plastic strain, accumulated slip
  and back strain of 4096 seeded voxels after the last step.
* ``cfg2_128cube_oracle.npz``: the 128^3 half-twinned RVE (500 grains), the
  first 8 of its 100 load steps (tension to 2 %), tol 1e-8: the same
  per-step values and 4096 sampled voxels after step 8.
* ``cfg4_64cube_adjoint_oracle.npz``: the 64^3 RVE of cfg1 over the first
  5 of its 50 load steps, forward and adjoint tol 1e-12: the loss
  L = sum_n (Sigma_11,n - target_n)^2 against a target curve solved with
  the 14 law parameters perturbed by factors 1 + 0.05 u (u uniform in
  [-1, 1], seeded), and its gradient by the oracle's discrete adjoint.

Usage: python tests/golden/make_goldens.py cfg1|cfg2|cfg4 ...
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import rvegen  # noqa: E402

N_SAMPLE = 4096
SAMPLE_SEED = 20240415
THETA_SEED = 20240419


def sample_indices(nvox, k=N_SAMPLE, seed=SAMPLE_SEED):
    """Sorted distinct voxel indices (x fastest), seeded."""
    return np.sort(np.random.default_rng(seed).choice(nvox, size=k, replace=False))


def _solve(w, tol, n_steps, tag):
    s = oracle.solver_for(w, oracle.Options(tol=tol))
    p = w.path
    out = {k: [] for k in ("Sigma", "E", "sig_eq_of_mean", "mean_sig_eq", "mean_v", "mean_f", "iters",
                           "err_eq", "err_bc")}
    t0 = time.time()
    for n in range(n_steps):
        its, ee, eb = s.step(p.t[n], p.t[n + 1], p.strain_ctrl[n], p.target[n])
        a, b, c, d = s.outputs()
        for k, v in (("Sigma", s.Sigma.copy()), ("E", s.E.copy()), ("sig_eq_of_mean", a), ("mean_sig_eq", b),
                     ("mean_v", c), ("mean_f", d), ("iters", its), ("err_eq", ee), ("err_bc", eb)):
            out[k].append(v)
        print("%s step %d/%d: %d iterations, Sigma_11 %.9g, %.0f s" % (tag, n + 1, n_steps, its, s.Sigma[0],
                                                                      time.time() - t0), flush=True)
    res = {k: np.asarray(v) for k, v in out.items()}
    f = s.fields()
    idx = sample_indices(s.n_vox)
    for name in ("stress", "strain", "plastic_strain", "acc_slip", "back_strain"):
        res["sample_" + name] = f[name].reshape(f[name].shape[0], -1)[:, idx].copy()
    res["sample_index"] = idx
    res["tol"] = np.float64(tol)
    res["n_steps"] = np.int64(n_steps)
    return res


def cfg1():
    w = rvegen.workload(1)
    res = _solve(w, 1e-8, w.path.n_steps, "cfg1")
    np.savez(os.path.join(HERE, "cfg1_64cube_oracle.npz"), **res)


def cfg2():
    w = rvegen.workload(2)
    res = _solve(w, 1e-8, 8, "cfg2")
    np.savez(os.path.join(HERE, "cfg2_128cube_oracle.npz"), **res)


THETA_KEYS = ("Q", "b", "c", "d", "K", "n")


def theta_of(w):
    """[2][7] = (r0, Q, b, c, d, K, n) of the slip and twin families."""
    S = w.systems
    rows = []
    for f, fam in ((0, w.law.slip), (1, w.law.twin)):
        rows.append([float(S.tau0[S.family == f][0])] + [float(getattr(fam, k)) for k in THETA_KEYS])
    return np.array(rows)


def with_params(w, th):
    """A copy of workload w with the family parameters th[2][7]."""
    import copy
    w2 = copy.deepcopy(w)
    S = w2.systems
    S.tau0 = np.where(S.family == 0, th[0, 0], th[1, 0]).astype(np.float64)
    for f, fam in ((0, w2.law.slip), (1, w2.law.twin)):
        for j, k in enumerate(THETA_KEYS):
            setattr(fam, k, float(th[f, 1 + j]))
    return w2


def cfg4(n_steps=5):
    w = rvegen.workload(4)
    th = theta_of(w)
    u = np.random.default_rng(THETA_SEED).uniform(-1.0, 1.0, size=th.shape)
    thp = th * (1.0 + 0.05 * u)
    t0 = time.time()
    sp = oracle.solver_for(with_params(w, thp), oracle.Options(tol=1e-12))
    Rp = sp.run(w.path, n_steps=n_steps)
    target = Rp.Sigma[:, 0].copy()
    print("cfg4 target", target, "%.0f s" % (time.time() - t0), flush=True)
    so = oracle.solver_for(w, oracle.Options(tol=1e-12))
    L, g, sxx = so.gradient(w.path, target, adj_tol=1e-12, n_steps=n_steps)
    print("cfg4 loss", L, "grad", g, "%.0f s" % (time.time() - t0), flush=True)
    np.savez(os.path.join(HERE, "cfg4_64cube_adjoint_oracle.npz"), theta=th, theta_target=thp, target=target,
             loss=np.float64(L), grad=g, sigma_xx=sxx, n_steps=np.int64(n_steps),
             target_iters=Rp.iters, adj_iters=np.asarray(so.adj_iters))


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cfg2", "cfg4", "cfg1"]:
        {"cfg1": cfg1, "cfg2": cfg2, "cfg4": cfg4}[name]()
