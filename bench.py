"""Benchmark: voxel-iterations/s of the Green-operator FFT solver on the
128^3 twinned synthetic RVE (500 grains, half of them split into twin
pairs, 750 labels, 12 slip + 4 twin systems, uniaxial tension at 1e-3/s to
2% in 100 load steps).

One bench "step" is one load step: the whole fixed-point iteration (local
law, forward FFT, Green operator with residual, inverse FFT, mixed
boundary update) repeated to convergence.  W warmup steps run from the
undeformed state, the solver is reset, and K steps are timed from t = 0
along the path (extended at the same rate if K > 100).

Prints one JSON line.  FP32 bulk with FP64 reductions is the headline; the
plain FP64 solve of the same steps is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iterations/s @128^3 twinned RVE; batched-FP32 & adjoint speedup vs FP64"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


# HBM bytes per launch of the x pass (the dominant kernel) at 128^3 FP32,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB copy (factors
# 0.5 and 1.0); valid only for the library sources they were taken on.
XPASS_TRAFFIC = {"src": "feb78cbf0f56681f", "read_bytes": 479.4e6, "write_bytes": 420.4e6}


def library_source_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2402_09996_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def law_flops(S: int, n_twin: int, M: int, nvox: int, n_active: float, n_newton: float) -> float:
    """Algorithmic FLOPs of one local-law evaluation of the whole grid
    (FMA = 2 flops, every other arithmetic op or transcendental = 1); the
    breakdown is documented with the kernel."""
    per_rate = 114 + 51 * S + 2 * n_twin
    per_active = 10
    per_newton = 16
    per_voxel_fixed = 450 + 12 + 30          # frame rotations, strain update, sums
    return nvox * (4 * M * per_rate + per_voxel_fixed) + n_active * per_active + n_newton * per_newton


def fft_pass_bytes(nx: int, ny: int, nz: int, rbytes: int) -> float:
    """Algorithmic HBM bytes of one y or z pass: read + write of the
    6-component half spectrum as the solve stores it (kx < nx/2; the Nyquist
    column is zero under the Green operator)."""
    return 2.0 * 6 * nz * ny * (nx // 2) * 2 * rbytes


def run_mode(cp, w, precision, K, W, tol, stag, green="continuous", timing=True):
    """K timed load steps after W warm-up steps.  timing: True (HIP events
    around every kernel) or "xpass" (around the x pass only: two events per
    iteration instead of ten, the least disturbance of a timed run)."""
    import torch
    prob = cp.Problem.from_workload(w)
    s = cp.Solver(prob, precision=precision, tol=tol, stag_tol=stag, green=green)
    for n in range(W):
        s.step(w.path, n)
    s.reset()
    s.set_timing(timing)
    torch.cuda.synchronize()
    iters, act, newt, outs = 0, 0.0, 0.0, []
    t0 = time.perf_counter()
    for n in range(K):
        o = s.step(w.path, n)
        iters += int(o["iters"])
        act += float(o["n_active"])
        newt += float(o["n_newton"])
        outs.append(o)
        print("[bench] %s %s step %d iters %d Sigma_xx %.4f err %.2e" %
              (precision, green, n, o["iters"], o["Sigma"][0], max(o["err_eq"], o["err_bc"])),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = s.timing()
    return s, dict(iters=iters, wall=wall, n_active=act, n_newton=newt, kernels=tm, outs=outs)


def cpu_baseline(w, s32, K, budget_s):
    """The oracle timed on the host on a bounded sample of the same
    workload: a few fixed-point iterations of the load step that follows the
    timed run, starting from the GPU's committed state."""
    import numpy as np
    import oracle
    nz, ny, nx = w.rve.labels.shape
    o = oracle.solver_for(w, oracle.Options(tol=1e-8, max_iter=1))
    f = {k: s32.field(k).double().cpu().numpy() for k in
         ("strain", "plastic_strain", "acc_slip", "back_strain", "stress")}
    pm = lambda a: a.reshape(a.shape[0], -1).T.copy()
    o.eps = oracle.to_mandel(pm(f["strain"]))
    o.y = np.hstack([oracle.to_mandel(pm(f["plastic_strain"])), pm(f["acc_slip"]),
                     pm(f["back_strain"])])
    o.sig = oracle.to_mandel(pm(f["stress"]))
    o.Sigma = f["stress"].reshape(6, -1).mean(axis=1)
    o.E = f["strain"].reshape(6, -1).mean(axis=1)
    n = min(K, w.path.n_steps - 1)
    state = (o.eps.copy(), o.y.copy(), o.sig.copy(), o.Sigma.copy(), o.E.copy())

    def sample(limit_s, max_its):
        o.eps, o.y, o.sig, o.Sigma, o.E = (a.copy() for a in state)
        its, t_used = 0, 0.0
        while its < max_its and (its == 0 or t_used < limit_s):
            t0 = time.perf_counter()
            try:
                o.step(w.path.t[n], w.path.t[n + 1], w.path.strain_ctrl[n], w.path.target[n])
            except oracle.NotConverged:
                pass
            t_used += time.perf_counter() - t0
            its += 1
            print("[bench] oracle iteration %d (%d threads): %.2f s" % (its, oracle.threads(), t_used),
                  file=sys.stderr, flush=True)
        return its, t_used

    cores = oracle.threads()
    its, t_used = sample(budget_s, 20)
    oracle.set_threads(1)
    its1, t1 = sample(0.0, 1)
    oracle.set_threads(cores)
    return {"value": its * nx * ny * nz / t_used, "unit": "voxel-iterations/s",
            "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d fixed-point iteration(s) of load step %d of the same 128^3 workload "
                      "(FP64 oracle, from the GPU's committed state), %.1f s" % (its, n, t_used),
            "single_thread": {"value": its1 * nx * ny * nz / t1, "unit": "voxel-iterations/s",
                              "cores": 1, "sample": "1 fixed-point iteration from the same state "
                              "(the oracle's C law on one thread; numpy's FFTs are single-threaded "
                              "in both figures), %.1f s" % t1}}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def batch_leg(cp, steps, ref_tol=1e-10):
    """Workload 3: 32 RVEs of uneven sizes (32^3..96^3), half twinned, the
    same law, 2% tension in 50 steps (the first `steps` steps are run).
    The FP32 batched solve (one launch per pass for all members, adaptive
    graph replays: normally one replay and one host poll per load step,
    autotuned tiles; tol 1e-6 with the stalled-residual acceptance below
    1e-4) against the sum of 32 plain FP64 single-RVE solves (direct
    launches) at the same tolerance 1e-6.  Accuracy: both against tight
    FP64 solves (tol ref_tol) of one member of each grid size, as the
    largest relative error of the mean stress over the steps."""
    import numpy as np
    import torch
    import rvegen
    C, law = rvegen.config_law()
    S = rvegen.config_systems(with_twins=True)
    members = rvegen.batch_members(32)
    path = rvegen.uniaxial_path(0.02 / 50 * steps, steps)
    probs = [cp.Problem(m.labels, m.euler, C, S.n_miller, S.l_miller, S.family, S.tau0, law)
             for m in members]
    nvox = sum(int(m.labels.size) for m in members)
    b = cp.Solver(probs, precision="fp32", tol=1e-6, stag_tol=1e-4, graph_iters="adaptive", autotune=True)
    b.step_batch(path, 0)          # warm-up: graph capture, first launches
    b.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, it32, syncs, stag = [], 0, [], 0
    for n in range(steps):
        o = b.step_batch(path, n)
        outs.append(o)
        it32 += sum(int(x["iters"]) * int(m.labels.size) for x, m in zip(o, members))
        syncs.append(int(o[0]["host_syncs"]))
        stag += sum(int(x["stagnated"]) for x in o)
        print("[bench] batch fp32 step %d: max iters %d, host polls %d" % (n, max(x["iters"] for x in o),
                                                                           syncs[-1]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    sig32 = np.array([[outs[n][j]["Sigma"] for n in range(steps)] for j in range(len(members))])

    def single(j, tol):
        s = cp.Solver(probs[j], precision="fp64", tol=tol)
        s.step(path, 0)
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.run(path)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    t64, it64, sig64 = 0.0, 0, []
    for j in range(len(members)):
        t, r = single(j, 1e-6)
        t64 += t
        it64 += int(r["iters"].sum()) * int(members[j].labels.size)
        sig64.append(r["Sigma"])
        print("[bench] fp64 single RVE %d (%d^3) at tol 1e-6 done, %.2f s so far" %
              (j, members[j].labels.shape[0], t64), file=sys.stderr, flush=True)
    sig64 = np.array(sig64)
    sizes = sorted(set(int(m.labels.shape[0]) for m in members))
    picks = [next(i for i, m in enumerate(members) if m.labels.shape[0] == n) for n in sizes]
    e32, e64 = 0.0, 0.0
    for j in picks:
        _, r = single(j, ref_tol)
        ref = r["Sigma"]
        scale = np.abs(ref[:, 0]).max()
        e32 = max(e32, float(np.abs(sig32[j] - ref).max() / scale))
        e64 = max(e64, float(np.abs(sig64[j] - ref).max() / scale))
    return {"workload": "32 RVEs, N in {32,48,64,96}^3, 50-300 grains, even members twinned, "
                        "2%%/50-step tension (%d steps)" % steps,
            "rves": len(members), "voxels": nvox, "grid_sizes": sizes, "steps": steps,
            "graph": "adaptive", "host_polls_per_step": {"mean": float(np.mean(syncs)), "max": int(max(syncs)),
                                                         "first_step": syncs[0]},
            "stalled_acceptances": stag,
            "tiles": {str(n): b.tiles(j) for n, j in zip(sizes, picks)},
            "fp32_batched_s": t32, "fp64_single_sum_s": t64, "speedup": t64 / t32,
            "tol": {"fp32_batched": 1e-6, "fp64_single": 1e-6, "reference": ref_tol},
            "max_rel_err_Sigma_vs_reference": {"fp32_batched": e32, "fp64_single": e64,
                                              "members": picks},
            "fp32_batched_voxel_iterations_per_s": it32 / t32,
            "fp64_single_voxel_iterations_per_s": it64 / t64}


def adjoint_leg(cp, steps, checkpoint_every=10):
    """Workload 4: gradient of L = sum_n (Sigma_xx,n - target_n)^2 over 50
    load steps of the 64^3 fully twinned RVE with respect to the 14 law
    parameters.  The target curve comes from a forward solve with every
    parameter scaled by (1 + 0.05 u), u ~ U[-1, 1] (seeded).  Times the
    device adjoint (checkpoints every 10 steps) against one FP64 forward
    solve; central differences need 28 such solves."""
    import numpy as np
    import torch
    import rvegen
    w = rvegen.workload(4, steps_override=steps)
    base = cp.Problem.from_workload(w)
    theta = np.array([[80.0] + [getattr(w.law.slip, k) for k in ("Q", "b", "c", "d", "K", "n")],
                      [120.0] + [getattr(w.law.twin, k) for k in ("Q", "b", "c", "d", "K", "n")]])
    u = np.random.default_rng(20240219).uniform(-1.0, 1.0, theta.shape)
    tgt = cp.Solver(cp.with_theta(base, theta * (1 + 0.05 * u)), precision="fp64",
                    tol=1e-8).run(w.path)["Sigma"][:, 0]

    def forward(prob):
        s = cp.Solver(prob, precision="fp64", tol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.run(w.path)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    t_fwd, r = forward(base)
    nvox = int(w.rve.labels.size)
    print("[bench] adjoint leg: FP64 forward %.2f s, %d iterations" % (t_fwd, int(r["iters"].sum())),
          file=sys.stderr, flush=True)
    out = {"workload": "64^3 fully twinned RVE (100 grains, 12+4 systems), 2%% tension in %d steps; "
                       "14 law parameters; target from parameters x (1 + 0.05 u)" % steps,
           "checkpoint_every": checkpoint_every, "fp64_forward_s": t_fwd,
           "fp64_forward_iterations": int(r["iters"].sum())}
    for key, prec, tol, ck in (("fp64", "fp64", 1e-8, checkpoint_every), ("fp32", "fp32", 1e-6, checkpoint_every),
                               ("fp64_every_step_checkpoint", "fp64", 1e-8, 1)):
        s = cp.Solver(base, precision=prec, tol=tol, stag_tol=0.0 if prec == "fp64" else 1e-4)
        need = s.adjoint_workspace_size(w.path, ck)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, g, _ = s.gradient(w.path, tgt, checkpoint_every=ck, adj_tol=tol)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        print("[bench] adjoint %s: %.2f s, L %.6g" % (key, t_adj, L), file=sys.stderr, flush=True)
        out[key] = {"adjoint_s": t_adj, "loss": L, "grad": g.tolist(), "tol": tol, "checkpoint_every": ck,
                    "workspace_MB": need / 1e6, **s.adjoint_stats(),
                    "fd_over_adjoint": 28 * t_fwd / t_adj, "adjoint_over_forward": t_adj / t_fwd}
        del s
    g64 = np.array(out["fp64"]["grad"])
    out["fp32_vs_fp64_grad_max_rel"] = float(np.abs(np.array(out["fp32"]["grad"]) - g64).max()
                                             / np.abs(g64).max())
    # one central difference at full size (slip K) as a check of the gradient
    h = 1e-5 * theta[0, 5]
    tp, tm = theta.copy(), theta.copy()
    tp[0, 5] += h
    tm[0, 5] -= h
    Lp = float(np.sum((forward(cp.with_theta(base, tp))[1]["Sigma"][:, 0] - tgt) ** 2))
    Lm = float(np.sum((forward(cp.with_theta(base, tm))[1]["Sigma"][:, 0] - tgt) ** 2))
    fd = (Lp - Lm) / (2 * h)
    out["fd_check_slip_K"] = {"fd": fd, "adjoint": float(g64[0, 5])}
    out["fd_estimate_s"] = 28 * t_fwd
    # matched accuracy: the central differences (FP64 forward solves at the
    # same tolerance) agree with the adjoint to the relative error below on
    # the parameter checked; the adjoint is held to 1e-9 against the oracle's
    # discrete adjoint in the tests
    out["matched_accuracy"] = {
        "fd_vs_adjoint_rel_diff": abs(fd - float(g64[0, 5])) / abs(float(g64[0, 5])),
        "fd_over_adjoint_fp64": 28 * t_fwd / out["fp64"]["adjoint_s"],
        "fd_over_adjoint_fp64_checkpoint_every_step": 28 * t_fwd / out["fp64_every_step_checkpoint"]["adjoint_s"]}
    out["voxels"] = nvox
    return out


def green_leg(cp, w, KG, W, r32, K, nvox):
    """The same FP32 workload with the rotated-scheme Green operator:
    iterations, throughput and time per load step against the continuous
    operator's run (which stores 64 of the 65 kx columns of a 128^3 grid;
    the rotated operator needs all 65).  Both runs time every kernel."""
    import numpy as np
    s, r = run_mode(cp, w, "fp32", KG, W, 1e-6, 1e-4, green="rotated")
    kern = r["kernels"]
    it = max(1, r["iters"])
    out = {"steps": KG, "iterations": r["iters"], "value": r["iters"] * nvox / r["wall"],
           "unit": "voxel-iterations/s", "ms_per_step": r["wall"] / KG * 1e3,
           "kernel_avg_ms": {k: kern[k][0] / it for k in kern}}
    if KG == K:
        out["iterations_vs_continuous"] = r["iters"] / max(1, r32["iters"])
        out["wall_vs_continuous"] = r["wall"] / r32["wall"]
        a = np.array([o["Sigma"][0] for o in r["outs"]])
        b = np.array([o["Sigma"][0] for o in r32["outs"]])
        out["max_rel_diff_Sigma_xx_vs_continuous"] = float(np.abs(a - b).max() / np.abs(b).max())
    del s
    return out


def micro_leg(cp, n=256, grains=1920.0, r=5.0, reps=3):
    """The stochastic microstructure model at the paper's window: 256^3
    voxels, hard-core radius 5 voxels, 1920 expected grains (the primary
    intensity from the type II relation lambda_h = (1 - exp(-lambda V_r)) /
    V_r), the three twin configurations.  Wall time of a whole realization
    (host draws and twin logic included), and the device time of the
    Voronoi labelling alone (HIP events) for the same generator count."""
    import numpy as np
    import torch
    Vr = 4.0 / 3.0 * math.pi * r ** 3
    lam_h = grains / n ** 3
    lam_p = -math.log(1.0 - lam_h * Vr) / Vr
    theta = math.radians(69.79)
    out = {"grid": [n, n, n], "r_voxels": r, "expected_grains": grains, "primary_lambda": lam_p,
           "delta": [0.1, 0.3], "configs": {}}
    for name, pn, pi in (("neighbouring", 1.0, 0.0), ("inclusion", 0.0, 1.0), ("none", 0.0, 0.0)):
        best, g = None, None
        for k in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g = cp.generate_microstructure((n, n, n), lam_p, r, pn, pi, (0.1, 0.3), theta, 1000 + k)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out["configs"][name] = {"ms_per_realization": best * 1e3, "grains": g["n_grains"],
                                "pairs": g["n_pairs"], "inclusions": g["n_inclusions"],
                                "fallback_tiles": g["fallback_tiles"]}
    # the labelling kernel alone, same generator count, events on the stream it runs on
    q = 16
    ng = out["configs"]["none"]["grains"]
    rng = np.random.default_rng(5)
    pts = np.zeros((ng, 4), np.int32)
    pts[:, :3] = rng.integers(0, n * q, (ng, 3))
    seeds = torch.from_numpy(pts).cuda()
    cp.micro_label((n, n, n), q, seeds)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cp.micro_label((n, n, n), q, seeds)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    out["label_kernel"] = {"ms": ms, "voxels_per_s": n ** 3 / (ms * 1e-3), "generators": ng,
                           "label_write_GB/s": 4.0 * n ** 3 / (ms * 1e-3) / 1e9}
    return out


def paper_leg(cp, steps=100, configs=("neighbouring",), n=256, seed=7, axes=(0,), aa_depth=0):
    """The paper's parameter set (tetragonal stiffness, Table 1 with tau0
    130/200/130 MPa, twin-fraction law; b = 10, q = 1) on a generated 256^3
    realization (1920 expected grains, r = 5 voxels), FP32: uniaxial
    shortening along x (or y, z) to 0.5 % at 1e-3 /s in ``steps`` load
    steps (the paper uses 1000).  Per configuration and axis: load-step
    time, throughput and the von Mises stress of the mean stress at ten
    points of the curve."""
    import numpy as np
    import torch
    import rvegen
    Vr = 4.0 / 3.0 * math.pi * 5.0 ** 3
    lam_p = -math.log(1.0 - 1920.0 / n ** 3 * Vr) / Vr
    C, law = rvegen.paper_law()
    S = rvegen.table1_systems(True)
    out = {"grid": [n, n, n], "steps": steps, "total_strain": -0.005, "precision": "fp32",
           "anderson_depth": aa_depth, "configs": {}}
    for name, axis in [(c, a) for c in configs for a in axes]:
        path = rvegen.uniaxial_path(-0.005, steps, axis=axis)
        pn, pi = {"neighbouring": (1.0, 0.0), "inclusion": (0.0, 1.0), "none": (0.0, 0.0)}[name]
        g = cp.generate_microstructure((n, n, n), lam_p, 5.0, pn, pi, (0.1, 0.3), math.radians(69.79), seed)
        prob = cp.Problem(g["labels"].cpu().numpy(), g["euler"], C, S.n_miller, S.l_miller, S.family, S.tau0,
                          law)
        s = cp.Solver(prob, precision="fp32", tol=1e-6, stag_tol=1e-4, aa_depth=aa_depth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, seq = 0, []
        for k in range(steps):
            o = s.step(path, k)
            iters += int(o["iters"])
            seq.append(float(o["sig_eq_of_mean"]))
            if k % 10 == 9:
                print("[bench] paper %s axis %d step %d iters %d sigma_eq %.2f" % (name, axis, k, o["iters"],
                                                                                    seq[-1]),
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        pick = [int(round((j + 1) * steps / 10)) - 1 for j in range(10)]
        out["configs"][name + ("" if tuple(axes) == (0,) else "_" + "xyz"[axis])] = {
            "labels": int(g["n_labels"]), "pairs": int(g["n_pairs"]), "inclusions": int(g["n_inclusions"]),
            "iterations": iters, "ms_per_step": wall / steps * 1e3,
            "voxel_iterations_per_s": iters * n ** 3 / wall,
            "curve": [[0.5 * (j + 1) / 10, seq[k]] for j, k in enumerate(pick)],
            "final_mean_f": float(o["mean_f"]), "final_mean_v": float(o["mean_v"])}
        del s, prob, g
        torch.cuda.empty_cache()
    return out


def eta_leg(cp, etas=(1e2, 1e3, 2e3, 5e3, 1e4, 3e4, 1e5, 3e5, 1e6)):
    """Fig. 3 analogue: yield stress of a single-crystal material point (a
    one-orientation 2x2x2 RVE, Bunge (0.3, 0.7, 1.1)) against eta, FP64,
    paper parameter set, tension along x at 1e-3 /s to 0.5 % in 20 steps of
    one RK4 step each; yield at 0.02 % axial plastic strain.  Too small an
    eta diverges (reported as null)."""
    import numpy as np
    import rvegen
    out = {"steps": 20, "rk4_substeps": 1, "offset": 2e-4, "yield_MPa": {}}
    for eta in etas:
        C, law = rvegen.paper_law()
        law.eta = eta
        S = rvegen.table1_systems(True)
        prob = cp.Problem(np.zeros((2, 2, 2), np.int32), np.array([[0.3, 0.7, 1.1]]), C, S.n_miller,
                          S.l_miller, S.family, S.tau0, law)
        try:
            R = cp.Solver(prob, precision="fp64", tol=1e-12, rk4_M=1).run(rvegen.uniaxial_path(0.005, 20))
        except cp.CpfError:
            out["yield_MPa"]["%g" % eta] = None
            continue
        E11, S11 = R["E"][:, 0], R["Sigma"][:, 0]
        ep = E11 - S11 / (S11[0] / E11[0])
        k = int(np.argmax(ep >= 2e-4))
        a = (2e-4 - ep[k - 1]) / (ep[k] - ep[k - 1])
        out["yield_MPa"]["%g" % eta] = float(S11[k - 1] + a * (S11[k] - S11[k - 1]))
    # the semi-quantitative check: ordinary system 3 at Schmid factor 1/2
    # (every other system a larger tau0 / m) should start to slip at 2 tau0
    # = 260 MPa; 100 steps of 0.005 % resolve the onset to 9 MPa
    S = rvegen.table1_systems(True)
    e = rvegen.schmid_half_orientation(S, 2)
    half = {"bunge": [float(x) for x in e], "steps": 100, "onset_bracket_MPa": {}, "yield_MPa": {}}
    for eta in (1e4, 1e5, 1e6):
        C, law = rvegen.paper_law()
        law.eta = eta
        prob = cp.Problem(np.zeros((2, 2, 2), np.int32), np.array([e]), C, S.n_miller, S.l_miller, S.family,
                          S.tau0, law)
        R = cp.Solver(prob, precision="fp64", tol=1e-12, rk4_M=1).run(rvegen.uniaxial_path(0.005, 100))
        E11, S11 = R["E"][:, 0], R["Sigma"][:, 0]
        k = int(np.argmax(R["mean_v"] > 0))
        half["onset_bracket_MPa"]["%g" % eta] = [float(S11[k - 1]), float(S11[k])]
        ep = E11 - S11 / (S11[0] / E11[0])
        j = int(np.argmax(ep >= 2e-4))
        a = (2e-4 - ep[j - 1]) / (ep[j] - ep[j - 1])
        half["yield_MPa"]["%g" % eta] = float(S11[j - 1] + a * (S11[j] - S11[j - 1]))
    out["schmid_half"] = half
    return out


def substeps_leg(cp, w, KS, r32, K, nvox, rk_tol=1e-8):
    """The same FP32 workload with frozen error-controlled substep counts
    (rk_tol on the state, Richardson's bound): iterations, time per load
    step, the mean substep count of the last step and the difference of
    Sigma_xx from the fixed-count run."""
    import numpy as np
    import torch
    prob = cp.Problem.from_workload(w)
    s = cp.Solver(prob, precision="fp32", tol=1e-6, stag_tol=1e-4, rk_tol=rk_tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, outs = 0, []
    for n in range(KS):
        o = s.step(w.path, n)
        iters += int(o["iters"])
        outs.append(o)
        if n % 10 == 9:
            print("[bench] substeps step %d iters %d Sigma_xx %.4f" % (n, o["iters"], o["Sigma"][0]),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts = s.field("substeps").double().cpu().numpy().ravel()
    out = {"rk_tol": rk_tol, "steps": KS, "iterations": iters, "ms_per_step": wall / KS * 1e3,
           "value": iters * nvox / wall, "unit": "voxel-iterations/s",
           "substeps_last_step": {"mean": float(counts.mean()), "max": float(counts.max()),
                                  "share_refined": float((counts > counts.min()).mean())}}
    if KS == K:
        a = np.array([o["Sigma"][0] for o in outs])
        b = np.array([o["Sigma"][0] for o in r32["outs"]])
        out["max_rel_diff_Sigma_xx_vs_fixed"] = float(np.abs(a - b).max() / np.abs(b).max())
        out["wall_vs_fixed"] = wall / r32["wall"]
    return out


def anderson_leg(cp, w, KA, r32, K, nvox, depth=4):
    """The same FP32 workload with the Anderson-accelerated fixed point:
    iterations, time per load step (the figure of merit here: the
    throughput per iteration drops by the extra passes) and the difference
    of Sigma_xx from the basic scheme's run."""
    import numpy as np
    import torch
    s = cp.Solver(cp.Problem.from_workload(w), precision="fp32", tol=1e-6, stag_tol=1e-4, aa_depth=depth)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, outs = 0, []
    for n in range(KA):
        o = s.step(w.path, n)
        iters += int(o["iters"])
        outs.append(o)
        if n % 10 == 9:
            print("[bench] anderson step %d iters %d Sigma_xx %.4f" % (n, o["iters"], o["Sigma"][0]),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"depth": depth, "steps": KA, "iterations": iters, "ms_per_step": wall / KA * 1e3,
           "value": iters * nvox / wall, "unit": "voxel-iterations/s"}
    if KA == K:
        a = np.array([o["Sigma"][0] for o in outs])
        b = np.array([o["Sigma"][0] for o in r32["outs"]])
        out["iterations_vs_basic"] = iters / max(1, r32["iters"])
        out["wall_vs_basic"] = wall / r32["wall"]
        out["max_rel_diff_Sigma_xx_vs_basic"] = float(np.abs(a - b).max() / np.abs(b).max())
    return out


def histogram_leg(s32, nvox, reps=20, nbins=150, lo=0.0, hi=1500.0):
    """Distribution of the local von Mises stress of the committed 128^3
    state (post-processing after the timed steps): the stress pass (reads
    strain, plastic strain, label; writes the stress into the spectrum
    area) and the histogram pass (reads it): 100 B per voxel in FP32."""
    import numpy as np
    import torch
    c = s32.von_mises_histogram(nbins, lo, hi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        c = s32.von_mises_histogram(nbins, lo, hi)
    dt = (time.perf_counter() - t0) / reps
    byts = 100.0 * nvox
    x = lo + (hi - lo) / nbins * (np.arange(nbins) + 0.5)
    inside = c[1:-1].astype(np.float64)
    return {"bins": nbins, "range_MPa": [lo, hi], "ms_per_call": dt * 1e3,
            "GB/s": byts / dt / 1e9, "algorithmic_bytes": byts,
            "below": int(c[0]), "above": int(c[-1]),
            "mode_MPa": float(x[int(np.argmax(inside))]) if inside.sum() else None}


def copy_probe(nbytes=1 << 30, reps=5):
    """Plain device-to-device copies of a known size: the reference for
    the FETCH_SIZE / WRITE_SIZE counters (bytes read and written per copy
    are both nbytes)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the second FP32 run that times every kernel")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--adjoint-steps", type=int, default=50)
    ap.add_argument("--no-micro", action="store_true", help="skip the microstructure generator leg")
    ap.add_argument("--micro-only", action="store_true", help="only run the microstructure generator leg")
    ap.add_argument("--paper-steps", type=int, default=100,
                    help="load steps of the paper-parameter 256^3 leg (0: skip)")
    ap.add_argument("--paper-configs", default="neighbouring",
                    help="twin configurations of that leg: comma list of none,neighbouring,inclusion or 'all'")
    ap.add_argument("--paper-only", action="store_true", help="only run the paper-parameter leg")
    ap.add_argument("--paper-axes", default="x", help="load axis of that leg: x or 'all' (x, y, z)")
    ap.add_argument("--paper-aa", type=int, default=0, help="Anderson depth of that leg (0: basic scheme)")
    ap.add_argument("--green-steps", type=int, default=None,
                    help="load steps of the rotated-operator FP32 leg (default: --steps)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run plain 1 GiB device copies (calibrates the HBM byte counters)")
    ap.add_argument("--only", choices=("batch", "adjoint"), default=None,
                    help="only run the batch or the adjoint leg")
    args = ap.parse_args()
    if args.only:
        import paper_2402_09996_amd as cp
        leg = batch_leg(cp, args.batch_steps) if args.only == "batch" else adjoint_leg(cp, args.adjoint_steps)
        print(json.dumps({{"batch": "batched", "adjoint": "adjoint"}[args.only]: leg}), flush=True)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.micro_only:
        import paper_2402_09996_amd as cp
        print(json.dumps({"microstructure": micro_leg(cp), "eta_sweep": eta_leg(cp)}), flush=True)
        return
    if args.paper_only:
        import paper_2402_09996_amd as cp
        cf = ("none", "neighbouring", "inclusion") if args.paper_configs == "all" else \
            tuple(args.paper_configs.split(","))
        ax = (0, 1, 2) if args.paper_axes == "all" else (0,)
        print(json.dumps({"paper_set": paper_leg(cp, args.paper_steps, cf, axes=ax, aa_depth=args.paper_aa)}),
              flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import rvegen
    import paper_2402_09996_amd as cp
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    K, W = args.steps, args.warmup
    K64 = args.fp64_steps if args.fp64_steps is not None else K
    nsteps = max(100, K, K64, W)
    w = rvegen.workload(2, steps_override=nsteps)
    nz, ny, nx = w.rve.labels.shape
    nvox = nx * ny * nz
    S = int(w.systems.family.shape[0])
    n_twin = int((w.systems.family == 1).sum())
    dt = w.path.t[1] - w.path.t[0]
    M = max(1, math.ceil(dt / 0.05 * (1 - 1e-12)))

    # headline: HIP events around the x pass only
    s32, r32 = run_mode(cp, w, "fp32", K, W, 1e-6, 1e-4, timing="xpass")
    value = r32["iters"] * nvox / r32["wall"]
    # the same steps again with every kernel timed: the per-kernel breakdown
    # (y and z pass rates) and the base of the rotated operator's comparison
    rk = None
    if not args.no_breakdown:
        sk, rk = run_mode(cp, w, "fp32", K, W, 1e-6, 1e-4, timing=True)
        del sk
    s64, r64 = (None, None)
    if K64 > 0:
        s64, r64 = run_mode(cp, w, "fp64", K64, min(W, 1), 1e-8, 0.0, timing="xpass")

    # dominant kernel (by the breakdown run when there is one)
    kern = rk["kernels"] if rk is not None else r32["kernels"]
    dom = max(kern, key=lambda k: kern[k][0])
    it = max(1, r32["iters"])
    if dom == "xpass_law":
        flops = law_flops(S, n_twin, M, nvox, r32["n_active"] / it, r32["n_newton"] / it)
        # the headline run's own events
        avg_s = r32["kernels"]["xpass_law"][0] / 1e3 / it
        ach = flops / avg_s / 1e12
        same = library_source_hash() == XPASS_TRAFFIC["src"] and (nz, ny, nx) == (128, 128, 128)
        traffic = XPASS_TRAFFIC["read_bytes"] + XPASS_TRAFFIC["write_bytes"] if same else None
        roof = {"bound": "alu", "kernel": "k_xpass_iter<float,16,1,false,false>", "achieved": ach,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "algorithmic_bytes": 428.0 * nvox, "avg_launch_ms": avg_s * 1e3,
                "flops_per_launch": flops}
    else:
        b = fft_pass_bytes(nx, ny, nz, 4)
        avg_s = kern[dom][0] / 1e3 / max(1, (rk or r32)["iters"])
        ach = b / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_ms": avg_s * 1e3}
    fft_gbs = {}
    for k in ("ypass_fwd", "zpass_green", "ypass_inv"):
        if kern[k][1] == 0:
            continue
        t = kern[k][0] / 1e3 / max(1, (rk or r32)["iters"])
        fft_gbs[k] = {"avg_ms": t * 1e3, "GB/s": fft_pass_bytes(nx, ny, nz, 4) / t / 1e9,
                      "frac_hbm": fft_pass_bytes(nx, ny, nz, 4) / t / 1e9 / HBM_PEAK_GBS}

    line = {
        "metric": METRIC, "value": value, "unit": "voxel-iterations/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": r32["wall"] / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name + " (FP32 bulk, FP64 reductions)", "grid": [nz, ny, nx],
                   "labels": int(w.rve.n_labels), "systems": S, "load_steps_timed": K,
                   "rk4_substeps": M, "tol": 1e-6, "global_batch": 1},
        "iterations": r32["iters"],
        "kernel_ms": {k: v[0] for k, v in kern.items() if v[1] > 0},
        "kernel_timing": ("x pass: HIP events of the timed run (x pass only); all kernels: a second run of "
                          "the same steps with every kernel timed" if rk is not None else
                          "HIP events of the timed run (x pass only)"),
        "fft_passes": fft_gbs,
        "roofline": roof,
    }
    if r64 is not None:
        v64 = r64["iters"] * nvox / r64["wall"]
        line["fp64"] = {"value": v64, "unit": "voxel-iterations/s", "steps": K64,
                        "iterations": r64["iters"], "ms_per_step": r64["wall"] / K64 * 1e3,
                        "tol": 1e-8, "kernel_ms": {k: v[0] for k, v in r64["kernels"].items() if v[1] > 0},
                        "fp32_over_fp64_wall": (r64["wall"] / K64) / (r32["wall"] / K)}
        if K64 == K:
            import numpy as np
            a = np.array([o["Sigma"][0] for o in r32["outs"]])
            b = np.array([o["Sigma"][0] for o in r64["outs"]])
            line["fp64"]["fp32_max_rel_err_Sigma_xx"] = float(np.abs(a - b).max() / np.abs(b).max())
    KG = args.green_steps if args.green_steps is not None else K
    if KG > 0:
        line["rotated_green"] = green_leg(cp, w, KG, min(W, 1), rk if rk is not None else r32, K, nvox)
        line["error_controlled_substeps"] = substeps_leg(cp, w, KG, r32, K, nvox)
        line["anderson"] = anderson_leg(cp, w, KG, r32, K, nvox)
    line["seq_histogram"] = histogram_leg(s32, nvox)
    if not args.no_micro:
        line["microstructure"] = micro_leg(cp)
        line["eta_sweep"] = eta_leg(cp)
    if args.paper_steps > 0:
        cf = ("none", "neighbouring", "inclusion") if args.paper_configs == "all" else \
            tuple(args.paper_configs.split(","))
        line["paper_set"] = paper_leg(cp, args.paper_steps, cf)
    if args.batch_steps > 0:
        line["batched"] = batch_leg(cp, args.batch_steps)
    if args.adjoint_steps > 0:
        line["adjoint"] = adjoint_leg(cp, args.adjoint_steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, s32, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
