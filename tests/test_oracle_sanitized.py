"""The oracle's C law under AddressSanitizer and UndefinedBehaviorSanitizer.

``oracle/build.py`` compiles ``cp_law.c`` a second time with every
sanitizer report fatal; a child Python process preloads the gcc sanitizer
runtimes, loads that build through ``CP_ORACLE_LIB`` and drives every entry
point of the C part on a small twinned RVE: the forward solve (probe,
update, per-substep update), the rate and RK4 vector-Jacobian products and
the discrete adjoint of a 3-step load path, in both twin laws and with the
regularization on and off.  CPU only.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import numpy as np
import oracle, rvegen
C, law = rvegen.config_law()
S = rvegen.config_systems(True)
rve = rvegen.make_rve((4, 4, 6), 3, 77, twin_share=0.5)
path = rvegen.uniaxial_path(0.006, 3, rate=1e-2)
for mode, eta in ((rvegen.TWIN_NORTON, law.eta), (rvegen.TWIN_PAPER, law.eta), (rvegen.TWIN_NORTON, 0.0)):
    law.twin_mode, law.eta = mode, eta
    if mode == rvegen.TWIN_PAPER:
        law.K_c, law.f_m = 1.45, 0.8
    w = rvegen.Workload("t", rve, S, C, law, path)
    m = oracle.solver_for(w, oracle.Options()).mat
    rng = np.random.default_rng(1)
    e = oracle.to_mandel(np.array([3e-3, -1.2e-3, -1.5e-3, 2e-4, -1e-4, 3e-4]))
    y = np.concatenate([rng.standard_normal(6) * 2e-4, rng.random(16) * 2e-3, rng.standard_normal(16) * 1e-3])
    assert np.all(np.isfinite(m.rate(0, e, y)))
    m.rate_vjp(0, e, y, rng.standard_normal(m.state_dim))
    if eta == 0.0:      # explicit RK4 on the unregularized law needs far smaller steps
        continue
    for sub in (0.0, 1e-4):
        o = oracle.solver_for(w, oracle.Options(tol=1e-10, rk_tol=sub))
        r = o.run(path)
        assert np.all(np.isfinite(r.Sigma))
    o = oracle.solver_for(w, oracle.Options(tol=1e-10))
    tgt = o.run(path).Sigma[:, 0] * 1.03
    L, grad, _ = o.gradient(path, tgt, adj_tol=1e-10)
    assert np.isfinite(L) and np.all(np.isfinite(grad))
for o_, A, K, n, eta in ((50.0, 1e-3, 10.0, 10.0, 1e4), (50.0, 1e-3, 10.0, 10.0, 0.0), (-1.0, 1e-3, 10.0, 10.0, 1e4)):
    assert np.isfinite(oracle.reg_rate(o_, A, K, n, eta))
print("sanitized oracle ok", oracle.threads(), "threads")
"""


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_c_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    lib = ob.build_sanitized(str(tmp_path / "cp_law_san.so"))
    env = dict(os.environ)
    env.update(CP_ORACLE_LIB=lib, LD_PRELOAD=asan + ":" + ubsan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    p = subprocess.run([sys.executable, "-c", DRIVER], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    report = p.stdout[-3000:] + p.stderr[-6000:]
    assert p.returncode == 0, report
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, report
    assert "sanitized oracle ok" in p.stdout
