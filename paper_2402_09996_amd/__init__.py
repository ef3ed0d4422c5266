"""MI355X Green-operator FFT solver for voxelized polycrystals with the
regularized Meric-Cailletaud crystal-plasticity law.

Thin Python layer over the C-ABI library ``libcpfft.so`` (declared in
``include/cpfft.h``): argument marshalling only.  Device memory and streams
come from PyTorch; every step of the solve runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import (CPF_FIELD_ACC_SLIP, CPF_FIELD_BACK_STRAIN, CPF_FIELD_PLASTIC_STRAIN,
                   CPF_FIELD_STRAIN, CPF_FIELD_STRESS, CPF_FIELD_SUBSTEPS, CPF_PREC_FP32, CPF_PREC_FP64,
                   CpfError, check)

FIELDS = {
    "stress": CPF_FIELD_STRESS,
    "strain": CPF_FIELD_STRAIN,
    "plastic_strain": CPF_FIELD_PLASTIC_STRAIN,
    "acc_slip": CPF_FIELD_ACC_SLIP,
    "back_strain": CPF_FIELD_BACK_STRAIN,
    "substeps": CPF_FIELD_SUBSTEPS,
}

__all__ = ["Problem", "Solver", "CpfError", "FIELDS", "version", "EffectiveStress", "StressCurveLoss",
           "theta_of", "with_theta", "von_mises_histogram_field", "generate_microstructure", "micro_thin", "micro_label", "micro_graph", "micro_slabs"]


def version() -> int:
    return _lib.lib().cpf_version()


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Problem:
    """Grain-label grid, orientations, stiffness, systems and law parameters.

    labels: int [nz][ny][nx]; euler: [n_labels][3] Bunge radians;
    C_voigt: 6x6 Voigt stiffness (MPa); n_miller, l_miller: [S][3];
    family: [S] (0 slip, 1 twin); tau0: [S] (MPa); law: object with
    ``slip``/``twin`` (Q, b, c, d, K, n, q_self, q_latent), ``twin_mode``,
    ``K_c``, ``f_m``, ``gamma_T``, ``eta``.
    """

    def __init__(self, labels, euler, C_voigt, n_miller, l_miller, family, tau0, law):
        L = _lib.lib()
        self.labels = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
        if self.labels.ndim != 3:
            raise ValueError("labels must be a 3D [nz][ny][nx] array")
        self.shape = self.labels.shape
        self.euler = _f64(euler).reshape(-1, 3)
        self.n_miller = _f64(n_miller).reshape(-1, 3)
        self.l_miller = _f64(l_miller).reshape(-1, 3)
        self.family = np.ascontiguousarray(np.asarray(family, dtype=np.int32))
        self.tau0 = _f64(tau0)
        self.n_sys = int(self.family.shape[0])
        self.law = law
        self.C_voigt = _f64(C_voigt).reshape(6, 6)
        d = _lib.CpfProblemDesc()
        d.nz, d.ny, d.nx = self.shape
        d.labels = _ptr(self.labels, ctypes.c_int32)
        d.n_labels = int(self.euler.shape[0])
        d.euler = _ptr(self.euler, ctypes.c_double)
        C = _f64(C_voigt).reshape(36)
        for i in range(36):
            d.C_crystal[i] = C[i]
        d.n_sys = self.n_sys
        d.n_miller = _ptr(self.n_miller, ctypes.c_double)
        d.l_miller = _ptr(self.l_miller, ctypes.c_double)
        d.family = _ptr(self.family, ctypes.c_int32)
        d.tau0 = _ptr(self.tau0, ctypes.c_double)
        for k, fam in enumerate((law.slip, law.twin)):
            for name in ("Q", "b", "c", "d", "K", "n", "q_self", "q_latent"):
                setattr(d.law[k], name, float(getattr(fam, name)))
        d.twin_mode = int(law.twin_mode)
        d.K_c, d.f_m, d.gamma_T, d.eta = (float(law.K_c), float(law.f_m),
                                          float(law.gamma_T), float(law.eta))
        h = ctypes.c_void_p()
        check(L.cpf_problem_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._destroy = L.cpf_problem_destroy   # usable during interpreter shutdown
        self.n_slip = int((self.family == 0).sum())
        self.n_twin = int((self.family == 1).sum())

    @classmethod
    def from_workload(cls, w) -> "Problem":
        return cls(w.rve.labels, w.rve.euler, w.C, w.systems.n_miller, w.systems.l_miller,
                   w.systems.family, w.systems.tau0, w.law)

    def reference_medium(self) -> tuple[float, float]:
        lam, mu = ctypes.c_double(), ctypes.c_double()
        check(_lib.lib().cpf_problem_reference_medium(self._h, ctypes.byref(lam), ctypes.byref(mu)))
        return lam.value, mu.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


class _PathArgs:
    """Keeps the numpy buffers of a cpf_path alive for one call."""

    def __init__(self, path):
        self.t = _f64(path.t)
        self.ctrl = np.ascontiguousarray(np.asarray(path.strain_ctrl, dtype=np.uint8))
        self.target = _f64(path.target)
        n = int(self.target.shape[0])
        if self.t.shape[0] != n + 1 or self.ctrl.shape != (n, 6) or self.target.shape != (n, 6):
            raise ValueError("path arrays must be t[n+1], strain_ctrl[n][6], target[n][6]")
        self.c = _lib.CpfPath(n, _ptr(self.t, ctypes.c_double), _ptr(self.ctrl, ctypes.c_uint8),
                              _ptr(self.target, ctypes.c_double))
        self.n = n


def _outs_to_dict(outs, n):
    keys = ("sig_eq_of_mean", "mean_sig_eq", "mean_v", "mean_f", "err_eq", "err_bc",
            "n_active", "n_newton")
    r = {"Sigma": np.array([list(outs[i].Sigma) for i in range(n)]).reshape(n, 6),
         "E": np.array([list(outs[i].E) for i in range(n)]).reshape(n, 6),
         "iters": np.array([outs[i].iters for i in range(n)], dtype=np.int64),
         "status": np.array([outs[i].status for i in range(n)], dtype=np.int64),
         "stagnated": np.array([outs[i].stagnated for i in range(n)], dtype=np.int64),
         "host_syncs": np.array([outs[i].host_syncs for i in range(n)], dtype=np.int64),
         "n_symptom": np.array([outs[i].n_symptom for i in range(n)], dtype=np.int64),
         "cutbacks": np.array([outs[i].cutbacks for i in range(n)], dtype=np.int64)}
    for k in keys:
        r[k] = np.array([getattr(outs[i], k) for i in range(n)])
    return r


GREEN = {"continuous": 0, "rotated": 1}
NYQUIST = {"zero": 0, "formula": 1}
REG = {"implicit": 0, "lagged": 1}
TIMING_OFF, TIMING_ALL, TIMING_XPASS = _lib.CPF_TIMING_OFF, _lib.CPF_TIMING_ALL, _lib.CPF_TIMING_XPASS


def _options(precision, tol, max_iter, h_max, rk4_M, lam0, mu0, stag_tol, check_every, green="continuous",
             rk_tol=0.0, aa_depth=0, nyquist="zero", cutback=0, reg="implicit"):
    o = _lib.CpfOptions()
    _lib.lib().cpf_options_default(ctypes.byref(o))
    o.precision = CPF_PREC_FP64 if precision == "fp64" else CPF_PREC_FP32
    o.tol, o.max_iter, o.h_max, o.rk4_M = float(tol), int(max_iter), float(h_max), int(rk4_M)
    if mu0 is not None:
        o.lam0, o.mu0 = float(lam0), float(mu0)
    o.stag_tol, o.check_every = float(stag_tol), int(check_every)
    if green not in GREEN:
        raise ValueError("green must be one of %s" % sorted(GREEN))
    o.green = GREEN[green]
    o.rk_tol = float(rk_tol)
    o.aa_depth = int(aa_depth)
    if nyquist not in NYQUIST:
        raise ValueError("nyquist must be one of %s" % sorted(NYQUIST))
    o.nyquist_mode = NYQUIST[nyquist]
    o.cutback = int(cutback)
    if reg not in REG:
        raise ValueError("reg must be one of %s" % sorted(REG))
    o.reg_mode = REG[reg]
    return o


class Solver:
    """A bound solver: device workspace from torch, work on a torch stream.

    ``problem`` is one :class:`Problem`, or a list of them for a batch
    (members share the law; see :meth:`step_batch`)."""

    def __init__(self, problem, precision: str = "fp64", tol: float = 1e-8,
                 max_iter: int = 1000, h_max: float = 0.05, rk4_M: int = 0,
                 lam0: Optional[float] = None, mu0: Optional[float] = None,
                 stag_tol: float = 0.0, check_every: int = 0, device: str = "cuda:0",
                 stream=None, graph_iters: int = 0, autotune: bool = False,
                 green: str = "continuous", rk_tol: float = 0.0, aa_depth: int = 0,
                 nyquist: str = "zero", cutback: int = 0, reg: str = "implicit"):
        import torch
        L = _lib.lib()
        probs = list(problem) if isinstance(problem, (list, tuple)) else [problem]
        self.problems = probs
        self.problem = probs[0]
        self.n_rve = len(probs)
        self.precision = precision
        self.dtype = {"fp64": torch.float64, "fp32": torch.float32}[precision]
        o = _options(precision, tol, max_iter, h_max, rk4_M, lam0, mu0, stag_tol, check_every, green, rk_tol,
                     aa_depth, nyquist, cutback, reg)
        self.green_operator = green
        self.nyquist = nyquist
        self.reg = reg
        h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * self.n_rve)(*[p._h.value for p in probs])
        check(L.cpf_batch_create(self.n_rve, arr, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._destroy = L.cpf_solver_destroy
        size = ctypes.c_size_t()
        check(L.cpf_solver_workspace_size(h, ctypes.byref(size)))
        self.device = torch.device(device)
        self.workspace = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        if stream is None:
            # graph capture needs a stream of its own (the legacy default
            # stream cannot be captured); default priority
            stream = torch.cuda.Stream(self.device) if graph_iters else \
                torch.cuda.current_stream(self.device)
        self.stream = stream
        check(L.cpf_solver_bind(h, ctypes.c_void_p(self._ws_ptr), int(size.value),
                                ctypes.c_void_p(self.stream.cuda_stream)))
        self.nz, self.ny, self.nx = self.problem.shape
        self.nvox = self.nx * self.ny * self.nz
        self.nhx = self.nx // 2 + 1
        self.autotuned = 0
        if autotune:
            self.autotune()
        if graph_iters:
            self.set_graph(graph_iters)

    def autotune(self) -> int:
        n = ctypes.c_int()
        check(_lib.lib().cpf_solver_autotune(self._h, ctypes.byref(n)))
        self.autotuned = n.value
        return n.value

    def tiles(self, rve: int = 0) -> tuple[int, int]:
        ty, tz = ctypes.c_int(), ctypes.c_int()
        check(_lib.lib().cpf_solver_tiles(self._h, int(rve), ctypes.byref(ty), ctypes.byref(tz)))
        return ty.value, tz.value

    def set_tiles(self, ty: int, tz: int, rve: int = 0):
        """y and z pass tile widths (kx columns per block) of one RVE."""
        check(_lib.lib().cpf_solver_set_tiles(self._h, int(rve), int(ty), int(tz)))

    def set_graph(self, iters_per_launch):
        """Graph launches of ``iters_per_launch`` iterations per replay,
        ``"adaptive"`` (a length per step from the previous step's count:
        normally one replay per step), or 0 (direct launches)."""
        if iters_per_launch == "adaptive":
            iters_per_launch = _lib.CPF_GRAPH_ADAPTIVE
        check(_lib.lib().cpf_solver_set_graph(self._h, int(iters_per_launch)))

    def step_batch(self, path, n: int) -> list[dict]:
        """Load step n for every member of the batch."""
        pa = _PathArgs(path)
        outs = (_lib.CpfStepOut * self.n_rve)()
        check(_lib.lib().cpf_batch_step(self._h, ctypes.byref(pa.c), int(n), outs))
        d = _outs_to_dict(outs, self.n_rve)
        return [{k: v[i] for k, v in d.items()} for i in range(self.n_rve)]

    def field_of(self, rve: int, name: str):
        import torch
        k = FIELDS[name]
        nz, ny, nx = self.problems[rve].shape
        nc = 6 if k in (CPF_FIELD_STRESS, CPF_FIELD_STRAIN, CPF_FIELD_PLASTIC_STRAIN) \
            else 1 if k == CPF_FIELD_SUBSTEPS else self.problem.n_sys
        out = torch.empty((nc, nz, ny, nx), dtype=self.dtype, device=self.device)
        check(_lib.lib().cpf_batch_field(self._h, int(rve), k, ctypes.c_void_p(out.data_ptr())))
        return out

    # -- solve ---------------------------------------------------------------
    def reset(self):
        check(_lib.lib().cpf_solver_reset(self._h))

    def run(self, path) -> dict:
        pa = _PathArgs(path)
        outs = (_lib.CpfStepOut * pa.n)()
        check(_lib.lib().cpf_solver_run(self._h, ctypes.byref(pa.c), outs))
        return _outs_to_dict(outs, pa.n)

    def step(self, path, n: int) -> dict:
        pa = _PathArgs(path)
        out = (_lib.CpfStepOut * 1)()
        check(_lib.lib().cpf_solver_step(self._h, ctypes.byref(pa.c), int(n), out))
        return {k: v[0] for k, v in _outs_to_dict(out, 1).items()}

    def field(self, name: str):
        """Committed local field as a torch tensor [ncomp][nz][ny][nx]."""
        import torch
        k = FIELDS[name]
        nc = 6 if k in (CPF_FIELD_STRESS, CPF_FIELD_STRAIN, CPF_FIELD_PLASTIC_STRAIN) \
            else 1 if k == CPF_FIELD_SUBSTEPS else self.problem.n_sys
        out = torch.empty((nc, self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        check(_lib.lib().cpf_solver_field(self._h, k, ctypes.c_void_p(out.data_ptr())))
        return out

    # -- gradients -------------------------------------------------------------
    THETA_NAMES = ("r0", "Q", "b", "c", "d", "K", "n")

    def adjoint_workspace_size(self, path, checkpoint_every: int = 10) -> int:
        pa = _PathArgs(path)
        size = ctypes.c_size_t()
        check(_lib.lib().cpf_adjoint_workspace_size(self._h, ctypes.byref(pa.c), int(checkpoint_every),
                                                    ctypes.byref(size)))
        return int(size.value)

    def gradient(self, path, target_xx, checkpoint_every: int = 10, adj_tol: float = 1e-10):
        """Loss sum_n (Sigma_11,n - target_xx[n])^2 over the path and its
        gradient [2][7] with respect to (r0, Q, b, c, d, K, n) of the slip
        and twin families, by the discrete adjoint on the device.  Returns
        (loss, grad, sigma_xx).  The solver is left at the undeformed state."""
        import torch
        pa = _PathArgs(path)
        tgt = _f64(target_xx)
        if tgt.shape != (pa.n,):
            raise ValueError("target_xx must have one value per load step")
        need = self.adjoint_workspace_size(path, checkpoint_every)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ptr = (ws.data_ptr() + 255) & ~255
        self._order_after_torch()
        loss = ctypes.c_double()
        grad = np.zeros(14)
        sxx = np.zeros(pa.n)
        check(_lib.lib().cpf_adjoint_gradient(self._h, ctypes.byref(pa.c), _ptr(tgt, ctypes.c_double),
                                              int(checkpoint_every), float(adj_tol), ctypes.c_void_p(ptr),
                                              need, ctypes.byref(loss), _ptr(grad, ctypes.c_double),
                                              _ptr(sxx, ctypes.c_double)))
        del ws
        return loss.value, grad.reshape(2, 7), sxx

    def vjp(self, path, sigma_bar, checkpoint_every: int = 10, adj_tol: float = 1e-10):
        """dJ/dtheta [2][7] of J = sum_n sigma_bar[n] . Sigma_n (cotangent
        sigma_bar[n_steps][6] of the mean stresses, tensor components) by the
        discrete adjoint, and the mean stress history Sigma[n_steps][6]."""
        import torch
        pa = _PathArgs(path)
        sb = _f64(sigma_bar)
        if sb.shape != (pa.n, 6):
            raise ValueError("sigma_bar must be [n_steps][6]")
        need = self.adjoint_workspace_size(path, checkpoint_every)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ptr = (ws.data_ptr() + 255) & ~255
        self._order_after_torch()
        grad = np.zeros(14)
        sig = np.zeros((pa.n, 6))
        check(_lib.lib().cpf_adjoint_vjp(self._h, ctypes.byref(pa.c), _ptr(sb, ctypes.c_double),
                                         int(checkpoint_every), float(adj_tol), ctypes.c_void_p(ptr), need,
                                         _ptr(grad, ctypes.c_double), _ptr(sig, ctypes.c_double)))
        del ws
        return grad.reshape(2, 7), sig

    def von_mises_histogram(self, nbins: int, lo: float, hi: float, rve: int = -1):
        """Counts [nbins + 2] of the local von Mises stress of the committed
        state over RVE ``rve`` (-1: every RVE of the batch): below lo, the
        nbins bins of [lo, hi), and the rest."""
        counts = np.zeros(int(nbins) + 2, dtype=np.uint64)
        self._order_after_torch()
        check(_lib.lib().cpf_seq_histogram(self._h, int(rve), int(nbins), float(lo), float(hi),
                                           counts.ctypes.data_as(ctypes.POINTER(ctypes.c_ulonglong))))
        return counts

    def von_mises_pdf(self, nbins: int, lo: float, hi: float, rve: int = -1):
        """Bin centres and the probability density of the local von Mises
        stress (counts / (all voxels * bin width))."""
        c = self.von_mises_histogram(nbins, lo, hi, rve).astype(np.float64)
        w = (hi - lo) / nbins
        return lo + w * (np.arange(nbins) + 0.5), c[1:-1] / (c.sum() * w)

    # -- committed state ---------------------------------------------------------
    def save_state(self):
        """The committed state of every RVE in a device buffer (torch uint8)."""
        import torch
        size = ctypes.c_size_t()
        check(_lib.lib().cpf_state_size(self._h, ctypes.byref(size)))
        buf = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        view = buf[off:off + int(size.value)]
        self._order_after_torch()
        check(_lib.lib().cpf_state_save(self._h, ctypes.c_void_p(view.data_ptr())))
        return view

    def restore_state(self, saved):
        """Make a buffer from :meth:`save_state` the committed state again."""
        self._order_after_torch()
        check(_lib.lib().cpf_state_restore(self._h, ctypes.c_void_p(saved.data_ptr())))

    def adjoint_stats(self) -> dict:
        """Work of the last :meth:`gradient` call."""
        f, a, r = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        check(_lib.lib().cpf_adjoint_last_stats(self._h, ctypes.byref(f), ctypes.byref(a), ctypes.byref(r)))
        return {"forward_iterations": f.value, "adjoint_iterations": a.value, "recomputed_steps": r.value}

    # -- kernel timing -------------------------------------------------------
    KERNELS = ("xpass_law", "ypass_fwd", "zpass_green", "ypass_inv", "bc_update")

    def set_timing(self, on=True):
        """Per-kernel HIP-event timing: True (every kernel class), False, or
        "xpass" (the x pass only: two events per iteration instead of ten)."""
        mode = TIMING_XPASS if on == "xpass" else (TIMING_ALL if on else TIMING_OFF)
        check(_lib.lib().cpf_solver_set_timing(self._h, mode))

    def timing(self) -> dict:
        ms = (ctypes.c_double * 5)()
        n = (ctypes.c_longlong * 5)()
        check(_lib.lib().cpf_solver_get_timing(self._h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(self.KERNELS)}

    def _order_after_torch(self):
        # inputs made by torch on its current stream must be complete before
        # the library reads them on the solver's stream
        import torch
        if self.stream != torch.cuda.current_stream(self.device):
            torch.cuda.current_stream(self.device).synchronize()

    # -- component operators ---------------------------------------------------
    def forward_fft(self, f):
        """Unnormalized 3D DFT of 6 real fields [6][nz][ny][nx] -> complex
        half spectrum [6][nz][ny][nx/2+1] (torch complex tensor)."""
        import torch
        f = f.to(device=self.device, dtype=self.dtype).contiguous()
        # the library's layout is [nz][ny][nx/2+1][6]; returned as a view
        spec = torch.empty((self.nz, self.ny, self.nhx, 6, 2), dtype=self.dtype, device=self.device)
        self._order_after_torch()
        check(_lib.lib().cpf_op_forward_fft(self._h, ctypes.c_void_p(f.data_ptr()),
                                            ctypes.c_void_p(spec.data_ptr())))
        return torch.view_as_complex(spec).permute(3, 0, 1, 2)

    def green(self, spec):
        """F^-1[Gamma0 : spec] on the grid and the residual sum.  `spec` is a
        complex half spectrum; a copy is consumed."""
        import torch
        # [6][nz][ny][nx/2+1] complex to the library's [nz][ny][nx/2+1][6]
        s = torch.view_as_real(spec.to(self.device).permute(1, 2, 3, 0)).to(self.dtype).contiguous().clone()
        out = torch.empty((6, self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        err2 = ctypes.c_double()
        self._order_after_torch()
        check(_lib.lib().cpf_op_green(self._h, ctypes.c_void_p(s.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), ctypes.byref(err2)))
        return out, err2.value

    def constitutive(self, eps0, eps1, state0, dt: float, M: int):
        """Local law over one increment at every voxel (device arrays)."""
        import torch
        D = 6 + 2 * self.problem.n_sys
        args = [t.to(device=self.device, dtype=self.dtype).contiguous()
                for t in (eps0, eps1, state0)]
        assert args[0].numel() == 6 * self.nvox and args[2].numel() == D * self.nvox
        st1 = torch.empty((D, self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        sig = torch.empty((6, self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        self._order_after_torch()
        check(_lib.lib().cpf_op_constitutive(
            self._h, *[ctypes.c_void_p(a.data_ptr()) for a in args],
            ctypes.c_void_p(st1.data_ptr()), ctypes.c_void_p(sig.data_ptr()), float(dt), int(M)))
        return st1, sig

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


def theta_of(problem: Problem) -> np.ndarray:
    """The law parameters theta[2][7] of ``problem``: per family (slip,
    twin) r0, Q, b, c, d, K, n, where r0 is the family's lowest initial
    resolved shear stress tau0 (0 for a family without systems)."""
    th = np.zeros((2, 7))
    for f, fam in enumerate((problem.law.slip, problem.law.twin)):
        sel = problem.tau0[problem.family == f]
        th[f, 0] = float(sel.min()) if sel.size else 0.0
        for k, name in enumerate(Solver.THETA_NAMES[1:], start=1):
            th[f, k] = float(getattr(fam, name))
    return th


def with_theta(problem: Problem, theta) -> Problem:
    """A copy of ``problem`` whose law parameters are theta[2][7]: per family
    (slip, twin) r0, Q, b, c, d, K, n.  r0 moves every tau0 of the family by
    the same amount, theta[f][0] - theta_of(problem)[f][0], so systems keep
    their offsets (Section 3's ordinary and superdislocation resistances
    differ by a constant), the problem's own theta gives back the problem,
    and the derivative with respect to r0 is that of a uniform shift, as
    the adjoint computes it."""
    import copy
    th = np.asarray(theta, dtype=np.float64).reshape(2, 7)
    ref = theta_of(problem)
    law = copy.deepcopy(problem.law)
    tau0 = problem.tau0.copy()
    for f, fam in enumerate((law.slip, law.twin)):
        tau0[problem.family == f] += th[f, 0] - ref[f, 0]
        for k, name in enumerate(Solver.THETA_NAMES[1:], start=1):
            setattr(fam, name, float(th[f, k]))
    return Problem(problem.labels, problem.euler, problem.C_voigt, problem.n_miller,
                   problem.l_miller, problem.family, tau0, law)


class EffectiveStress:
    """torch.autograd binding of the solve: ``EffectiveStress.apply(theta,
    problem, path, options)`` with theta a float64 tensor [2][7] (per family
    r0, Q, b, c, d, K, n) returns the mean stress history Sigma[n_steps][6]
    (tensor components) of the solve along ``path``; its backward is
    :meth:`Solver.vjp` with the incoming cotangent, so any loss built from
    Sigma in torch gets its parameter gradient from the discrete adjoint.
    options: :class:`Solver` keyword arguments plus ``checkpoint_every`` and
    ``adj_tol``."""

    @staticmethod
    def _function():
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta, problem, path, options):
                opts = dict(options or {})
                ck = opts.pop("checkpoint_every", 10)
                at = opts.pop("adj_tol", 1e-10)
                p = with_theta(problem, theta.detach().cpu().numpy())
                s = Solver(p, **opts)
                sig = s.run(path)["Sigma"]
                ctx.solver, ctx.path, ctx.ck, ctx.at = s, path, ck, at
                return torch.as_tensor(sig, dtype=theta.dtype, device=theta.device)

            @staticmethod
            def backward(ctx, gout):
                g, _ = ctx.solver.vjp(ctx.path, gout.detach().double().cpu().numpy(),
                                      checkpoint_every=ctx.ck, adj_tol=ctx.at)
                return torch.as_tensor(g, dtype=gout.dtype, device=gout.device), None, None, None

        return _Fn

    @classmethod
    def apply(cls, theta, problem, path, options=None):
        return cls._function().apply(theta, problem, path, options)


class StressCurveLoss:
    """torch.autograd binding of :meth:`Solver.gradient`.

    ``StressCurveLoss.apply(theta, problem, path, target_xx, options)`` with
    theta a float64 tensor [2][7] returns the scalar loss; its backward
    multiplies the adjoint gradient by the incoming cotangent.  options: a
    dict of :class:`Solver` keyword arguments plus ``checkpoint_every`` and
    ``adj_tol``."""

    @staticmethod
    def _function():
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta, problem, path, target_xx, options):
                opts = dict(options or {})
                ck = opts.pop("checkpoint_every", 10)
                at = opts.pop("adj_tol", 1e-10)
                p = with_theta(problem, theta.detach().cpu().numpy())
                s = Solver(p, **opts)
                L, g, _ = s.gradient(path, target_xx, checkpoint_every=ck, adj_tol=at)
                ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
                return torch.tensor(L, dtype=theta.dtype, device=theta.device)

            @staticmethod
            def backward(ctx, gout):
                (g,) = ctx.saved_tensors
                return gout * g, None, None, None, None

        return _Fn

    @classmethod
    def apply(cls, theta, problem, path, target_xx, options=None):
        return cls._function().apply(theta, problem, path, target_xx, options)


# ---------------------------------------------------------------------------
# Stochastic microstructure model (Section 2), include/cpfft_micro.h
# ---------------------------------------------------------------------------
def _micro_params(shape, lam, r, p_neigh, p_incl, delta, theta, seed, q):
    p = _lib.CpfMicroParams()
    p.nz, p.ny, p.nx = (int(v) for v in shape)
    p.q = int(q)
    p.lambda_, p.r = float(lam), float(r)
    p.p_neigh, p.p_incl = float(p_neigh), float(p_incl)
    p.delta_lo, p.delta_hi = float(delta[0]), float(delta[1])
    p.theta = float(theta)
    p.seed = int(seed) & ((1 << 64) - 1)
    return p


def generate_microstructure(shape, lam: float, r: float, p_neigh: float = 0.0, p_incl: float = 0.0,
                            delta=(0.1, 0.3), theta: float = 1.2180652849668427, seed: int = 1, q: int = 16,
                            device: str = "cuda:0", stream=None) -> dict:
    """One realization of the Section 2 model on the device.

    shape (nz, ny, nx) voxels; lam: primary Poisson intensity per voxel^3;
    r: hard-core radius (voxels); p_neigh, p_incl: twin parameters;
    delta: relative inclusion thickness bounds; theta: twin angle (radians,
    default 69.79 degrees).  Returns labels (device int32 tensor
    [nz][ny][nx]), rotations [n_labels][3][3] (crystal to lab), euler
    [n_labels][3] (Bunge), pairs [n_pairs][3] and the counts of
    cpf_micro_info."""
    import torch
    L = _lib.lib()
    p = _micro_params(shape, lam, r, p_neigh, p_incl, delta, theta, seed, q)
    size = ctypes.c_size_t()
    check(L.cpf_micro_workspace_size(ctypes.byref(p), ctypes.byref(size)))
    dev = torch.device(device)
    ws = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=dev)
    base = (ws.data_ptr() + 255) & ~255
    labels = torch.empty(tuple(int(v) for v in shape), dtype=torch.int32, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    mu = float(lam) * labels.numel()
    max_labels = 2 * (int(mu + 20.0 * mu ** 0.5 + 20.0) + 1)
    rot = np.zeros((max_labels, 9))
    eul = np.zeros((max_labels, 3))
    pairs = np.zeros((max_labels // 2, 3), dtype=np.int32)
    info = _lib.CpfMicroInfo()
    check(L.cpf_micro_generate(ctypes.byref(p), ctypes.c_void_p(base), int(size.value),
                               ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(labels.data_ptr()),
                               max_labels, _ptr(rot, ctypes.c_double), _ptr(eul, ctypes.c_double),
                               _ptr(pairs, ctypes.c_int32), ctypes.byref(info)))
    n = info.n_labels
    out = {k: getattr(info, k) for k, _ in _lib.CpfMicroInfo._fields_}
    out.update(labels=labels, rotations=rot[:n].reshape(n, 3, 3).copy(), euler=eul[:n].copy(),
               pairs=pairs[:info.n_pairs].copy())
    return out


def von_mises_histogram_field(stress, nbins: int, lo: float, hi: float, stream=None):
    """Counts [nbins + 2] of the local von Mises stress of a device stress
    field ``stress`` (torch float32/float64, [6][...] components 11, 22,
    33, 23, 13, 12), with the bins of :meth:`Solver.von_mises_histogram`;
    no solver and no workspace (cpf_seq_histogram_field allocates nothing)."""
    import torch
    if stress.dtype not in (torch.float32, torch.float64) or not stress.is_cuda:
        raise TypeError("stress must be a float32 or float64 device tensor")
    if stress.shape[0] != 6 or not stress.is_contiguous():
        raise ValueError("stress must be a contiguous [6][...] tensor")
    prec = CPF_PREC_FP64 if stress.dtype == torch.float64 else CPF_PREC_FP32
    counts = np.zeros(int(nbins) + 2, dtype=np.uint64)
    with torch.cuda.device(stress.device):
        check(_lib.lib().cpf_seq_histogram_field(ctypes.c_void_p(stress.data_ptr()), prec, stress[0].numel(),
                                                 int(nbins), float(lo), float(hi),
                                                 counts.ctypes.data_as(ctypes.POINTER(ctypes.c_ulonglong)),
                                                 _stream_ptr(stream, stress)))
    return counts


def _stream_ptr(stream, t):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(s.cuda_stream)


def micro_thin(points, L, r_q: float, stream=None):
    """Matern type II keep flags of device points int32 [n][4] in the box L
    (lattice units): uint8 [n] device tensor."""
    import torch
    keep = torch.empty(points.shape[0], dtype=torch.uint8, device=points.device)
    check(_lib.lib().cpf_micro_thin(int(points.shape[0]), ctypes.c_void_p(points.data_ptr()), int(L[0]),
                                    int(L[1]), int(L[2]), float(r_q), ctypes.c_void_p(keep.data_ptr()),
                                    _stream_ptr(stream, points)))
    return keep


def micro_label(shape, q: int, seeds, stream=None):
    """Periodic Voronoi labels [nz][ny][nx] of device generators int32
    [n][4]; returns (labels, number of tiles that searched every seed)."""
    import torch
    labels = torch.empty(tuple(int(v) for v in shape), dtype=torch.int32, device=seeds.device)
    fb = torch.zeros(1, dtype=torch.int32, device=seeds.device)
    nz, ny, nx = shape
    check(_lib.lib().cpf_micro_label(int(nx), int(ny), int(nz), int(q), int(seeds.shape[0]),
                                     ctypes.c_void_p(seeds.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                                     ctypes.c_void_p(fb.data_ptr()), _stream_ptr(stream, seeds)))
    return labels, fb


def micro_graph(labels, n: int, stream=None):
    """Face adjacency bit matrix uint32 [n][(n+31)/32] (as int32) and
    voxel counts [n] (as int64) of a device label grid."""
    import torch
    nz, ny, nx = labels.shape
    W = (n + 31) // 32
    adj = torch.empty((n, W), dtype=torch.int32, device=labels.device)
    vol = torch.empty(n, dtype=torch.int64, device=labels.device)
    check(_lib.lib().cpf_micro_graph(int(nx), int(ny), int(nz), ctypes.c_void_p(labels.data_ptr()), int(n),
                                     ctypes.c_void_p(adj.data_ptr()), ctypes.c_void_p(vol.data_ptr()),
                                     _stream_ptr(stream, labels)))
    return adj, vol


def micro_slabs(labels, q: int, n: int, slab_of, slabs, stream=None):
    """Apply inclusion slabs in place: slab_of int32 [n] (-1 or slab
    index), slabs float64 [m][8] (n0 n1 n2 x0 y0 z0 half child), device."""
    nz, ny, nx = labels.shape
    check(_lib.lib().cpf_micro_slabs(int(nx), int(ny), int(nz), int(q), ctypes.c_void_p(labels.data_ptr()),
                                     int(n), ctypes.c_void_p(slab_of.data_ptr()), ctypes.c_void_p(slabs.data_ptr()),
                                     _stream_ptr(stream, labels)))
    return labels
