"""ctypes binding of ``libcpfft.so`` (argument marshalling only).

The library must have been built in-tree (``__graft_entry__.build()`` or
``python paper_2402_09996_amd/build.py``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CPFFT_LIBRARY may point at another build of the same library (e.g. a
# variant compiled with different launch bounds for a timing comparison).
LIB_PATH = os.environ.get("CPFFT_LIBRARY", os.path.join(HERE, "libcpfft.so"))

CPF_OK = 0
CPF_E_INVALID_ARG = -1
CPF_E_WORKSPACE = -2
CPF_E_HIP = -3
CPF_E_NOT_CONVERGED = -4
CPF_E_NAN = -5
CPF_E_UNSUPPORTED_SIZE = -6
CPF_E_BAD_STATE = -7

CPF_PREC_FP64 = 0
CPF_PREC_FP32 = 1

CPF_FIELD_STRESS = 0
CPF_FIELD_STRAIN = 1
CPF_FIELD_PLASTIC_STRAIN = 2
CPF_FIELD_ACC_SLIP = 3
CPF_FIELD_BACK_STRAIN = 4
CPF_FIELD_SUBSTEPS = 5

CPF_REG_IMPLICIT = 0
CPF_REG_LAGGED = 1

CPF_TIMING_OFF = 0
CPF_TIMING_ALL = 1
CPF_TIMING_XPASS = 2

CPF_MAX_SYSTEMS = 32
CPF_GRAPH_ADAPTIVE = -1

_d = ctypes.c_double
_i = ctypes.c_int
_p = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class CpfLaw(ctypes.Structure):
    _fields_ = [(n, _d) for n in ("Q", "b", "c", "d", "K", "n", "q_self", "q_latent")]


class CpfProblemDesc(ctypes.Structure):
    _fields_ = [
        ("nx", _i), ("ny", _i), ("nz", _i),
        ("labels", _ip), ("n_labels", _i), ("euler", _dp),
        ("C_crystal", _d * 36), ("n_sys", _i),
        ("n_miller", _dp), ("l_miller", _dp), ("family", _ip), ("tau0", _dp),
        ("law", CpfLaw * 2), ("twin_mode", _i),
        ("K_c", _d), ("f_m", _d), ("gamma_T", _d), ("eta", _d),
    ]


class CpfOptions(ctypes.Structure):
    _fields_ = [
        ("precision", _i), ("tol", _d), ("max_iter", _i), ("h_max", _d),
        ("rk4_M", _i), ("lam0", _d), ("mu0", _d), ("stag_tol", _d),
        ("check_every", _i), ("green", _i), ("rk_tol", _d), ("aa_depth", _i),
        ("nyquist_mode", _i), ("cutback", _i), ("reg_mode", _i),
    ]


class CpfPath(ctypes.Structure):
    _fields_ = [("n_steps", _i), ("t", _dp), ("strain_ctrl", _u8p), ("target", _dp)]


class CpfStepOut(ctypes.Structure):
    _fields_ = [
        ("Sigma", _d * 6), ("E", _d * 6),
        ("sig_eq_of_mean", _d), ("mean_sig_eq", _d), ("mean_v", _d), ("mean_f", _d),
        ("err_eq", _d), ("err_bc", _d), ("n_active", _d), ("n_newton", _d),
        ("iters", _i), ("status", _i), ("stagnated", _i), ("host_syncs", _i),
        ("n_symptom", ctypes.c_longlong), ("cutbacks", _i),
    ]


class CpfMicroParams(ctypes.Structure):
    _fields_ = [("nx", _i), ("ny", _i), ("nz", _i), ("q", _i), ("lambda_", _d), ("r", _d),
                ("p_neigh", _d), ("p_incl", _d), ("delta_lo", _d), ("delta_hi", _d), ("theta", _d),
                ("seed", ctypes.c_uint64)]


class CpfMicroInfo(ctypes.Structure):
    _fields_ = [("n_primary", _i), ("n_grains", _i), ("n_neigh_drawn", _i), ("n_pairs", _i),
                ("n_inclusions", _i), ("n_labels", _i), ("draws", ctypes.c_longlong),
                ("fallback_tiles", _i)]


# name -> (restype, argtypes); every symbol include/*.h declares
SIGNATURES = {
    "cpf_version": (_i, []),
    "cpf_error_string": (ctypes.c_char_p, [_i]),
    "cpf_last_error_message": (ctypes.c_char_p, []),
    "cpf_options_default": (None, [ctypes.POINTER(CpfOptions)]),
    "cpf_problem_create": (_i, [ctypes.POINTER(CpfProblemDesc), ctypes.POINTER(_p)]),
    "cpf_problem_destroy": (None, [_p]),
    "cpf_problem_reference_medium": (_i, [_p, _dp, _dp]),
    "cpf_solver_create": (_i, [_p, ctypes.POINTER(CpfOptions), ctypes.POINTER(_p)]),
    "cpf_solver_workspace_size": (_i, [_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cpf_solver_bind": (_i, [_p, _p, ctypes.c_size_t, _p]),
    "cpf_solver_reset": (_i, [_p]),
    "cpf_solver_step": (_i, [_p, ctypes.POINTER(CpfPath), _i, ctypes.POINTER(CpfStepOut)]),
    "cpf_solver_run": (_i, [_p, ctypes.POINTER(CpfPath), ctypes.POINTER(CpfStepOut)]),
    "cpf_solver_field": (_i, [_p, _i, _p]),
    "cpf_solver_destroy": (None, [_p]),
    "cpf_batch_create": (_i, [_i, ctypes.POINTER(_p), ctypes.POINTER(CpfOptions), ctypes.POINTER(_p)]),
    "cpf_batch_size": (_i, [_p, ctypes.POINTER(_i)]),
    "cpf_batch_step": (_i, [_p, ctypes.POINTER(CpfPath), _i, ctypes.POINTER(CpfStepOut)]),
    "cpf_batch_field": (_i, [_p, _i, _i, _p]),
    "cpf_solver_set_graph": (_i, [_p, _i]),
    "cpf_solver_autotune": (_i, [_p, ctypes.POINTER(_i)]),
    "cpf_solver_tiles": (_i, [_p, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "cpf_solver_set_tiles": (_i, [_p, _i, _i, _i]),
    "cpf_solver_set_timing": (_i, [_p, _i]),
    "cpf_solver_get_timing": (_i, [_p, _dp, ctypes.POINTER(ctypes.c_longlong)]),
    "cpf_op_forward_fft": (_i, [_p, _p, _p]),
    "cpf_op_green": (_i, [_p, _p, _p, _dp]),
    "cpf_op_constitutive": (_i, [_p, _p, _p, _p, _p, _p, _d, _i]),
    "cpf_adjoint_workspace_size": (_i, [_p, ctypes.POINTER(CpfPath), _i, ctypes.POINTER(ctypes.c_size_t)]),
    "cpf_adjoint_gradient": (_i, [_p, ctypes.POINTER(CpfPath), _dp, _i, _d, _p, ctypes.c_size_t, _dp, _dp, _dp]),
    "cpf_adjoint_vjp": (_i, [_p, ctypes.POINTER(CpfPath), _dp, _i, _d, _p, ctypes.c_size_t, _dp, _dp]),
    "cpf_seq_histogram": (_i, [_p, _i, _i, _d, _d, ctypes.POINTER(ctypes.c_ulonglong)]),
    "cpf_seq_histogram_field": (_i, [_p, _i, ctypes.c_longlong, _i, _d, _d, ctypes.POINTER(ctypes.c_ulonglong),
                                     _p]),
    "cpf_state_size": (_i, [_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cpf_state_save": (_i, [_p, _p]),
    "cpf_state_restore": (_i, [_p, _p]),
    "cpf_micro_workspace_size": (_i, [ctypes.POINTER(CpfMicroParams), ctypes.POINTER(ctypes.c_size_t)]),
    "cpf_micro_generate": (_i, [ctypes.POINTER(CpfMicroParams), _p, ctypes.c_size_t, _p, _p, _i, _dp, _dp,
                                _ip, ctypes.POINTER(CpfMicroInfo)]),
    "cpf_micro_thin": (_i, [_i, _p, _i, _i, _i, _d, _p, _p]),
    "cpf_micro_label": (_i, [_i, _i, _i, _i, _i, _p, _p, _p, _p]),
    "cpf_micro_graph": (_i, [_i, _i, _i, _p, _i, _p, _p, _p]),
    "cpf_micro_slabs": (_i, [_i, _i, _i, _i, _p, _i, _p, _p, _p]),
    "cpf_adjoint_last_stats": (_i, [_p, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(_i)]),
}

_lib = None


class CpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("cpfft error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("%s is not built: run __graft_entry__.build() "
                              "or python paper_2402_09996_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != CPF_OK:
        raise CpfError(code, lib().cpf_last_error_message().decode())
    return code
