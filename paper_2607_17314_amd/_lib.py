"""ctypes declarations of the C ABI in include/isdf_xtc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisdfxtc.so")

XTC_OK, XTC_WARN_RANK_DEFICIENT, XTC_WARN_JITTER, XTC_WARN_FALLBACK = 0, 1, 2, 3
XTC_ERR_INVALID_ARG, XTC_ERR_NOT_SPD, XTC_ERR_HIP, XTC_ERR_NO_WORKSPACE, XTC_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
XTC_FP64, XTC_FP32, XTC_SPLIT_F16 = 0, 1, 2
XTC_U_EE, XTC_U_BH = 0, 1
XTC_U1, XTC_U3, XTC_ULAP, XTC_D1, XTC_D4, XTC_FIELD, XTC_ESCALE = 1, 2, 4, 8, 16, 32, 64
XTC_SELECT_QR, XTC_SELECT_LEARNED, XTC_SELECT_LEARNED_JUDGED = 0, 1, 2
XTC_FIT_XI, XTC_FIT_XIGRAD, XTC_FIT_KEEP_CHOL = 1, 2, 4
XTC_WS_XIGRAD_BLOCKS = 1 << 24
XTC_WS_BH = 1 << 25


def chol_system_doubles(n_mu: int) -> int:
    """XTC_CHOL_SYSTEM_DOUBLES: one system's kept factor and inverted diagonal blocks."""
    return n_mu * n_mu + 4096 * ((n_mu + 63) // 64)
XTC_CALL_EVAL_ORBITALS, XTC_CALL_SELECT, XTC_CALL_FIT, XTC_CALL_CONTRACT, XTC_CALL_GRAD = 1, 2, 3, 4, 5
XTC_CALL_FEATURES, XTC_CALL_MLP_GRAD, XTC_CALL_EXCHANGE = 6, 7, 8
XTC_CALL_ASSEMBLY, XTC_CALL_ONE_BODY, XTC_CALL_VMC = 9, 10, 11
XTC_ASM_K, XTC_ASM_DU, XTC_ASM_W = 1, 2, 4

STATUS_NAMES = {0: "XTC_OK", 1: "XTC_WARN_RANK_DEFICIENT", 2: "XTC_WARN_JITTER",
                3: "XTC_WARN_FALLBACK", -1: "XTC_ERR_INVALID_ARG", -2: "XTC_ERR_NOT_SPD",
                -3: "XTC_ERR_HIP", -4: "XTC_ERR_NO_WORKSPACE", -5: "XTC_ERR_UNSUPPORTED"}

P = C.c_void_p
D = C.POINTER(C.c_double)
I32 = C.POINTER(C.c_int32)
I64 = C.POINTER(C.c_int64)


class Grid(C.Structure):
    _fields_ = [("n_g", C.c_int64), ("xyz", P), ("w", P)]


class Basis(C.Structure):
    _fields_ = [("n_atom", C.c_int32), ("atom_xyz", D), ("n_shell", C.c_int32),
                ("shell_center", I32), ("shell_l", I32), ("shell_prim_start", I32),
                ("prim_exp", D), ("prim_coef", D), ("comp_factor", D), ("n_ao", C.c_int32)]


class Correlator(C.Structure):
    _fields_ = [("form", C.c_int32), ("n_terms", C.c_int32), ("mno", I32), ("n_types", C.c_int32),
                ("c", D), ("d", C.c_double), ("b", D), ("n_nuc", C.c_int32), ("nuc_xyz", D),
                ("nuc_type", I32)]


class Exchange(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("phi_piv", P), ("n_q", C.c_int32), ("lq", P), ("X2", P),
                ("X3", P)]


class XiSource(C.Structure):
    _fields_ = [("xi_prec", C.c_int32), ("phi4", P), ("n_orb", C.c_int32), ("chol", P),
                ("rhot", P)]


class Assembly(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_mu", C.c_int32), ("phi4_piv", P), ("u1", P), ("u3", P),
                ("D1", P), ("D4", P), ("X2", P), ("X3", P)]


class VmcSystem(C.Structure):
    _fields_ = [("basis", C.POINTER(Basis)), ("n_occ", C.c_int32), ("C_occ", P), ("n_nuc", C.c_int32),
                ("nuc_xyz", D), ("nuc_charge", D), ("e_nuc", C.c_double)]


class Mlp(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("hidden", C.c_int32), ("params", P), ("feat_shift", P),
                ("feat_scale", P), ("kappa", C.c_double), ("n_nuc", C.c_int32), ("nuc_xyz", D),
                ("judge", C.c_int32), ("ref_a", C.c_double), ("ref_b", C.c_double),
                ("stride", C.c_int32), ("bf16", C.c_int32)]


_lib = None


class NativeMissing(RuntimeError):
    pass


def lib() -> C.CDLL:
    """The loaded native library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NativeMissing(f"{LIB_PATH} not found: build it with `python -m paper_2607_17314_amd.build` "
                            "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    st = C.c_int32
    L.xtc_last_error.restype = C.c_char_p
    L.xtc_version.restype = C.c_char_p
    L.xtc_workspace_bytes.restype = C.c_size_t
    L.xtc_workspace_bytes.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_uint32]
    L.xtc_eval_orbitals.restype = st
    L.xtc_eval_orbitals.argtypes = [C.POINTER(Basis), C.POINTER(Grid), P, C.c_int32, C.c_int32, P, P,
                                    P, C.c_size_t, P]
    L.isdf_select_points.restype = st
    L.isdf_select_points.argtypes = [P, C.POINTER(Grid), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.POINTER(Mlp), C.c_double, I64, I32, D, P, C.c_size_t, P]
    L.isdf_fit.restype = st
    L.isdf_fit.argtypes = [P, C.POINTER(Grid), C.c_int32, I64, C.c_int32, C.c_uint32, C.c_int32, P,
                           P, P, P, P, D, P, C.c_size_t, P]
    L.xtc_kernel_contract.restype = st
    L.xtc_kernel_contract.argtypes = [C.POINTER(Grid), C.POINTER(Correlator), C.c_int32, P, P, P, I64,
                                      C.c_uint32, C.c_int32, C.c_int64, C.c_int64, P, P, P, P, P,
                                      P, D, C.POINTER(Exchange), C.POINTER(XiSource), P, C.c_size_t,
                                      P]
    L.xtc_kernel_contract_noalloc.restype = st
    L.xtc_kernel_contract_noalloc.argtypes = [C.POINTER(Grid), C.POINTER(Correlator), C.c_int32, P, P,
                                              P, I64, C.c_uint32, C.c_int32, C.c_int64, C.c_int64,
                                              P, P, P, P, P, P, D, C.POINTER(Exchange),
                                              C.POINTER(XiSource), P]
    L.xtc_grad.restype = st
    L.xtc_grad.argtypes = [C.POINTER(Grid), C.POINTER(Correlator), C.c_int32, P, P, P, I64, C.c_int64,
                           C.c_int64, P, P, P, P, P, P, P, P, P, C.c_size_t, P]
    L.xtc_exchange_terms.restype = st
    L.xtc_exchange_terms.argtypes = [C.POINTER(Grid), C.POINTER(Correlator), C.c_int32, P,
                                     C.c_int32, P, C.c_int32, P, C.c_int32, C.c_int64, C.c_int64,
                                     P, P, P, C.c_size_t, P]
    L.xtc_assembly_prepare.restype = st
    L.xtc_assembly_prepare.argtypes = [C.POINTER(Assembly), C.c_uint32, P, C.c_size_t, P]
    L.xtc_assembly_panel.restype = st
    L.xtc_assembly_panel.argtypes = [C.POINTER(Assembly), C.c_uint32, C.c_int32, C.c_int32, P, P, P,
                                     P, C.c_size_t, P]
    L.xtc_one_body.restype = st
    L.xtc_one_body.argtypes = [C.POINTER(Assembly), C.c_int32, C.c_double, P, P, D, P, C.c_size_t, P]
    L.xtc_vmc_sample.restype = st
    L.xtc_vmc_sample.argtypes = [C.POINTER(VmcSystem), C.c_int64, P, C.c_int32, C.c_double, P, P, P,
                                 P, C.c_size_t, P]
    L.xtc_vmc_local_energy.restype = st
    L.xtc_vmc_local_energy.argtypes = [C.POINTER(VmcSystem), C.POINTER(Correlator), C.c_int64, P, P, P,
                                       P, C.c_size_t, P]
    L.xtc_vmc_gn_step.restype = st
    L.xtc_vmc_gn_step.argtypes = [C.c_int64, C.c_int32, P, P, C.c_double, C.c_double, P, P, P]
    L.xtc_timing.restype = st
    L.xtc_timing.argtypes = [C.c_int32, D]
    L.xtc_mlp_features.restype = st
    L.xtc_mlp_features.argtypes = [P, C.POINTER(Grid), C.c_int32, C.c_int32, C.c_int32, D, P, P,
                                   C.c_size_t, P]
    L.xtc_mlp_forward.restype = st
    L.xtc_mlp_forward.argtypes = [C.POINTER(Mlp), P, C.c_int64, C.c_int64, P, P]
    L.xtc_mlp_loss_grad.restype = st
    L.xtc_mlp_loss_grad.argtypes = [C.POINTER(Mlp), P, C.c_int64, C.c_int64, P, C.c_float, P, P, P,
                                    C.c_size_t, P]
    L.xtc_adam_step.restype = st
    L.xtc_adam_step.argtypes = [P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float,
                                C.c_int32, P]
    _lib = L
    return L


EXPORTED = ["xtc_last_error", "xtc_version", "xtc_workspace_bytes", "xtc_eval_orbitals",
            "isdf_select_points", "isdf_fit", "xtc_kernel_contract", "xtc_kernel_contract_noalloc",
            "xtc_grad", "xtc_timing",
            "xtc_exchange_terms", "xtc_assembly_prepare", "xtc_assembly_panel", "xtc_one_body",
            "xtc_mlp_features", "xtc_mlp_forward", "xtc_mlp_loss_grad", "xtc_adam_step",
            "xtc_vmc_sample", "xtc_vmc_local_energy", "xtc_vmc_gn_step"]
TIMING_CATEGORIES = ["stage1", "stage2", "select", "fit", "orbitals", "grad", "mlp", "split_prep",
                     "stage1_kernel", "x_pairs", "x_gemm", "x_stage1", "x_mfma", "asm_panel",
                     "vmc_sample", "vmc_energy", "vmc_gn", "bh_pairs"]
