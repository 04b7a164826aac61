"""ctypes binding of libwbsph.so (argument marshalling only).

The names mirror include/wbsph.h.  Loading fails loudly when the library has
not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("WBSPH_LIB") or os.path.join(HERE, "lib", "libwbsph.so")

# status codes
SPH_OK = 0
SPH_EINVAL = -1
SPH_EWORKSPACE = -2
SPH_EHIP = -3
SPH_EDOMAIN = -4
SPH_ENONFINITE = -5
SPH_ESTATE = -6
SPH_EUNSUPPORTED = -7
SPH_ECAPACITY = -8
MLP_NOALLOC_MAX_ROWS = 8192  # SPH_MLP_NOALLOC_MAX_ROWS

SPH_FP64, SPH_MIXED, SPH_FP32 = 0, 1, 2
SPH_FS_NONE, SPH_FS_EXACT, SPH_FS_LEARNED = 0, 1, 2
SPH_F_DELTA, SPH_F_PST, SPH_F_TIC, SPH_F_FS_PROJECT, SPH_F_CONT_UNCORR, SPH_F_FEATURES = 1, 2, 4, 8, 16, 32
SPH_F_KEEP_LISTS = 64
SPH_F_KEEP_ACROSS_STEPS = 128
SPH_F_GRAPH = 256

FIELDS = {
    "x": 0, "u": 1, "phi": 2, "rho": 3, "p": 4, "dudt": 5, "dphidt": 6, "delta_u": 7, "lambda": 8,
    "normal": 9, "fs": 10, "tic": 11, "nnb": 12, "cell": 13, "features": 14, "mass": 15,
    "mirror_src": 16, "logit": 17, "fs_path": 18,
}

MLP_NPARAM = 5313


class SphParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("precision", C.c_int32), ("fs_mode", C.c_int32), ("flags", C.c_uint32),
        ("dx", C.c_double), ("h", C.c_double), ("c0", C.c_double), ("rho0", C.c_double), ("nu", C.c_double),
        ("delta", C.c_double), ("cfl", C.c_double), ("pst_R", C.c_double), ("pst_n", C.c_double),
        ("lambda_tic", C.c_double), ("lambda_fs_lo", C.c_double), ("lambda_fs_hi", C.c_double),
        ("lambda_singular", C.c_double),
        ("gravity", C.c_double * 3), ("forcing_amp", C.c_double * 3), ("forcing_omega", C.c_double),
        ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3), ("cell_size", C.c_double),
        ("body_pieces", C.c_int32), ("body_pad_", C.c_int32), ("body_t", C.c_double * 5),
        ("body_a", (C.c_double * 3) * 4), ("body_b", (C.c_double * 3) * 4),
        ("body_free", C.c_int32), ("body_pad2_", C.c_int32), ("body_mass", C.c_double),
        ("body_inertia", C.c_double * 6), ("body_c0", C.c_double * 3), ("body_state0", C.c_double * 13),
    ]


class SphError(RuntimeError):
    def __init__(self, code, what, detail=""):
        msg = f"{what}: status {code}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    P = C.POINTER(SphParams)
    sig = {
        "sph_validate": (i32, [P]),
        "sph_workspace_bytes": (sz, [P, i64, i64]),
        "sph_status_string": (C.c_char_p, [i32]),
        "sph_init": (i32, [P, i64, vp, vp, vp, vp, vp, vp, i32, vp, sz, vp, C.POINTER(vp)]),
        "sph_destroy": (None, [vp]),
        "sph_last_error": (C.c_char_p, [vp]),
        "sph_build_cells": (i32, [vp]),
        "sph_step": (i32, [vp, i32, C.c_double]),
        "sph_eval_rates": (i32, [vp]),
        "sph_sync": (i32, [vp]),
        "sph_set_time": (i32, [vp, C.c_double]),
        "sph_fields": (i32, [vp, i32, vp, i32]),
        "sph_stats": (i32, [vp, vp]),
        "sph_body_state": (i32, [vp, vp]),
        "sph_neighbors": (i32, [vp, vp, vp, i64, C.POINTER(i64)]),
        "sph_profile": (i32, [vp, i32]),
        "sph_profile_read": (i32, [vp, vp]),
        "sph_set_classifier": (i32, [vp, vp, i64, vp, vp, C.c_float]),
        "sph_mlp_workspace_bytes": (sz, [i64]),
        "sph_mlp_create": (i32, [i64, vp, vp, vp, vp, sz, vp, C.POINTER(vp)]),
        "sph_mlp_destroy": (None, [vp]),
        "sph_mlp_forward": (i32, [vp, vp, i64, vp]),
        "sph_mlp_loss_grad": (i32, [vp, vp, vp, vp, i64, vp, vp]),
        "sph_mlp_adam": (i32, [vp, C.c_float, C.c_float, C.c_float, C.c_float]),
        "sph_mlp_train_epoch": (i32, [vp, vp, vp, vp, vp, i64, i64, C.c_float, C.POINTER(C.c_float)]),
        "sph_mlp_get_params": (i32, [vp, vp, i32]),
        "sph_mlp_infer_bf16": (i32, [vp, vp, vp, vp, i64, vp, vp]),
        "sph_mlp_forward_noalloc": (i32, [vp, vp, vp, vp, i64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names the binding expects the library to export."""
    return [
        "sph_validate", "sph_workspace_bytes", "sph_status_string", "sph_init", "sph_destroy",
        "sph_last_error", "sph_build_cells", "sph_step", "sph_eval_rates", "sph_sync", "sph_set_time", "sph_fields",
        "sph_stats", "sph_body_state", "sph_neighbors", "sph_profile", "sph_profile_read", "sph_set_classifier", "sph_mlp_workspace_bytes", "sph_mlp_create",
        "sph_mlp_destroy", "sph_mlp_forward", "sph_mlp_loss_grad", "sph_mlp_adam", "sph_mlp_train_epoch",
        "sph_mlp_get_params", "sph_mlp_infer_bf16", "sph_mlp_forward_noalloc",
    ]


def params_from_dict(pd: dict, body: dict | None = None) -> SphParams:
    """sph_params from the plain parameter dictionary of a workload; body:
    the free body's initial state {"c", "q", "v", "w"} (with body_free)."""
    p = SphParams()
    p.dim = int(pd["dim"])
    p.precision = {"fp64": SPH_FP64, "mixed": SPH_MIXED, "fp32": SPH_FP32}[pd.get("precision", "fp64")]
    p.fs_mode = {"none": SPH_FS_NONE, "exact": SPH_FS_EXACT, "learned": SPH_FS_LEARNED}[pd.get("fs_mode", "none")]
    p.flags = ((SPH_F_DELTA if pd.get("delta_sph") else 0) | (SPH_F_PST if pd.get("pst") else 0)
               | (SPH_F_TIC if pd.get("tic") else 0) | (SPH_F_FS_PROJECT if pd.get("fs_project") else 0)
               | (SPH_F_CONT_UNCORR if pd.get("cont_uncorr") else 0)
               | (SPH_F_FEATURES if pd.get("features") else 0)
               | (SPH_F_KEEP_LISTS if pd.get("keep_lists") or pd.get("keep_across_steps") else 0)
               | (SPH_F_KEEP_ACROSS_STEPS if pd.get("keep_across_steps") else 0)
               | (SPH_F_GRAPH if pd.get("graph") else 0))
    for k in ("dx", "h", "c0", "rho0", "nu", "delta", "cfl", "pst_R", "pst_n", "lambda_tic", "lambda_fs_lo",
              "lambda_fs_hi", "lambda_singular", "forcing_omega", "cell_size"):
        setattr(p, k, float(pd.get(k, 0.0)))
    for k in ("gravity", "forcing_amp", "domain_lo", "domain_hi"):
        v = list(pd.get(k, [0.0, 0.0, 0.0])) + [0.0] * 3
        setattr(p, k, (C.c_double * 3)(*[float(a) for a in v[:3]]))
    bt = list(pd.get("body_t", []))
    if bt:
        p.body_pieces = len(bt) - 1
        for k, v in enumerate(bt[:5]):
            p.body_t[k] = float(v)
        for name in ("body_a", "body_b"):
            arr = getattr(p, name)
            for k, row in enumerate(list(pd[name])[:4]):
                for c, v in enumerate(list(row)[:3]):
                    arr[k][c] = float(v)
    if pd.get("body_free"):
        if body is None:
            raise ValueError("a free body needs its initial state")
        p.body_free = 1
        p.body_mass = float(pd["body_mass"])
        for k, v in enumerate(list(pd["body_inertia"])[:6]):
            p.body_inertia[k] = float(v)
        for k, v in enumerate(list(pd["body_c0"])[:3]):
            p.body_c0[k] = float(v)
        st = [float(v) for v in (list(body["c"])[:3] + [0.0] * 3)[:3]]
        st += [float(v) for v in body["q"]]
        st += [float(v) for v in (list(body["v"]) + [0.0] * 3)[:3]]
        st += [float(v) for v in (list(body["w"]) + [0.0] * 3)[:3]]
        for k, v in enumerate(st):
            p.body_state0[k] = v
    return p


def status_string(code: int) -> str:
    return lib().sph_status_string(int(code)).decode()
