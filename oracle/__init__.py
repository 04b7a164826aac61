"""CPU oracle for the well-balanced WCSPH hot path -- TEST INFRASTRUCTURE ONLY.

The arithmetic lives in ``wbsph_oracle.c`` (plain C, FP64, contraction off) and
``mlp.py`` (NumPy, FP64).  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library under ``paper_2608_22269_amd`` and never imports it.

This module only marshals arguments (ctypes) and builds the C file with gcc.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wbsph_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

FLAG_DELTA = 1
FLAG_PST = 2
FLAG_TIC = 4
FLAG_FS_PROJECT = 8
FLAG_CONT_UNCORR = 16

FS_NONE = 0
FS_EXACT = 1

NFEAT = 16


def _compile(src: str, out: str) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        _compile(_SRC, _LIB)
    return _LIB


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def build_variant(text: str, workdir: str) -> str:
    """Compiles a variant of the oracle's C source (a test's planted mistake)
    into workdir/liborc_variant.so, with the oracle's own flags."""
    os.makedirs(workdir, exist_ok=True)
    src = os.path.join(workdir, "wbsph_oracle_variant.c")
    with open(src, "w") as f:
        f.write(text)
    return _compile(src, os.path.join(workdir, "liborc_variant.so"))


@contextlib.contextmanager
def using_library(path: str):
    """Routes every call of this module to the library at `path` (a variant
    built by build_variant) inside the with-block."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("fs_mode", C.c_int32), ("flags", C.c_uint32), ("pad_", C.c_uint32),
        ("dx", C.c_double), ("h", C.c_double), ("c0", C.c_double), ("rho0", C.c_double),
        ("nu", C.c_double), ("delta", C.c_double), ("cfl", C.c_double), ("pst_R", C.c_double),
        ("pst_n", C.c_double),
        ("lambda_tic", C.c_double), ("lambda_fs_lo", C.c_double), ("lambda_fs_hi", C.c_double),
        ("lambda_singular", C.c_double),
        ("gravity", C.c_double * 3), ("forcing_amp", C.c_double * 3), ("forcing_omega", C.c_double),
        ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3), ("cell_size", C.c_double),
        ("body_pieces", C.c_int32), ("pad2_", C.c_int32),
        ("body_t", C.c_double * 5), ("body_a", C.c_double * 12), ("body_b", C.c_double * 12),
        ("body_free", C.c_int32), ("pad3_", C.c_int32),
        ("body_mass", C.c_double), ("body_inertia", C.c_double * 6), ("body_c0", C.c_double * 3),
    ]


class Body(C.Structure):
    """State of a free rigid body: centre, unit quaternion (w, x, y, z),
    velocity, angular velocity (world frame)."""
    _fields_ = [("c", C.c_double * 3), ("q", C.c_double * 4), ("v", C.c_double * 3), ("w", C.c_double * 3)]


class _Rates(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in (
        "acc", "dphi", "dushift", "lam", "normal", "fs", "tic", "nnb", "feat", "fs_margin",
        "mir_phi", "mir_u", "mir_src", "scal")]


_lib = None


def _load(path):
    L = C.CDLL(path)
    P = C.POINTER(Params)
    vp = C.c_void_p
    L.orc_W.restype = C.c_double
    L.orc_W.argtypes = [C.c_int, C.c_double, C.c_double]
    L.orc_K.restype = C.c_double
    L.orc_K.argtypes = [C.c_int, C.c_double, C.c_double]
    L.orc_cells.argtypes = [P, C.c_int64, vp, vp, vp]
    L.orc_neighbors_brute.argtypes = [P, C.c_int64, vp, vp, vp, C.c_int64, vp]
    L.orc_neighbors_cells.argtypes = [P, C.c_int64, vp, vp, vp, C.c_int64, vp]
    L.orc_eigvals.argtypes = [C.c_int, vp, vp]
    L.orc_eigvals.restype = None
    L.orc_eval_rates.argtypes = [P, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_double, C.c_int, vp,
                                 C.POINTER(_Rates), C.POINTER(Body)]
    L.orc_dt.restype = C.c_double
    L.orc_dt.argtypes = [P, C.c_int64, vp, vp]
    L.orc_step.argtypes = [P, C.c_int64, vp, vp, vp, vp, vp, vp, C.POINTER(C.c_double),
                           C.c_int32, C.c_double, C.c_int, C.POINTER(C.c_double), C.POINTER(Body)]
    L.orc_body_motion.argtypes = [P, C.c_double, vp, vp]
    L.orc_body_motion.restype = None
    L.orc_num_threads.restype = C.c_int
    L.orc_set_num_threads.argtypes = [C.c_int]
    L.orc_set_num_threads.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _load(_LIB)
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _check(code, what):
    if code != 0:
        raise OracleError(code, what)


def make_params(pd: dict) -> Params:
    """Oracle parameter struct from the plain parameter dictionary produced by
    the workload generators."""
    p = Params()
    p.dim = int(pd["dim"])
    mode = pd.get("fs_mode", "none")
    # the oracle has no learned detector: its reference for "learned" is the exact criterion
    p.fs_mode = FS_NONE if mode == "none" else FS_EXACT
    p.flags = ((FLAG_DELTA if pd.get("delta_sph") else 0) | (FLAG_PST if pd.get("pst") else 0)
               | (FLAG_TIC if pd.get("tic") else 0) | (FLAG_FS_PROJECT if pd.get("fs_project") else 0)
               | (FLAG_CONT_UNCORR if pd.get("cont_uncorr") else 0))
    for k in ("dx", "h", "c0", "rho0", "nu", "delta", "cfl", "pst_R", "pst_n", "lambda_tic",
              "lambda_fs_lo", "lambda_fs_hi", "lambda_singular", "forcing_omega", "cell_size"):
        setattr(p, k, float(pd.get(k, 0.0)))
    for k in ("gravity", "forcing_amp", "domain_lo", "domain_hi"):
        v = list(pd.get(k, [0.0, 0.0, 0.0])) + [0.0] * 3
        setattr(p, k, (C.c_double * 3)(*[float(a) for a in v[:3]]))
    bt = list(pd.get("body_t", []))
    if bt:
        k = len(bt) - 1
        if not 1 <= k <= 4:
            raise ValueError("body motion needs 1 to 4 pieces")
        p.body_pieces = k
        p.body_t = (C.c_double * 5)(*([float(v) for v in bt] + [0.0] * (5 - len(bt))))
        for name in ("body_a", "body_b"):
            rows = [list(r) + [0.0] * 3 for r in pd[name]]
            flat = [float(r[c]) for r in rows[:k] for c in range(3)]
            setattr(p, name, (C.c_double * 12)(*(flat + [0.0] * (12 - len(flat)))))
    if pd.get("body_free"):
        p.body_free = 1
        p.body_mass = float(pd["body_mass"])
        p.body_inertia = (C.c_double * 6)(*[float(v) for v in pd["body_inertia"]])
        c0 = list(pd["body_c0"]) + [0.0] * 3
        p.body_c0 = (C.c_double * 3)(*[float(v) for v in c0[:3]])
    return p


def make_body(state):
    """Body struct from a dict with c, q, v, w (missing components zero)."""
    b = Body()
    for k, nk in (("c", 3), ("q", 4), ("v", 3), ("w", 3)):
        v = list(state.get(k, [1.0, 0.0, 0.0, 0.0] if k == "q" else [0.0] * nk)) + [0.0] * nk
        setattr(b, k, (C.c_double * nk)(*[float(a) for a in v[:nk]]))
    return b


def body_dict(b):
    return {k: np.array(getattr(b, k)[:]) for k in ("c", "q", "v", "w")}


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def W(dim, h, q):
    return lib().orc_W(dim, h, q)


def K(dim, h, q):
    return lib().orc_K(dim, h, q)


def eigvals(dim, S):
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(dim, dim)
    lam = np.zeros(3)
    lib().orc_eigvals(dim, _ptr(S), _ptr(lam))
    return lam[:dim] if dim == 3 else lam[:2]


def cells(pd, x):
    p = make_params(pd)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    cell3 = np.zeros((n, 3), dtype=np.int32)
    hsh = np.zeros(n, dtype=np.int64)
    _check(lib().orc_cells(C.byref(p), n, _ptr(x), _ptr(cell3), _ptr(hsh)), "cells")
    return cell3, hsh


def neighbors(pd, x, mode="cells"):
    """CSR neighbour lists (offsets int64[n+1], ids int32[nnz]).  mode is
    'brute' (O(n^2), ascending j) or 'cells' (Algorithm 1 order)."""
    p = make_params(pd)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    off = np.zeros(n + 1, dtype=np.int64)
    need = C.c_int64(0)
    fn = lib().orc_neighbors_brute if mode == "brute" else lib().orc_neighbors_cells
    st = fn(C.byref(p), n, _ptr(x), _ptr(off), None, 0, C.byref(need))
    if st not in (0, -8):
        _check(st, "neighbors")
    ids = np.zeros(max(need.value, 1), dtype=np.int32)
    _check(fn(C.byref(p), n, _ptr(x), _ptr(off), _ptr(ids), need.value, C.byref(need)), "neighbors")
    return off, ids[: need.value]


def _state(case):
    dim = int(case["params"]["dim"])
    x = np.ascontiguousarray(case["x"], dtype=np.float64).reshape(-1, dim)
    n = x.shape[0]
    u = np.ascontiguousarray(case["u"], dtype=np.float64).reshape(n, dim)
    phi = np.ascontiguousarray(case["phi"], dtype=np.float64).reshape(n)
    kind = np.ascontiguousarray(case["kind"], dtype=np.uint8).reshape(n)
    nd = np.ascontiguousarray(case["normal"], dtype=np.float64).reshape(n, dim)
    m = case.get("mass")
    if m is None:
        m = mass_from_phi(case["params"], phi)
    m = np.ascontiguousarray(m, dtype=np.float64).reshape(n)
    return dim, n, x, u, phi, m, kind, nd


def mass_from_phi(pd, phi):
    """m = rho(phi) dx^d with rho = rho0 exp(phi / C0^2) (Sec. 2.2.1)."""
    dim = int(pd["dim"])
    return pd["rho0"] * np.exp(np.asarray(phi, dtype=np.float64) / (pd["c0"] ** 2)) * pd["dx"] ** dim


def eval_rates(case, t=None, mode="cells", rows=None):
    """One evaluation of the semi-discrete system at the case's state.
    Returns a dict of per-particle arrays in the case's particle order.
    rows: optional indices of the fluid particles to evaluate (the other
    rows of the fluid outputs stay zero); for samples of large cases."""
    dim, n, x, u, phi, m, kind, nd = _state(case)
    p = make_params(case["params"])
    t = float(case.get("t", 0.0) if t is None else t)
    out = {
        "acc": np.zeros((n, dim)), "dphi": np.zeros(n), "dushift": np.zeros((n, dim)),
        "lam": np.zeros((n, 3)), "normal": np.zeros((n, dim)),
        "fs": np.zeros(n, dtype=np.int32), "tic": np.zeros(n, dtype=np.int32),
        "nnb": np.zeros(n, dtype=np.int32), "feat": np.zeros((n, NFEAT)),
        "fs_margin": np.zeros(n), "mir_phi": np.zeros(n), "mir_u": np.zeros((n, dim)),
        "mir_src": np.zeros(n, dtype=np.int32), "scal": np.zeros(10),
    }
    r = _Rates(*[_ptr(out[k]) for k in ("acc", "dphi", "dushift", "lam", "normal", "fs", "tic", "nnb",
                                        "feat", "fs_margin", "mir_phi", "mir_u", "mir_src", "scal")])
    only = None
    if rows is not None:
        only = np.zeros(n, dtype=np.uint8)
        only[np.asarray(rows, dtype=np.int64)] = 1
    body = make_body(case["body"]) if case.get("body") is not None else None
    st = lib().orc_eval_rates(C.byref(p), n, _ptr(x), _ptr(u), _ptr(phi), _ptr(m), _ptr(kind), _ptr(nd),
                              t, 0 if mode == "brute" else 1, _ptr(only) if only is not None else None,
                              C.byref(r), C.byref(body) if body is not None else None)
    _check(st, "eval_rates")
    out["umax"], out["gmag"], out["t"], out["n_singular"] = out["scal"][:4].tolist()
    out["body_force"], out["body_torque"] = out["scal"][4:7].copy(), out["scal"][7:10].copy()
    return out


def body_motion(pd, t):
    """Displacement since T_0 and velocity at t of the prescribed body
    motion (both (3,) arrays)."""
    p = make_params(pd)
    D = np.zeros(3)
    U = np.zeros(3)
    lib().orc_body_motion(C.byref(p), float(t), _ptr(D), _ptr(U))
    return D, U


def dt(case):
    dim, n, x, u, phi, m, kind, nd = _state(case)
    p = make_params(case["params"])
    return lib().orc_dt(C.byref(p), n, _ptr(u), _ptr(kind))


def step(case, nsteps=1, dt_override=0.0, mode="cells"):
    """SSP-RK2 steps from the case state; returns a new case dict holding the
    advanced x, u, phi, t, the (fixed) particle masses and ``dt`` (last step).
    Rows of the moving body keep their positions of time T_0."""
    dim, n, x, u, phi, m, kind, nd = _state(case)
    x, u, phi = x.copy(), u.copy(), phi.copy()
    p = make_params(case["params"])
    t = C.c_double(float(case.get("t", 0.0)))
    dtl = C.c_double(0.0)
    body = make_body(case["body"]) if case.get("body") is not None else None
    st = lib().orc_step(C.byref(p), n, _ptr(x), _ptr(u), _ptr(phi), _ptr(m), _ptr(kind), _ptr(nd),
                        C.byref(t), int(nsteps), float(dt_override), 0 if mode == "brute" else 1,
                        C.byref(dtl), C.byref(body) if body is not None else None)
    _check(st, "step")
    out = dict(case)
    out.update({"x": x, "u": u, "phi": phi, "t": t.value, "mass": m, "dt": dtl.value})
    if body is not None:
        out["body"] = body_dict(body)
    return out


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(k):
    lib().orc_set_num_threads(int(k))
