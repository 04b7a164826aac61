"""Thin Python front end of the C ABI: torch provides the device workspace and
the stream; every computation happens in libwbsph.so."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L

_DTYPES = {
    "x": np.float64, "u": np.float64, "phi": np.float64, "rho": np.float64, "p": np.float64,
    "dudt": np.float64, "dphidt": np.float64, "delta_u": np.float64, "lambda": np.float64,
    "normal": np.float64, "mass": np.float64, "fs": np.int32, "tic": np.int32, "nnb": np.int32,
    "cell": np.int32, "features": np.float32, "mirror_src": np.int32, "logit": np.float32, "fs_path": np.int32,
}


def _width(name, dim):
    if name in ("x", "u", "dudt", "delta_u", "normal"):
        return dim
    if name in ("lambda", "cell"):
        return 3
    if name == "features":
        return 16
    return 1


def _check(code, what, ctx=None):
    if code != L.SPH_OK:
        detail = ""
        if ctx:
            detail = L.lib().sph_last_error(ctx).decode()
        raise L.SphError(code, what, detail or L.status_string(code))


def device_buffer(nbytes: int, device="cuda"):
    """A torch uint8 tensor whose data pointer is 256-byte aligned."""
    import torch
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


class Simulation:
    """One context of the library over a workload dictionary (see workloads)."""

    def __init__(self, case: dict, device="cuda", stream=None, device_inputs=False, **overrides):
        """device_inputs: hand sph_init device copies of the particle arrays
        (its inputs_on_device path) instead of host arrays."""
        import torch
        self.torch = torch
        pd = dict(case["params"])
        pd.update(overrides)
        self.params = pd
        self.dim = int(pd["dim"])
        self.p = L.params_from_dict(pd, case.get("body"))
        lib = L.lib()
        _check(lib.sph_validate(C.byref(self.p)), "sph_validate")
        kind = np.ascontiguousarray(case["kind"], dtype=np.uint8)
        self.n = int(kind.shape[0])
        self.nf = int((kind == 0).sum())
        self.nd = self.n - self.nf
        nbytes = lib.sph_workspace_bytes(C.byref(self.p), self.nf, self.nd)
        if nbytes == 0:
            raise L.SphError(L.SPH_EINVAL, "sph_workspace_bytes")
        self.device = torch.device(device)
        self._ws, ptr = device_buffer(nbytes, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        x = np.ascontiguousarray(case["x"], dtype=np.float64)
        u = np.ascontiguousarray(case["u"], dtype=np.float64)
        phi = np.ascontiguousarray(case["phi"], dtype=np.float64)
        nrm = np.ascontiguousarray(case["normal"], dtype=np.float64)
        m = case.get("mass")
        m = None if m is None else np.ascontiguousarray(m, dtype=np.float64)
        ctx = C.c_void_p()
        if device_inputs:
            held = [torch.from_numpy(a).to(self.device) if a is not None else None for a in (x, u, phi, m, kind, nrm)]
            torch.cuda.synchronize(self.device)
            p_ = lambda a: C.c_void_p(a.data_ptr()) if a is not None else None
            x_, u_, phi_, m_, kind_, nrm_ = held
            st = lib.sph_init(C.byref(self.p), self.n, p_(x_), p_(u_), p_(phi_), p_(m_), p_(kind_), p_(nrm_), 1,
                              C.c_void_p(ptr), nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
            self.stream.synchronize()
            del held
        else:
            p_ = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
            st = lib.sph_init(C.byref(self.p), self.n, p_(x), p_(u), p_(phi), p_(m), p_(kind), p_(nrm), 0,
                              C.c_void_p(ptr), nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        _check(st, "sph_init")
        self.ctx = ctx
        t0 = float(case.get("t", 0.0))
        if t0 != 0.0:
            self.set_time(t0)

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            L.lib().sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- hot path
    def build_cells(self):
        _check(L.lib().sph_build_cells(self.ctx), "sph_build_cells", self.ctx)

    def step(self, nsteps=1, dt=0.0):
        _check(L.lib().sph_step(self.ctx, int(nsteps), float(dt)), "sph_step", self.ctx)

    def eval_rates(self):
        _check(L.lib().sph_eval_rates(self.ctx), "sph_eval_rates", self.ctx)

    def set_time(self, t):
        _check(L.lib().sph_set_time(self.ctx, float(t)), "sph_set_time", self.ctx)

    def sync(self):
        _check(L.lib().sph_sync(self.ctx), "sph_sync", self.ctx)

    # -- outputs
    def field(self, name):
        w = _width(name, self.dim)
        out = np.empty((self.n, w) if w > 1 else (self.n,), dtype=_DTYPES[name])
        st = L.lib().sph_fields(self.ctx, L.FIELDS[name], out.ctypes.data_as(C.c_void_p), 0)
        _check(st, f"sph_fields({name})", self.ctx)
        return out

    def field_device(self, name, out_tensor):
        st = L.lib().sph_fields(self.ctx, L.FIELDS[name], C.c_void_p(out_tensor.data_ptr()), 1)
        _check(st, f"sph_fields({name})", self.ctx)
        return out_tensor

    def stats(self):
        out = np.zeros(20)
        _check(L.lib().sph_stats(self.ctx, out.ctypes.data_as(C.c_void_p)), "sph_stats", self.ctx)
        keys = ["t", "dt", "steps", "umax", "n_fluid", "n_dummy", "n_fs", "n_cons", "n_scan", "n_mlp",
                "n_singular", "pairs", "n_cand", "tests", "n_kept", "n_rebuilt", "pairs_search", "tests_search",
                "pairs_kept", "tests_kept"]
        return {k: float(out[i]) for i, k in enumerate(keys)}

    def body_state(self):
        """The free body's state and the water's force and torque of the last
        right-hand side: {"c", "q", "v", "w", "force", "torque"}."""
        out = np.zeros(19)
        _check(L.lib().sph_body_state(self.ctx, out.ctypes.data_as(C.c_void_p)), "sph_body_state", self.ctx)
        return {"c": out[0:3].copy(), "q": out[3:7].copy(), "v": out[7:10].copy(), "w": out[10:13].copy(),
                "force": out[13:16].copy(), "torque": out[16:19].copy()}

    def profile(self, enable=True):
        _check(L.lib().sph_profile(self.ctx, int(bool(enable))), "sph_profile", self.ctx)

    def profile_read(self):
        out = np.zeros(16)
        _check(L.lib().sph_profile_read(self.ctx, out.ctypes.data_as(C.c_void_p)), "sph_profile_read", self.ctx)
        names = ["pair", "mirror", "rebuild", "fs_detect", "stage", "pair_kept"]
        return {k: {"ms": float(out[2 * i]), "launches": int(out[2 * i + 1])} for i, k in enumerate(names)}

    def neighbors(self):
        lib = L.lib()
        off = np.zeros(self.n + 1, dtype=np.int64)
        need = C.c_int64(0)
        st = lib.sph_neighbors(self.ctx, off.ctypes.data_as(C.c_void_p), None, 0, C.byref(need))
        if st not in (L.SPH_OK, L.SPH_ECAPACITY):
            _check(st, "sph_neighbors", self.ctx)
        ids = np.zeros(max(need.value, 1), dtype=np.int32)
        st = lib.sph_neighbors(self.ctx, off.ctypes.data_as(C.c_void_p), ids.ctypes.data_as(C.c_void_p),
                               need.value, C.byref(need))
        _check(st, "sph_neighbors", self.ctx)
        return off, ids[: need.value]

    def set_classifier(self, params, mean, std, margin):
        params = np.ascontiguousarray(params, dtype=np.float32)
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        std = np.ascontiguousarray(std, dtype=np.float32)
        st = L.lib().sph_set_classifier(self.ctx, params.ctypes.data_as(C.c_void_p), params.size,
                                        mean.ctypes.data_as(C.c_void_p), std.ctypes.data_as(C.c_void_p),
                                        float(margin))
        _check(st, "sph_set_classifier", self.ctx)
