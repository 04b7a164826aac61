"""Front end of the learned free-surface classifier entry points of the C ABI
(training object, BF16 inference) and of the data it learns from.  All
arithmetic runs in libwbsph.so; this module marshals torch device buffers."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from .sim import Simulation, _check, device_buffer

NFEAT = 16
NPARAM = L.MLP_NPARAM


def _dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    return t if dtype is None else t.to(dtype)


class MLPTrainer:
    """FP32 trainer (hand-written HIP forward, backward and Adam kernels)."""

    def __init__(self, params0, mean, std, max_batch=4096, stream=None):
        import torch
        self.torch = torch
        lib = L.lib()
        nbytes = lib.sph_mlp_workspace_bytes(int(max_batch))
        if nbytes == 0:
            raise L.SphError(L.SPH_EINVAL, "sph_mlp_workspace_bytes")
        self._ws, ptr = device_buffer(nbytes)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p0 = np.ascontiguousarray(params0, dtype=np.float32)
        mu = np.ascontiguousarray(mean, dtype=np.float32)
        sd = np.ascontiguousarray(std, dtype=np.float32)
        self.mean, self.std = mu, sd
        h = C.c_void_p()
        pp = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(lib.sph_mlp_create(int(max_batch), pp(p0), pp(mu), pp(sd), C.c_void_p(ptr), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)), "sph_mlp_create")
        self.h = h
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "h", None):
            L.lib().sph_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, X):
        X = _dev(X, self.torch.float32)
        out = self.torch.empty(X.shape[0], dtype=self.torch.float32, device="cuda")
        _check(L.lib().sph_mlp_forward(self.h, C.c_void_p(X.data_ptr()), X.shape[0], C.c_void_p(out.data_ptr())),
               "sph_mlp_forward")
        return out.cpu().numpy()

    def loss_grad(self, X, y, w=None):
        torch = self.torch
        X = _dev(X, torch.float32)
        y = _dev(y, torch.float32)
        wd = None if w is None else _dev(w, torch.float32)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        grad = torch.empty(NPARAM, dtype=torch.float32, device="cuda")
        _check(L.lib().sph_mlp_loss_grad(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                                         C.c_void_p(wd.data_ptr()) if wd is not None else None, X.shape[0],
                                         C.c_void_p(loss.data_ptr()), C.c_void_p(grad.data_ptr())),
               "sph_mlp_loss_grad")
        return float(loss.item()), grad.cpu().numpy()

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(L.lib().sph_mlp_adam(self.h, lr, beta1, beta2, eps), "sph_mlp_adam")

    def train_epoch(self, Xd, yd, wd, perm_d, batch, lr):
        """One epoch over device tensors (X n x 16 f32, y, w f32, perm int32)."""
        ml = C.c_float(0.0)
        _check(L.lib().sph_mlp_train_epoch(self.h, C.c_void_p(Xd.data_ptr()), C.c_void_p(yd.data_ptr()),
                                           C.c_void_p(wd.data_ptr()) if wd is not None else None,
                                           C.c_void_p(perm_d.data_ptr()), Xd.shape[0], int(batch), float(lr),
                                           C.byref(ml)), "sph_mlp_train_epoch")
        return ml.value

    def params(self):
        out = np.empty(NPARAM, dtype=np.float32)
        _check(L.lib().sph_mlp_get_params(self.h, out.ctypes.data_as(C.c_void_p), 0), "sph_mlp_get_params")
        return out


def infer_bf16(params, mean, std, X, stream=None):
    """Logits of the rows of X with BF16 MFMA inference (device tensors or arrays)."""
    import torch
    w = _dev(params, torch.float32)
    mu = _dev(mean, torch.float32)
    sd = _dev(std, torch.float32)
    Xd = X if isinstance(X, torch.Tensor) else _dev(X, torch.float32)
    out = torch.empty(Xd.shape[0], dtype=torch.float32, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(L.lib().sph_mlp_infer_bf16(C.c_void_p(w.data_ptr()), C.c_void_p(mu.data_ptr()), C.c_void_p(sd.data_ptr()),
                                      C.c_void_p(Xd.data_ptr()), Xd.shape[0], C.c_void_p(out.data_ptr()),
                                      C.c_void_p(s.cuda_stream)), "sph_mlp_infer_bf16")
    return out


def forward_noalloc(params, mean, std, X, stream=None):
    """FP32 logits of the rows of X through sph_mlp_forward_noalloc (the
    trainer's forward pass without a trainer or workspace; at most
    SPH_MLP_NOALLOC_MAX_ROWS rows).  Returns a device tensor."""
    import torch
    w = _dev(params, torch.float32)
    mu = _dev(mean, torch.float32)
    sd = _dev(std, torch.float32)
    Xd = X if isinstance(X, torch.Tensor) else _dev(X, torch.float32)
    out = torch.empty(Xd.shape[0], dtype=torch.float32, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(L.lib().sph_mlp_forward_noalloc(C.c_void_p(w.data_ptr()), C.c_void_p(mu.data_ptr()),
                                           C.c_void_p(sd.data_ptr()), C.c_void_p(Xd.data_ptr()), Xd.shape[0],
                                           C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)),
           "sph_mlp_forward_noalloc")
    return out


def candidate_samples(sim: Simulation):
    """Features and exact labels of the particles the scan-region pass decided
    in the last right-hand side (lambda between the two thresholds)."""
    path = sim.field("fs_path")
    sel = path == 1
    feats = sim.field("features")[sel]
    labels = sim.field("fs")[sel].astype(np.float32)
    return feats, labels
