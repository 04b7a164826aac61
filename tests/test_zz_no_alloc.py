"""The allocation-free entry point sph_mlp_forward_noalloc (activations in
the library's fixed scratch array) against the trainer's sph_mlp_forward
(activations in the trainer's workspace): the same kernel, so the logits
agree bit for bit; two calls in a row, the second smaller, plus the largest
batch, and a batch beyond the maximum rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_forward_equals_trainer_forward():
    import torch
    from paper_2608_22269_amd import _lib as L, learn
    rng = np.random.default_rng(17)
    params = (rng.normal(size=L.MLP_NPARAM) * 0.3).astype(np.float32)
    mean = rng.normal(size=16).astype(np.float32)
    std = (0.5 + rng.random(16)).astype(np.float32)
    nmax = L.MLP_NOALLOC_MAX_ROWS
    tr = learn.MLPTrainer(params, mean, std, max_batch=nmax)
    for B in (5000, 37, nmax, 1):
        X = (rng.normal(size=(B, 16)) * 2.0).astype(np.float32)
        print(f"noalloc forward: B = {B}", flush=True)
        ref = tr.forward(X)
        got = learn.forward_noalloc(params, mean, std, X).cpu().numpy()
        torch.cuda.synchronize()
        assert got.shape == (B,)
        assert np.isfinite(ref).all()
        assert np.array_equal(got, ref), (B, np.abs(got - ref).max())
    tr.close()
    # beyond the maximum (and negative): rejected on the host, nothing launched
    out = torch.zeros(4, device="cuda")
    p = C.c_void_p(out.data_ptr())
    for B in (nmax + 1, -1):
        st = L.lib().sph_mlp_forward_noalloc(p, p, p, p, B, p, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == L.SPH_EINVAL
    torch.cuda.synchronize()
    assert (out == 0).all()
