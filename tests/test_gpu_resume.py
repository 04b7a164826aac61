"""Resume from exported fields (checkpoint / restart through the C ABI).

A run of 10 steps against 6 steps, export of the state (positions,
velocities, potential, masses in the caller's order, time from sph_stats),
a fresh context from it (sph_set_time) and 4 more steps.  The library orders
particles by (cell, original index) at every sort and recomputes everything
else from the state, so the FP64 path resumes bit for bit: with fixed walls,
with a moving body (given, as always, at its reference time) and with kept
candidate lists (the resumed context builds them at its first stage, as the
uninterrupted one does at the start of every step).  Two identical runs are
bitwise equal as well.
"""
import numpy as np
import pytest

import workloads as wl
from test_gpu_parity import _flags_all

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


def _cases():
    dyn = wl.random_velocity(wl.jitter(wl.tank2d(dx=0.01, **_flags_all()), 0.1, 41), 0.05, 42)
    body = wl.random_velocity(wl.jitter(wl.entry2d(**_flags_all()), 0.1, 43), 0.05, 44)
    box = wl.random_velocity(wl.jitter(wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2), **_flags_all()), 0.1, 45),
                             0.05, 46)
    kept = wl.with_params(box, cell_size=1.01 * box["params"]["h"], keep_lists=True)
    return [("tank2d-dyn", dyn), ("entry2d-body", body), ("box3d-kept-lists", kept)]


CASES = _cases()


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_resume_is_bit_exact(Sim, name, case):
    a = Sim(case)
    a.step(10)
    b = Sim(case)
    b.step(6)
    d = case["kind"] != 0
    saved = dict(case)
    for k in ("x", "u", "phi", "mass"):
        v = b.field(k)
        if k in ("x", "u", "phi"):
            v[d] = case[k][d]  # walls and the body as given
        saved[k] = v
    saved["t"] = b.stats()["t"]
    b.close()
    c = Sim(saved)
    c.step(4)
    f = case["kind"] == 0
    for k in ("x", "u", "phi", "dudt", "dphidt", "nnb", "fs"):
        assert np.array_equal(a.field(k)[f], c.field(k)[f]), k
    assert a.stats()["t"] == c.stats()["t"]
    if (case["kind"] == 2).any():
        bd = case["kind"] == 2
        assert np.array_equal(a.field("x")[bd], c.field("x")[bd])


@pytest.mark.parametrize("name,case", [CASES[2], ("box3d-kept-lists mixed", wl.with_params(CASES[2][1],
                                                                                            precision="mixed"))],
                         ids=[CASES[2][0], "box3d-kept-lists-mixed"])
def test_two_runs_are_bit_identical(Sim, name, case):
    """Run-to-run determinism: the counting sort's atomic slots are
    reordered by original index in every cell, the reductions are maxima and
    integer counts, so two runs give the same bits."""
    a = Sim(case)
    b = Sim(case)
    a.step(8)
    b.step(8)
    for k in ("x", "u", "phi", "dudt", "dphidt", "nnb", "fs", "lambda"):
        assert np.array_equal(a.field(k), b.field(k)), k
    assert a.stats()["t"] == b.stats()["t"]
