"""The library driven from plain C (paper_2608_22269_amd/examples/run_case.c,
built with gcc against the HIP runtime API): the program allocates its own
workspace and stream, creates a context from host arrays, runs sph_step and
writes the fields; the result matches the oracle at the trajectory bars.
Nothing of PyTorch or of the Python binding takes part in the run."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as wl
from c_caller import EXAMPLE, read_output, write_case
from test_gpu_parity import _flags_all

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

CASES = [
    ("tank2d-dyn", wl.random_velocity(wl.jitter(wl.tank2d(dx=0.02, **_flags_all()), 0.1, 71), 0.05, 72), 10),
    ("dambreak3d-mini", wl.dambreak3d(dx=0.04, tank=(0.8, 0.4, 0.4), column=(0.3, 0.4, 0.22)), 6),
    ("tank2d-mixed", wl.with_params(wl.jitter(wl.tank2d(dx=0.02, **_flags_all()), 0.1, 73), precision="mixed"), 4),
]


@pytest.mark.parametrize("name,case,nsteps", CASES, ids=[c[0] for c in CASES])
def test_c_caller_matches_oracle(tmp_path, name, case, nsteps):
    assert os.path.exists(EXAMPLE), "run __graft_entry__.build() first"
    cf, of = tmp_path / "case.bin", tmp_path / "out.bin"
    write_case(cf, case, nsteps)
    print(name, flush=True)
    r = subprocess.run([EXAMPLE, str(cf), str(of)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = read_output(of)
    ref = oracle.step(case, nsteps)
    assert out["steps"] == nsteps
    f = case["kind"] == 0
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    umax = max(np.abs(ref["u"][f]).max(), 1e-3)
    pmax = np.abs(ref["phi"][f]).max()
    dx = np.abs(out["x"][f] - ref["x"][f]).max()
    du = np.abs(out["u"][f] - ref["u"][f]).max() / umax
    dp = np.abs(out["phi"][f] - ref["phi"][f]).max() / pmax
    print(f"|dx| {dx:.2e} m, rel |dU| {du:.2e}, rel |dphi| {dp:.2e}")
    if case["params"].get("precision", "fp64") == "fp64":  # the trajectory bars
        assert abs(out["t"] - ref["t"]) <= 1e-15
        assert dx <= 1e-12 * L and du <= 1e-12 and dp <= 1e-12
    else:  # the mixed path's trajectory bars (the FP32 resolution of its state)
        assert abs(out["t"] - ref["t"]) <= 1e-12
        assert dx <= 1e-7 and du <= 1e-4 and dp <= 1e-4
