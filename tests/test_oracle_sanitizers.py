"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_driver.c compiles the oracle into a standalone
program (gcc -fsanitize=address,undefined, no recovery, no OpenMP) that
evaluates one right-hand side and a few steps of a case read from a file.
Cases: the dynamic 2D tank with every stabiliser, the 2D body entry (moving
walls), a 3D box.  The run must end cleanly, and its results must equal the
oracle library's bit for bit (same code, contraction off).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "sanitize", "oracle_driver.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fno-fast-math", DRIVER, "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _flags():
    return dict(delta_sph=True, pst=True, tic=True, fs_project=True, cont_uncorr=True, fs_mode="exact")


CASES = [
    ("tank2d-dyn", wl.random_velocity(wl.jitter(wl.tank2d(dx=0.02, **_flags()), 0.1, 51), 0.05, 52)),
    ("entry2d-body", wl.random_velocity(wl.jitter(wl.entry2d(dx=0.02, **_flags()), 0.1, 53), 0.05, 54)),
    ("box3d", wl.random_velocity(wl.jitter(wl.box3d(0.04, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2), **_flags()), 0.1, 55),
                                 0.05, 56)),
]


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_oracle_clean_under_sanitizers(driver, tmp_path, name, case):
    dim, n, x, u, phi, m, kind, nd = oracle._state(case)
    p = oracle.make_params(case["params"])
    nsteps = 3
    t = float(case.get("t", 0.0))
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        f.write(np.int64(n).tobytes() + np.int32(dim).tobytes() + np.int32(nsteps).tobytes() + np.float64(t).tobytes())
        f.write(bytes(p))
        for a in (x, u, phi, m, kind, nd):
            f.write(np.ascontiguousarray(a).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([driver, fin, fout], env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr
    raw = open(fout, "rb").read()
    off = 0

    def take(count, dtype):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off)
        off += a.nbytes
        return a

    acc = take(n * dim, np.float64).reshape(n, dim)
    dphi = take(n, np.float64)
    nnb = take(n, np.int32)
    xs = take(n * dim, np.float64).reshape(n, dim)
    us = take(n * dim, np.float64).reshape(n, dim)
    ps = take(n, np.float64)
    ref = oracle.eval_rates(case)
    assert np.array_equal(acc, ref["acc"]) and np.array_equal(dphi, ref["dphi"]) and np.array_equal(nnb, ref["nnb"])
    st = oracle.step(case, nsteps)
    assert np.array_equal(xs, st["x"]) and np.array_equal(us, st["u"]) and np.array_equal(ps, st["phi"])
