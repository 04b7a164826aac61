"""Case and output files of the plain C caller (paper_2608_22269_amd/examples/
run_case.c); the format is stated in that file's header."""
import ctypes as C
import os
import struct

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "paper_2608_22269_amd", "lib", "run_case")


def write_case(path, case, nsteps):
    from paper_2608_22269_amd import _lib
    p = _lib.params_from_dict(case["params"], case.get("body"))
    x = np.ascontiguousarray(case["x"], np.float64)
    n, dim = x.shape
    with open(path, "wb") as f:
        f.write(b"WBSPHCS1")
        f.write(struct.pack("<Q", C.sizeof(p)))
        f.write(bytes(p))
        f.write(struct.pack("<qii", n, dim, nsteps))
        f.write(x.tobytes())
        f.write(np.ascontiguousarray(case["u"], np.float64).tobytes())
        f.write(np.ascontiguousarray(case["phi"], np.float64).tobytes())
        f.write(np.ascontiguousarray(case["kind"], np.uint8).tobytes())
        f.write(np.ascontiguousarray(case["normal"], np.float64).tobytes())


def read_output(path):
    with open(path, "rb") as f:
        assert f.read(8) == b"WBSPHOUT"
        n, dim, steps, t = struct.unpack("<qiid", f.read(24))
        x = np.frombuffer(f.read(8 * n * dim), np.float64).reshape(n, dim)
        u = np.frombuffer(f.read(8 * n * dim), np.float64).reshape(n, dim)
        phi = np.frombuffer(f.read(8 * n), np.float64)
    return {"x": x, "u": u, "phi": phi, "steps": steps, "t": t}
