"""The C-ABI library loads on a machine without a GPU, exports every symbol
include/wbsph.h declares, and rejects bad inputs on the host before any
device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2608_22269_amd import _lib
    _lib.lib()
    return _lib


def _declared():
    src = open(os.path.join(ROOT, "include", "wbsph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(L.exported_symbols()) == names


def test_validate_and_workspace(L):
    lib = L.lib()
    c = wl.tank2d()
    p = L.params_from_dict(c["params"])
    assert lib.sph_validate(C.byref(p)) == L.SPH_OK
    assert lib.sph_workspace_bytes(C.byref(p), 5000, 678) > 0
    for field, val in (("dim", 4), ("h", -1.0), ("cfl", 0.0), ("precision", 7), ("fs_mode", 9)):
        q = L.params_from_dict(c["params"])
        setattr(q, field, val)
        assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
        assert lib.sph_workspace_bytes(C.byref(q), 10, 10) == 0
    q = L.params_from_dict(c["params"])
    q.cell_size = 0.5 * q.h  # reach 4 > 3
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    q = L.params_from_dict(c["params"])
    q.flags |= 512  # no such flag
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    q = L.params_from_dict(c["params"])
    q.flags |= L.SPH_F_GRAPH
    assert lib.sph_validate(C.byref(q)) == L.SPH_OK
    q.flags |= L.SPH_F_KEEP_LISTS  # their reuse test reads the device between stages
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    q = L.params_from_dict(c["params"])
    q.flags |= L.SPH_F_KEEP_ACROSS_STEPS  # needs SPH_F_KEEP_LISTS
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    q.flags |= L.SPH_F_KEEP_LISTS
    assert lib.sph_validate(C.byref(q)) == L.SPH_OK


def test_kept_lists_workspace(L):
    """SPH_F_KEEP_LISTS adds about 1 KiB per fluid particle (8 chunks of 32
    entries per lane, counts and chunk counts) when the cells have room for a
    skin (either precision), nothing otherwise."""
    lib = L.lib()
    c = wl.tank2d()
    h = c["params"]["h"]
    nf, nd = 5000, 678
    lanes = -(-nf // 256) * 256

    def ws(**kw):
        q = L.params_from_dict(wl.with_params(c, **kw)["params"])
        assert lib.sph_validate(C.byref(q)) == L.SPH_OK
        return lib.sph_workspace_bytes(C.byref(q), nf, nd)

    base = ws(cell_size=2.1 * h)
    kept = ws(cell_size=2.1 * h, keep_lists=True)
    extra = 8 * 32 * lanes * 4 + lanes * 8
    assert extra <= kept - base <= extra + 3 * 256
    assert ws(cell_size=2.0 * h, keep_lists=True) == ws(cell_size=2.0 * h)  # reach R - 2h = 0: no room
    mixed = ws(cell_size=2.1 * h, keep_lists=True, precision="mixed") - ws(cell_size=2.1 * h, precision="mixed")
    assert extra <= mixed <= extra + 3 * 256


def test_body_motion_validation_and_workspace(L):
    """The prescribed body motion: 1..4 pieces with strictly increasing, finite
    breakpoints and finite coefficients; a moving body adds a second buffer
    for the dummies and their reference positions, and no kept lists."""
    lib = L.lib()
    c = wl.entry2d()
    p = L.params_from_dict(c["params"])
    assert p.body_pieces == 2
    assert lib.sph_validate(C.byref(p)) == L.SPH_OK
    for field, val in (("body_pieces", 5), ("body_pieces", -1)):
        q = L.params_from_dict(c["params"])
        setattr(q, field, val)
        assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    q = L.params_from_dict(c["params"])
    q.body_t[1] = q.body_t[0]
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    q = L.params_from_dict(c["params"])
    q.body_b[1][0] = float("nan")
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL
    nf, nd = 1770, 558
    still = L.params_from_dict({k: v for k, v in c["params"].items() if not k.startswith("body_")})
    extra = lib.sph_workspace_bytes(C.byref(p), nf, nd) - lib.sph_workspace_bytes(C.byref(still), nf, nd)
    # per dummy: the second buffer (x, n: 4 doubles; m, phi_in; id, src), the
    # reference positions and motion flags of both buffers; per particle: the
    # staging of the reference positions and flags at init; alignment
    per = 8 * 4 + 8 + 8 + 4 + 4 + 2 * (8 * 2 + 1)
    assert nd * per <= extra <= nd * per + (8 * 2 + 1) * (nf + nd) + 16 * 256
    h = c["params"]["h"]
    kept = L.params_from_dict(wl.with_params(c, keep_lists=True, cell_size=2.1 * h)["params"])
    plain = L.params_from_dict(wl.with_params(c, cell_size=2.1 * h)["params"])
    assert lib.sph_workspace_bytes(C.byref(kept), nf, nd) == lib.sph_workspace_bytes(C.byref(plain), nf, nd)


def _free_case():
    c = wl.tank2d(dx=0.02, width=1.0, depth=0.6, wall_height=0.7)
    return wl.with_free_body(c, (0.4, 0.2), (0.6, 0.32), 1500.0)


def test_free_body_validation_and_workspace(L):
    """The free body: any precision, no prescribed motion beside it,
    positive mass, a positive definite inertia tensor, a unit quaternion,
    planar motion in 2D; it adds the reference normals and the force
    partials to the moving body's workspace."""
    lib = L.lib()
    c = _free_case()
    p = L.params_from_dict(c["params"], c["body"])
    assert p.body_free == 1 and p.body_state0[3] == 1.0
    assert lib.sph_validate(C.byref(p)) == L.SPH_OK
    with pytest.raises(ValueError):
        L.params_from_dict(c["params"])  # no initial state

    def variant(fn):
        q = L.params_from_dict(c["params"], c["body"])
        fn(q)
        return lib.sph_validate(C.byref(q))

    for prec in (L.SPH_MIXED, L.SPH_FP32):
        assert variant(lambda q: setattr(q, "precision", prec)) == L.SPH_OK
    bad = [
        lambda q: setattr(q, "body_pieces", 1),
        lambda q: setattr(q, "body_mass", 0.0),
        lambda q: setattr(q, "body_mass", float("inf")),
        lambda q: q.body_inertia.__setitem__(2, 0.0),
        lambda q: q.body_state0.__setitem__(3, 0.9),          # |q| != 1
        lambda q: q.body_state0.__setitem__(12, float("nan")),
        lambda q: q.body_c0.__setitem__(0, float("nan")),
        lambda q: (q.body_state0.__setitem__(3, 0.6), q.body_state0.__setitem__(4, 0.8)),  # tilts out of plane
        lambda q: q.body_state0.__setitem__(10, 0.5),         # omega_x in 2D
    ]
    for k, fn in enumerate(bad):
        assert variant(fn) == L.SPH_EINVAL, k
    # in-plane turn: accepted
    assert variant(lambda q: (q.body_state0.__setitem__(3, 0.6), q.body_state0.__setitem__(6, 0.8))) == L.SPH_OK
    # 3D: an indefinite tensor is refused, a rotated box accepted
    c3 = wl.with_free_body(wl.box3d(0.04, (0.8, 0.6, 0.8), (0.8, 0.6, 0.6)), (0.28, 0.2, 0.24), (0.52, 0.4, 0.4),
                           1500.0)
    p3 = L.params_from_dict(c3["params"], c3["body"])
    assert lib.sph_validate(C.byref(p3)) == L.SPH_OK
    p3.body_inertia[3] = 2.0 * max(p3.body_inertia[0], p3.body_inertia[1])
    assert lib.sph_validate(C.byref(p3)) == L.SPH_EINVAL
    # workspace: the prescribed body's, plus reference normals (2 buffers x
    # dim doubles), six force partials per block of 256 dummies and the
    # normals' staging at init
    nf, nd = int((c["kind"] == 0).sum()), int((c["kind"] != 0).sum())
    moving = L.params_from_dict(dict({k: v for k, v in c["params"].items() if not k.startswith("body_")},
                                     body_t=[0.0, 1.0], body_a=[[0.0, 0.0, 0.0]], body_b=[[0.0, 0.0, 0.0]]))
    extra = lib.sph_workspace_bytes(C.byref(p), nf, nd) - lib.sph_workspace_bytes(C.byref(moving), nf, nd)
    lo = nd * 2 * 8 * 2 + 6 * 8 * ((nd + 255) // 256)
    assert lo <= extra <= lo + 8 * 2 * (nf + nd) + 16 * 256


def test_single_precision_form_validates_with_kept_lists(L):
    """SPH_FP32 is a valid precision; its kept lists take the workspace of the
    mixed path's; an unknown precision is rejected."""
    lib = L.lib()
    c = wl.tank2d()
    h = c["params"]["h"]
    q = L.params_from_dict(wl.with_params(c, precision="fp32", cell_size=2.1 * h, keep_lists=True)["params"])
    assert q.precision == L.SPH_FP32
    assert lib.sph_validate(C.byref(q)) == L.SPH_OK
    r = L.params_from_dict(wl.with_params(c, precision="mixed", cell_size=2.1 * h, keep_lists=True)["params"])
    assert lib.sph_workspace_bytes(C.byref(q), 5000, 678) == lib.sph_workspace_bytes(C.byref(r), 5000, 678)
    q.precision = 3
    assert lib.sph_validate(C.byref(q)) == L.SPH_EINVAL


def _init(L, case, x=None, u=None, phi=None, kind=None, normal=None, ws=256, ws_bytes=1 << 40):
    lib = L.lib()
    p = L.params_from_dict(case["params"])
    x = case["x"] if x is None else x
    u = case["u"] if u is None else u
    phi = case["phi"] if phi is None else phi
    kind = case["kind"] if kind is None else kind
    normal = case["normal"] if normal is None else normal
    pp = lambda a: a.ctypes.data_as(C.c_void_p)
    ctx = C.c_void_p()
    return lib.sph_init(C.byref(p), len(kind), pp(x), pp(u), pp(phi), None, pp(kind), pp(normal), 0,
                        C.c_void_p(ws), ws_bytes, None, C.byref(ctx))


def test_host_validation_before_any_launch(L):
    c = wl.tank2d(dx=0.05)
    x = c["x"].copy()
    x[2, 1] = 50.0
    assert _init(L, c, x=x) == L.SPH_EDOMAIN
    u = c["u"].copy()
    u[0, 0] = np.nan
    assert _init(L, c, u=u) == L.SPH_ENONFINITE
    k = c["kind"].copy()
    k[0] = 5
    assert _init(L, c, kind=k) == L.SPH_EINVAL
    nrm = c["normal"].copy()
    nrm[-1] = [0.3, 0.3]
    assert _init(L, c, normal=nrm) == L.SPH_EINVAL
    # misaligned workspace
    assert _init(L, c, ws=300) == L.SPH_EWORKSPACE


def test_size_limits(L):
    """The grid's limits (2047 x 2047 x 1023 cells, 2e9 cells with the
    margin) and the particle limit (n < 2^31: 32-bit indices) are refused
    on the host."""
    lib = L.lib()
    c = wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2))
    R = 2.0 * c["params"]["h"]

    def with_cells(ncx, ncy, ncz):
        q = L.params_from_dict(c["params"])
        q.cell_size = R
        for a, nc in enumerate((ncx, ncy, ncz)):
            q.domain_lo[a] = 0.0
            q.domain_hi[a] = (nc - 0.5) * R  # floor(span / R) + 1 = nc cells
        return q

    for a, nmax in enumerate((2047, 2047, 1023)):
        cells = [12, 12, 12]
        cells[a] = nmax
        assert lib.sph_validate(C.byref(with_cells(*cells))) == L.SPH_OK, a
        cells[a] = nmax + 1
        assert lib.sph_validate(C.byref(with_cells(*cells))) == L.SPH_EINVAL, a
    assert lib.sph_validate(C.byref(with_cells(2047, 2047, 400))) == L.SPH_OK
    assert lib.sph_validate(C.byref(with_cells(2047, 2047, 600))) == L.SPH_EINVAL  # 2.6e9 cells
    p = L.params_from_dict(c["params"])
    assert lib.sph_workspace_bytes(C.byref(p), 2 ** 31 - 11, 10) > 0
    assert lib.sph_workspace_bytes(C.byref(p), 2 ** 31 - 10, 10) == 0
    ctx = C.c_void_p()
    assert lib.sph_init(C.byref(p), 2 ** 31, None, None, None, None, None, None, 0, None, 0, None,
                        C.byref(ctx)) == L.SPH_EINVAL
    assert not ctx.value


def test_status_strings(L):
    for code in range(-8, 1):
        assert L.status_string(code)


def test_c_caller_rejects_bad_input(tmp_path):
    """The plain C caller is built next to the library and refuses a
    malformed case file (exit status 2) before it touches a GPU."""
    import subprocess
    from c_caller import EXAMPLE, write_case
    assert os.path.exists(EXAMPLE), "run __graft_entry__.build() first"
    r = subprocess.run([EXAMPLE], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
    bad = tmp_path / "bad.case"
    bad.write_bytes(b"WBSPHCS1" + b"\0" * 8)
    r = subprocess.run([EXAMPLE, str(bad), str(tmp_path / "out")], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "sph_params" in r.stderr
    good = tmp_path / "tank.case"
    write_case(good, wl.tank2d(dx=0.05), 1)
    with open(good, "r+b") as f:  # a truncated file is refused while reading
        f.truncate(os.path.getsize(good) - 8)
    r = subprocess.run([EXAMPLE, str(good), str(tmp_path / "out")], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "cannot read" in r.stderr

