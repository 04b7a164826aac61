"""Pins of the oracle's free rigid body (kind-2 dummies moving under G(t) and
the water's force and torque; in the cylinder water entry of Sec. 4 the body's
motion results from its weight and the force the water exerts on it).

* free flight away from the water: the centre follows x0 + v0 t + G t^2 / 2
  and the velocity v0 + G t exactly (SSP-RK2 integrates a constant
  acceleration without error);
* torque-free spin of a body with isotropic inertia: the angular velocity
  stays constant and the orientation is the rotation by |w| t about w (the
  quaternion's stage error only); an asymmetric body precesses with its
  world-frame angular momentum and its kinetic energy unchanged;
* pose: the fluid's rates next to a body turned and shifted to a pose equal
  those next to fixed walls placed explicitly at the rotated positions with
  rotated normals (the body at rest): neighbour counts, branches and mirror
  sources exactly, rates to rounding;
* slip relative to the moving wall: each body dummy carries the wall's normal
  velocity, U_d . n = U_w . n with U_w = v + w x (x_d - c), and its source
  particle's tangential velocity;
* Archimedes: a box at rest in hydrostatic water feels rho0 g times its
  volume (area in 2D) upward to 2% (the lattice's kernel moments at fixed
  h/dx), no horizontal force and no torque;
* covariance: turning the whole scene (water, walls, body, gravity) by a
  rotation Q turns the force and the torque by Q;
* the torque's reference point: with the centre moved to c', the torque is
  T + (c - c') x F.
"""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _far_fluid_case(dim, v0, w0, inertia=None):
    """A small fluid block far from a free box body (no fluid within 2h of it)."""
    dx = 0.02
    lo = [-0.4] * dim + [0.0] * (3 - dim)
    hi = [0.8] * dim + [0.0] * (3 - dim)
    pd = wl.base_params(dim, dx, domain_lo=lo, domain_hi=hi)
    xf = wl._lattice([0] * dim, [3] * dim, dx) - 0.2
    n = len(xf)
    case = {"params": pd, "x": xf, "u": np.zeros((n, dim)), "phi": np.zeros(n), "kind": np.zeros(n, np.uint8),
            "normal": np.zeros((n, dim)), "mass": None, "t": 0.0, "meta": {"H": 0.0}}
    body_lo = [0.2] * dim
    body_hi = [0.26] * dim  # a small body: its dummies meet no water
    c = wl.with_free_body(case, body_lo, body_hi, 1200.0, v0=v0, w0=w0)
    if inertia is not None:
        c["params"]["body_inertia"] = inertia
    return c


@pytest.mark.parametrize("dim", [2, 3])
def test_free_flight_is_exact(orc, dim):
    v0 = [0.3, 1.7, -0.4][:dim]
    c = _far_fluid_case(dim, v0, [0.0, 0.0, 0.0])
    dt = 1e-3
    out = orc.step(c, 50, dt_override=dt)
    t = out["t"]
    G = np.asarray(c["params"]["gravity"][:dim])
    c0 = np.asarray(c["body"]["c"][:dim])
    want_c = c0 + np.asarray(v0) * t + 0.5 * G * t * t
    assert np.abs(out["body"]["c"][:dim] - want_c).max() <= 1e-13
    assert np.abs(out["body"]["v"][:dim] - (np.asarray(v0) + G * t)).max() <= 1e-13
    assert np.abs(out["body"]["q"] - [1, 0, 0, 0]).max() == 0.0


def test_torque_free_spin(orc):
    w0 = np.array([0.8, -1.1, 2.3])
    iso = [0.7, 0.7, 0.7, 0.0, 0.0, 0.0]
    c = _far_fluid_case(3, [0.0, 0.0, 0.0], list(w0), inertia=iso)
    c["params"]["gravity"] = [0.0, 0.0, 0.0]
    dt = 2e-4
    out = orc.step(c, 500, dt_override=dt)
    t = out["t"]
    assert np.abs(out["body"]["w"] - w0).max() <= 1e-13
    wn = np.linalg.norm(w0)
    want_q = np.concatenate([[math.cos(0.5 * wn * t)], math.sin(0.5 * wn * t) * w0 / wn])
    # SSP-RK2 on the quaternion: local error O((|w| dt)^3), here ~1e-9 in total
    assert np.abs(out["body"]["q"] - want_q).max() <= 1e-7
    assert abs(np.linalg.norm(out["body"]["q"]) - 1.0) <= 1e-15


def test_torque_free_precession_keeps_angular_momentum(orc):
    """An asymmetric body (principal moments 1, 2, 3 at a turned pose)
    spinning without torque: the angular momentum in the world frame
    R I R^T w and the kinetic energy stay put (Euler's equations), to the
    SSP-RK2 error."""
    Ib = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 3.0]]) * 0.01
    w0 = np.array([1.3, 0.4, -0.9])
    c = _far_fluid_case(3, [0.0, 0.0, 0.0], list(w0), inertia=[0.01, 0.02, 0.03, 0.0, 0.0, 0.0])
    c["params"]["gravity"] = [0.0, 0.0, 0.0]
    q0 = _quat(3, 0.6)
    c["body"] = dict(c["body"], q=q0)

    def momentum(q, w):
        R = _qmat(q)
        Iw = R @ Ib @ R.T
        return Iw @ w, 0.5 * w @ Iw @ w

    L0, E0 = momentum(np.asarray(q0), w0)
    out = orc.step(c, 2000, dt_override=1e-3)
    L1, E1 = momentum(out["body"]["q"], out["body"]["w"])
    assert np.abs(out["body"]["w"] - w0).max() > 0.05  # it does precess
    assert np.abs(L1 - L0).max() <= 1e-5 * np.abs(L0).max()
    assert abs(E1 - E0) <= 1e-5 * E0


def _qmat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _rot(dim, angle, axis=(0.3, -0.5, 0.8)):
    if dim == 2:
        ca, sa = math.cos(angle), math.sin(angle)
        return np.array([[ca, -sa], [sa, ca]])
    a = np.asarray(axis) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def _quat(dim, angle, axis=(0.3, -0.5, 0.8)):
    if dim == 2:
        return [math.cos(0.5 * angle), 0.0, 0.0, math.sin(0.5 * angle)]
    a = np.asarray(axis) / np.linalg.norm(axis)
    return [math.cos(0.5 * angle)] + list(math.sin(0.5 * angle) * a)


def _immersed(dim, **kw):
    if dim == 2:
        c = wl.tank2d(dx=0.02, width=1.0, depth=0.6, wall_height=0.7, **kw)
        return wl.with_free_body(c, (0.4, 0.2), (0.6, 0.32), 1500.0)
    c = wl.box3d(0.04, (0.8, 0.6, 0.8), (0.8, 0.6, 0.6), **kw)
    return wl.with_free_body(c, (0.28, 0.2, 0.24), (0.52, 0.4, 0.4), 1500.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_pose_equals_explicit_walls(orc, dim):
    c = wl.random_velocity(_immersed(dim, delta_sph=True, pst=True, tic=True, fs_project=True, cont_uncorr=True,
                                     fs_mode="exact"), 0.05, 3)
    Q = _rot(dim, 0.37)
    shift = np.array([0.013, -0.021, 0.008][:dim])
    c["body"] = dict(c["body"], q=_quat(dim, 0.37),
                     c=list(np.asarray(c["body"]["c"][:dim]) + shift) + [0.0] * (3 - dim))
    r = orc.eval_rates(c)
    b = c["kind"] == 2
    c0 = np.asarray(c["params"]["body_c0"][:dim])
    ex = dict(c)
    ex["x"] = c["x"].copy()
    ex["normal"] = c["normal"].copy()
    ex["x"][b] = c0 + shift + (c["x"][b] - c0) @ Q.T
    ex["normal"][b] = c["normal"][b] @ Q.T
    ex["kind"] = np.where(b, 1, c["kind"]).astype(np.uint8)
    ex["params"] = {k: v for k, v in c["params"].items() if not k.startswith("body_")}
    ex.pop("body")
    re = orc.eval_rates(ex)
    f = c["kind"] == 0
    for k in ("nnb", "tic"):
        assert np.array_equal(r[k][f], re[k][f]), k
    assert np.array_equal(r["mir_src"], re["mir_src"])
    # the rotations are formed differently (quaternion matrix, Rodrigues):
    # positions agree to rounding, the rates to the parity bar
    for k in ("acc", "dphi", "dushift"):
        scale = max(np.abs(re[k][f]).max(), 1e-30)
        assert np.abs(r[k][f] - re[k][f]).max() <= 1e-11 * scale, k


@pytest.mark.parametrize("dim", [2, 3])
def test_slip_relative_to_moving_wall(orc, dim):
    c = wl.random_velocity(_immersed(dim), 0.3, 5)
    v = [0.4, -0.7, 0.2][:dim] + [0.0] * (3 - dim)
    w = [0.0, 0.0, 1.3] if dim == 2 else [0.5, -0.9, 1.3]
    c["body"] = dict(c["body"], v=v, w=w, q=_quat(dim, 0.2))
    r = orc.eval_rates(c)
    b = (c["kind"] == 2) & (r["mir_src"] >= 0)
    assert b.sum() > 20
    Q = _rot(dim, 0.2)
    c0 = np.asarray(c["params"]["body_c0"][:dim])
    cc = np.asarray(c["body"]["c"][:dim])
    xd = cc + (c["x"][b] - c0) @ Q.T
    nd = c["normal"][b] @ Q.T
    arm = np.zeros((b.sum(), 3))
    arm[:, :dim] = xd - cc
    uw = (np.asarray(v) + np.cross(np.asarray(w), arm))[:, :dim]
    ud = r["mir_u"][b]
    uf = c["u"][r["mir_src"][b]]
    # normal: the wall's; tangential: the source particle's
    assert np.abs(((ud - uw) * nd).sum(1)).max() <= 1e-14
    tang = lambda a: a - (a * nd).sum(1)[:, None] * nd
    assert np.abs(tang(ud) - tang(uf)).max() <= 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_archimedes(orc, dim):
    c = _immersed(dim)
    r = orc.eval_rates(c)
    F, T = r["body_force"], r["body_torque"]
    vol = 0.2 * 0.12 if dim == 2 else 0.24 * 0.2 * 0.16
    want = 1000.0 * 9.81 * vol
    assert abs(F[dim - 1] / want - 1.0) <= 0.02, F
    assert np.abs(F[:dim - 1]).max() <= 1e-9 * want
    assert np.abs(T).max() <= 1e-9 * want * 0.1


def _immersed_cylinder(dim):
    """A solid cylinder (D = 0.05 m; 3D: length 0.06 m along y) at rest in
    hydrostatic water, centred on a node of the fluid's lattice."""
    if dim == 2:
        c = wl.tank2d(dx=0.005, width=0.4, depth=0.3, wall_height=0.35)
        return wl.with_free_cylinder(c, (0.2, 0.15), 0.05, 1370.0)
    c = wl.box3d(0.005, (0.2, 0.12, 0.2), (0.2, 0.12, 0.16))
    return wl.with_free_cylinder(c, (0.1, 0.06, 0.08), 0.05, 1370.0, length=0.06)


@pytest.mark.parametrize("dim", [2, 3])
def test_archimedes_cylinder(orc, dim):
    """The curved body of the water-entry case: buoyancy rho0 g pi R^2 (L)
    to 2%, no side force or torque beyond rounding (the scene is symmetric)."""
    c = _immersed_cylinder(dim)
    r = orc.eval_rates(c)
    F, T = r["body_force"], r["body_torque"]
    want = 1000.0 * 9.81 * math.pi * 0.025 ** 2 * (0.06 if dim == 3 else 1.0)
    assert abs(F[dim - 1] / want - 1.0) <= 0.02, F
    assert np.abs(F[:dim - 1]).max() <= 1e-9 * want
    assert np.abs(T).max() <= 1e-9 * want * 0.025


@pytest.mark.parametrize("dim", [2, 3])
def test_force_and_torque_rotate_with_the_scene(orc, dim):
    c = wl.random_potential(wl.random_velocity(wl.jitter(_immersed(dim, tic=True), 0.1, 7), 0.1, 8), 0.5, 9)
    r = orc.eval_rates(c)
    Q = _rot(dim, 0.9)
    centre = np.full(dim, 0.4)
    rc = dict(c)
    rc["x"] = centre + (c["x"] - centre) @ Q.T
    rc["u"] = c["u"] @ Q.T
    rc["normal"] = c["normal"] @ Q.T
    G = np.asarray(c["params"]["gravity"][:dim]) @ Q.T
    pd = dict(c["params"])
    pd["gravity"] = list(G) + [0.0] * (3 - dim)
    pd["body_c0"] = list(centre + (np.asarray(pd["body_c0"][:dim]) - centre) @ Q.T) + [0.0] * (3 - dim)
    pd["domain_lo"] = [-2.0] * dim + [0.0] * (3 - dim)
    pd["domain_hi"] = [3.0] * dim + [0.0] * (3 - dim)
    rc["params"] = pd
    rc["body"] = dict(c["body"], c=pd["body_c0"])
    # the same potential field: phi is a state variable, turned with the scene
    rr = orc.eval_rates(rc)
    F, T = r["body_force"][:dim], r["body_torque"]
    scale = np.abs(F).max()
    assert scale > 1.0
    assert np.abs(rr["body_force"][:dim] - F @ Q.T).max() <= 1e-9 * scale
    if dim == 2:
        assert abs(rr["body_torque"][2] - T[2]) <= 1e-9 * max(abs(T[2]), scale * 0.1)
    else:
        assert np.abs(rr["body_torque"] - T @ Q.T).max() <= 1e-9 * max(np.abs(T).max(), scale * 0.1)


@pytest.mark.parametrize("dim", [2, 3])
def test_torque_reference_point(orc, dim):
    c = wl.random_potential(wl.jitter(_immersed(dim, tic=True), 0.1, 11), 0.5, 12)
    r = orc.eval_rates(c)
    d = np.array([0.031, -0.017, 0.023])
    moved = dict(c)
    pd = dict(c["params"])
    pd["body_c0"] = list(np.asarray(pd["body_c0"]) + np.concatenate([d[:dim], [0.0] * (3 - dim)]))
    moved["params"] = pd
    moved["body"] = dict(c["body"], c=pd["body_c0"])
    rm = orc.eval_rates(moved)
    F, T = r["body_force"], r["body_torque"]
    assert np.array_equal(rm["body_force"], F)  # same dummy positions: same forces
    dd = np.concatenate([d[:dim], [0.0] * (3 - dim)])
    want = T + np.cross(-dd, F)  # (x - c') x F = (x - c) x F + (c - c') x F
    assert np.abs(rm["body_torque"] - want).max() <= 1e-10 * max(np.abs(F).max(), 1.0)
