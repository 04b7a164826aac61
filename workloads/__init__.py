"""Seeded synthetic inputs shaped like the paper's workloads.

This module builds particle sets (positions, velocities, potential, kind,
wall normals) and a plain parameter dictionary.  It holds none of the
solver's arithmetic: both the CPU oracle and the HIP library consume what it
returns, each converting the dictionary into its own parameter struct.

Every case is a dict:
    params : dict of physical / numerical parameters (see ``base_params``)
    x, u   : (n, dim) float64      positions, velocities
    phi    : (n,) float64          auxiliary potential
    kind   : (n,) uint8            0 fluid, 1 fixed wall dummy, 2 dummy of the
                                   moving body (position at its reference time)
    normal : (n, dim) float64      unit wall normal (dummies; zero for fluid)
    mass   : None                  (each side derives m = rho(phi) dx^d)
    t      : float                 initial time
    meta   : dict                  description and sizes

Geometry: particles sit on the lattice ((i+1/2) dx, (j+1/2) dx[, (k+1/2) dx]);
walls are ``layers`` lattice layers of dummies outside the container.  The
initial potential is the hydrostatic solution phi = G.x + H |G| (zero at the
still-water level H), velocity zero.
"""
from __future__ import annotations

import math

import numpy as np

G_EARTH = 9.81


def base_params(dim, dx, *, h_factor=1.3, c0=None, depth=1.0, gravity=None, rho0=1000.0,
                nu=1e-4, cfl=0.2, delta=0.1, pst_R=0.2, pst_n=4.0, delta_sph=False, pst=False,
                tic=False, fs_project=False, cont_uncorr=False, fs_mode="none", precision="fp64",
                forcing_amp=(0.0, 0.0, 0.0), forcing_omega=0.0, domain_lo=None, domain_hi=None,
                features=False):
    if gravity is None:
        gravity = [0.0, -G_EARTH, 0.0] if dim == 2 else [0.0, 0.0, -G_EARTH]
    if c0 is None:
        c0 = 10.0 * math.sqrt(G_EARTH * depth)
    h = h_factor * dx
    return {
        "dim": dim, "dx": dx, "h": h, "c0": float(c0), "rho0": rho0, "nu": nu, "cfl": cfl,
        "delta": delta, "pst_R": pst_R, "pst_n": pst_n,
        "lambda_tic": 0.75, "lambda_fs_lo": 0.2, "lambda_fs_hi": 0.75, "lambda_singular": 1e-6,
        "gravity": list(gravity), "forcing_amp": list(forcing_amp), "forcing_omega": float(forcing_omega),
        "domain_lo": list(domain_lo) if domain_lo is not None else [0.0] * 3,
        "domain_hi": list(domain_hi) if domain_hi is not None else [0.0] * 3,
        "cell_size": 2.0 * h,
        "delta_sph": bool(delta_sph), "pst": bool(pst), "tic": bool(tic),
        "fs_project": bool(fs_project), "cont_uncorr": bool(cont_uncorr),
        "fs_mode": fs_mode, "precision": precision, "features": bool(features),
    }


def _lattice(lo_idx, hi_idx, dx):
    axes = [(np.arange(a, b) + 0.5) * dx for a, b in zip(lo_idx, hi_idx)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def _assemble(params, xf, xd, nd, H, meta):
    dim = params["dim"]
    x = np.concatenate([xf, xd], axis=0).astype(np.float64)
    n = x.shape[0]
    kind = np.concatenate([np.zeros(len(xf), np.uint8), np.ones(len(xd), np.uint8)])
    normal = np.zeros((n, dim))
    normal[len(xf):] = nd
    G = np.asarray(params["gravity"][:dim], dtype=np.float64)
    gmag = float(np.linalg.norm(params["gravity"]))
    phi = x @ G + H * gmag
    meta = dict(meta)
    meta.update({"n_fluid": int(len(xf)), "n_dummy": int(len(xd)), "H": H})
    return {"params": params, "x": x, "u": np.zeros((n, dim)), "phi": phi, "kind": kind,
            "normal": normal, "mass": None, "t": 0.0, "meta": meta}


def _box_walls(dim, dx, n_cells, layers, open_top_cells=None):
    """Dummy lattice points in a `layers`-thick shell around the box
    [0, n_cells*dx] (axis dim-1 vertical).  With open_top_cells the vertical
    shell stops at that many cells (no lid)."""
    lo = [-layers] * dim
    hi = [n + layers for n in n_cells]
    if open_top_cells is not None:
        hi[dim - 1] = open_top_cells
    pts = _lattice(lo, hi, dx)
    box_hi = np.array(n_cells, dtype=np.float64) * dx
    inside = np.all((pts > 0.0) & (pts < box_hi), axis=1)
    pts = pts[~inside]
    nrm = np.zeros_like(pts)
    for a in range(dim):
        nrm[:, a] += (pts[:, a] < 0.0).astype(np.float64)
        nrm[:, a] -= (pts[:, a] > box_hi[a]).astype(np.float64)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts, nrm


def tank2d(dx=0.01, width=1.0, depth=0.5, wall_height=0.6, layers=3, **kw):
    """2D hydrostatic tank with a flat bottom (1.0 m x 0.5 m water at dx = 0.01:
    5,000 fluid particles, 678 dummies)."""
    nx, ny, nw = round(width / dx), round(depth / dx), round(wall_height / dx)
    kw.setdefault("depth", depth)
    ceiling = wall_height + 0.25 * wall_height
    params = base_params(2, dx, domain_lo=[-layers * dx, -layers * dx, 0.0],
                         domain_hi=[width + layers * dx, ceiling, 0.0], **kw)
    xf = _lattice([0, 0], [nx, ny], dx)
    xd, nd = _box_walls(2, dx, [nx, nw], layers, open_top_cells=nw)
    return _assemble(params, xf, xd, nd, depth,
                     {"name": "tank2d", "desc": f"2D hydrostatic tank {width}x{depth} m, dx={dx}"})


def bump2d(shape="gauss", dx=0.002, width=2.0, depth=0.5, amp=0.1, sigma=0.1, bump_width=0.4,
           wall_height=None, layers=3, **kw):
    """2D hydrostatic water layer over a bottom bump.  shape 'gauss':
    b(x) = amp exp(-(x - W/2)^2 / (2 sigma^2)); 'rect': a block of height amp and
    width bump_width; 'tri': a triangle of height amp and base bump_width."""
    if wall_height is None:
        wall_height = depth + 0.1 * depth
    nx, nw = round(width / dx), round(wall_height / dx)
    xc = 0.5 * width
    kw.setdefault("depth", depth)
    ceiling = wall_height * 1.25
    params = base_params(2, dx, domain_lo=[-layers * dx, -layers * dx, 0.0],
                         domain_hi=[width + layers * dx, ceiling, 0.0], **kw)

    def bottom(x):
        if shape == "gauss":
            return amp * np.exp(-((x - xc) ** 2) / (2.0 * sigma ** 2))
        if shape == "tri":
            return np.maximum(0.0, amp * (1.0 - np.abs(x - xc) / (0.5 * bump_width)))
        return np.where(np.abs(x - xc) <= 0.5 * bump_width, amp, 0.0)

    def bottom_slope(x):
        if shape == "gauss":
            return -(x - xc) / sigma ** 2 * bottom(x)
        if shape == "tri":
            inside = np.abs(x - xc) < 0.5 * bump_width
            return np.where(inside, -np.sign(x - xc) * amp / (0.5 * bump_width), 0.0)
        return np.zeros_like(x)

    pts = _lattice([0, 0], [nx, round(depth / dx)], dx)
    b = bottom(pts[:, 0])
    xf = pts[pts[:, 1] > b]
    # dummies: the box shell plus lattice points inside the bump within `layers` cells of its surface
    xd_box, nd_box = _box_walls(2, dx, [nx, nw], layers, open_top_cells=nw)
    solid = pts[pts[:, 1] <= b]
    keep = []
    nrm = []
    for p in solid:
        xb = p[0]
        if shape == "rect":
            top_gap = amp - p[1]
            side_gap = 0.5 * bump_width - abs(xb - xc)
            if min(top_gap, side_gap) >= layers * dx:
                continue
            keep.append(p)
            if top_gap <= side_gap:
                nrm.append([0.0, 1.0])
            else:
                nrm.append([math.copysign(1.0, xb - xc), 0.0])
        else:
            bb = float(bottom(np.array([xb]))[0])
            if bb - p[1] >= layers * dx:
                continue
            s = float(bottom_slope(np.array([xb]))[0])
            v = np.array([-s, 1.0])
            keep.append(p)
            nrm.append(v / np.linalg.norm(v))
    if keep:
        xd = np.concatenate([xd_box, np.array(keep)], axis=0)
        nd = np.concatenate([nd_box, np.array(nrm)], axis=0)
    else:
        xd, nd = xd_box, nd_box
    return _assemble(params, xf, xd, nd, depth,
                     {"name": f"bump2d-{shape}",
                      "desc": f"2D {width}x{depth} m layer over a {shape} bump (amp {amp}), dx={dx}"})


def box3d(dx, tank, fluid_hi, layers=3, name="box3d", desc="", **kw):
    """3D closed box [0, tank] (lid included) with a fluid block
    [0, fluid_hi] at rest; gravity along -z."""
    n_cells = [round(t / dx) for t in tank]
    nf = [round(f / dx) for f in fluid_hi]
    kw.setdefault("depth", fluid_hi[2])
    params = base_params(3, dx, domain_lo=[-layers * dx] * 3,
                         domain_hi=[t + layers * dx for t in tank], **kw)
    xf = _lattice([0, 0, 0], nf, dx)
    xd, nd = _box_walls(3, dx, n_cells, layers)
    return _assemble(params, xf, xd, nd, fluid_hi[2], {"name": name, "desc": desc})


def dambreak3d(dx=0.01, tank=(3.22, 1.0, 1.0), column=(1.2, 1.0, 0.55), **kw):
    """3D dam break: column at rest against the x = 0 wall of a closed tank
    (660,000 fluid + 465,408 dummies at dx = 0.01)."""
    kw.setdefault("c0", 30.0)
    kw.setdefault("delta_sph", True)
    kw.setdefault("pst", True)
    kw.setdefault("tic", True)
    kw.setdefault("fs_project", True)
    kw.setdefault("cont_uncorr", True)
    kw.setdefault("fs_mode", "exact")
    return box3d(dx, tank, column, name="dambreak3d",
                 desc=f"3D dam break, tank {tank}, column {column}, dx={dx}", **kw)


def _floor_obstacle(lo, hi, dx, layers):
    """Dummy lattice points of a solid box [lo, hi] standing on the floor
    z = 0 (corners on multiples of dx): the points within `layers` spacings of
    its side and top faces, each with the outward normal of its nearest of
    those faces (its bottom face rests on the floor and meets no water)."""
    lo_ext = (lo[0], lo[1], -(layers + 1) * dx)
    pts, nrm = _body_box(3, lo_ext, hi, dx, layers)
    keep = pts[:, 2] > 0.0
    return pts[keep], nrm[keep]


def dambreak_obstacle3d(dx=0.161 / 30, tank=(3.22, 1.0, 2.0), column=(1.228, 1.0, 0.55),
                        obstacle=((2.3955, 0.2985), (0.161, 0.403, 0.161)), layers=3, **kw):
    """The paper's 3D dam break against an obstacle (Sec. 4): a water column
    at rest against the x = 0 wall of a closed reservoir and a box obstacle
    on the floor downstream, obstacle corner (x, y) and size (dx, dy, dz);
    every length snapped to the lattice.  At the default spacing (the
    obstacle 30 particles wide): 4.34M fluid."""
    for k, v in (("c0", 30.0), ("delta_sph", True), ("pst", True), ("tic", True), ("fs_project", True),
                 ("cont_uncorr", True), ("fs_mode", "exact")):
        kw.setdefault(k, v)
    snap = lambda v: round(v / dx) * dx  # noqa: E731
    tank = tuple(snap(t) for t in tank)
    column = tuple(snap(c) for c in column)
    kw.setdefault("depth", column[2])
    case = box3d(dx, tank, column, layers=layers, name="dambreak_obstacle3d", **kw)
    (ox, oy), size = obstacle
    lo = (snap(ox), snap(oy), 0.0)
    hi = (lo[0] + snap(size[0]), lo[1] + snap(size[1]), snap(size[2]))
    xo, no = _floor_obstacle(lo, hi, dx, layers)
    x = case["x"]
    inside = (case["kind"] == 0) & np.all((x > np.array(lo) - 0.25 * dx) & (x < np.array(hi) + 0.25 * dx), axis=1)
    keep = ~inside
    G = np.asarray(case["params"]["gravity"], dtype=np.float64)
    H = case["meta"]["H"]
    c = dict(case)
    c["x"] = np.concatenate([x[keep], xo])
    c["u"] = np.concatenate([case["u"][keep], np.zeros_like(xo)])
    c["phi"] = np.concatenate([case["phi"][keep], xo @ G + H * float(np.linalg.norm(G))])
    c["kind"] = np.concatenate([case["kind"][keep], np.ones(len(xo), np.uint8)])
    c["normal"] = np.concatenate([case["normal"][keep], no])
    meta = dict(case["meta"])
    meta.update({"n_fluid": int((c["kind"] == 0).sum()), "n_dummy": int((c["kind"] != 0).sum()),
                 "n_obstacle": int(len(xo)),
                 "desc": f"3D dam break against an obstacle, tank {tank}, column {column}, obstacle {lo}-{hi}, dx={dx:.6g}"})
    c["meta"] = meta
    return c


def dambreak2d(dx=0.01, tank=(3.22, 1.0), column=(1.2, 0.55), **kw):
    """2D dam break: the 3D case's vertical section, a column at rest against
    the x = 0 wall of a closed tank (6,600 fluid at dx = 0.01)."""
    kw.setdefault("c0", 30.0)
    for k in ("delta_sph", "pst", "tic", "fs_project", "cont_uncorr"):
        kw.setdefault(k, True)
    kw.setdefault("fs_mode", "exact")
    kw.setdefault("depth", column[1])
    layers = 3
    params = base_params(2, dx, domain_lo=[-layers * dx, -layers * dx, 0.0],
                         domain_hi=[tank[0] + layers * dx, tank[1] + layers * dx, 0.0], **kw)
    xf = _lattice([0, 0], [round(column[0] / dx), round(column[1] / dx)], dx)
    xd, nd = _box_walls(2, dx, [round(tank[0] / dx), round(tank[1] / dx)], layers)
    return _assemble(params, xf, xd, nd, column[1],
                     {"name": "dambreak2d", "desc": f"2D dam break, tank {tank}, column {column}, dx={dx}"})


def slosh_omega(length=1.0, depth=0.28, factor=1.2):
    """Forcing frequency for a period `factor` times the first natural sloshing
    period (linear theory: w1^2 = g k tanh(k d), k = pi / L)."""
    k = math.pi / length
    w1 = math.sqrt(G_EARTH * k * math.tanh(k * depth))
    return w1 / factor


def slosh3d(dx=0.002, tank=(1.0, 0.5, 0.56), depth=0.28, amp=0.005, surface_amp=0.0, **kw):
    """3D sloshing tank forced horizontally in its own frame: G(t) = (A w^2
    sin wt, 0, -g).  At dx = 0.002: 17,500,000 fluid + 2,047,296 dummies.
    surface_amp > 0: the first sloshing mode's shape released from rest, the
    free surface at depth + surface_amp cos(pi x / L) and the potential
    hydrostatic below it, phi = g (eta(x) - z)."""
    kw.setdefault("delta_sph", True)
    kw.setdefault("pst", True)
    kw.setdefault("tic", True)
    kw.setdefault("fs_project", True)
    kw.setdefault("cont_uncorr", True)
    kw.setdefault("fs_mode", "exact")
    w = slosh_omega(tank[0], depth)
    kw.setdefault("forcing_amp", (amp, 0.0, 0.0))
    kw.setdefault("forcing_omega", w)
    kw.setdefault("depth", depth)
    case = box3d(dx, tank, (tank[0], tank[1], depth + surface_amp), name="slosh3d",
                 desc=f"3D sloshing tank {tank}, depth {depth}, forcing A={amp} m, dx={dx}"
                      + (f", surface {surface_amp} cos(pi x/L)" if surface_amp > 0 else ""), **kw)
    if surface_amp <= 0.0:
        return case
    f = case["kind"] == 0
    eta = depth + surface_amp * np.cos(math.pi * case["x"][:, 0] / tank[0])
    keep = ~f | (case["x"][:, 2] < eta)
    out = {k: (v[keep] if isinstance(v, np.ndarray) else v) for k, v in case.items()}
    g = float(np.linalg.norm(case["params"]["gravity"]))
    fk = out["kind"] == 0
    out["phi"] = out["phi"].copy()
    out["phi"][fk] = g * (eta[keep][fk] - out["x"][fk, 2])
    out["meta"] = dict(case["meta"], n_fluid=int(fk.sum()), H=depth)
    return out


def jitter(case, sigma=0.1, seed=0):
    """Copy of `case` with fluid positions displaced by N(0, (sigma dx)^2)."""
    c = dict(case)
    rng = np.random.default_rng(seed)
    x = case["x"].copy()
    f = case["kind"] == 0
    x[f] += rng.normal(0.0, sigma * case["params"]["dx"], size=x[f].shape)
    c["x"] = x
    return c


def random_velocity(case, amp=0.1, seed=1):
    c = dict(case)
    rng = np.random.default_rng(seed)
    u = case["u"].copy()
    f = case["kind"] == 0
    u[f] = rng.normal(0.0, amp, size=u[f].shape)
    c["u"] = u
    return c


def random_potential(case, amp=1.0, seed=2):
    c = dict(case)
    rng = np.random.default_rng(seed)
    c["phi"] = case["phi"] + amp * rng.normal(0.0, 1.0, size=case["phi"].shape)
    return c


def with_params(case, **kw):
    c = dict(case)
    p = dict(case["params"])
    p.update(kw)
    c["params"] = p
    return c


def ditching_motion():
    """The body velocity history of the paper's aircraft-ditching case (Sec. 4):
    U = -5 m/s for T <= 0.8 s, then 5/2 (T - 3) m/s up to T = 2.8 s, along x;
    as pieces a_k + b_k T for the parameter keys body_t / body_a / body_b."""
    return {"body_t": [0.0, 0.8, 2.8],
            "body_a": [[-5.0, 0.0, 0.0], [-7.5, 0.0, 0.0]],
            "body_b": [[0.0, 0.0, 0.0], [2.5, 0.0, 0.0]]}


def _body_box(dim, lo, hi, dx, layers):
    """Dummy lattice points of a solid box [lo, hi] (corners on multiples of
    dx): the points within `layers` spacings of its surface, each with the
    outward normal of its nearest face(s) (corners: the normalised sum)."""
    lo = np.asarray(lo[:dim], dtype=np.float64)
    hi = np.asarray(hi[:dim], dtype=np.float64)
    n = [int(round((b - a) / dx)) for a, b in zip(lo, hi)]
    pts = _lattice([0] * dim, n, dx) + lo
    dlo, dhi = pts - lo, hi - pts
    dmin = np.minimum(dlo, dhi)
    m = dmin.min(axis=1)
    keep = m < layers * dx
    pts, dlo, dhi, dmin, m = pts[keep], dlo[keep], dhi[keep], dmin[keep], m[keep]
    nrm = np.zeros_like(pts)
    near = dmin <= m[:, None] + 1e-9 * dx
    nrm[near & (dlo <= dhi)] = -1.0  # a point midway between two faces takes the lower one
    nrm[near & (dhi < dlo)] = 1.0
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts, nrm


def with_body(case, lo, hi, motion, layers=3):
    """Copy of `case` with a solid box body [lo, hi] of kind-2 dummies moving
    with the prescribed velocity history `motion` (keys body_t, body_a,
    body_b, pieces a_k + b_k t); fluid particles inside the box are removed.
    The box is given at its position of time body_t[0]."""
    pd = dict(case["params"])
    dim = pd["dim"]
    dx = pd["dx"]
    xb, nb = _body_box(dim, lo, hi, dx, layers)
    x = case["x"]
    lo_a = np.asarray(lo[:dim]) - 0.25 * dx
    hi_a = np.asarray(hi[:dim]) + 0.25 * dx
    inside = (case["kind"] == 0) & np.all((x > lo_a) & (x < hi_a), axis=1)
    keep = ~inside
    G = np.asarray(pd["gravity"][:dim], dtype=np.float64)
    gmag = float(np.linalg.norm(pd["gravity"]))
    H = case["meta"]["H"]
    c = dict(case)
    c["x"] = np.concatenate([x[keep], xb])
    c["u"] = np.concatenate([case["u"][keep], np.zeros_like(xb)])
    c["phi"] = np.concatenate([case["phi"][keep], xb @ G + H * gmag])
    c["kind"] = np.concatenate([case["kind"][keep], np.full(len(xb), 2, np.uint8)])
    c["normal"] = np.concatenate([case["normal"][keep], nb])
    pd.update({k: [list(map(float, r)) if isinstance(r, (list, tuple)) else float(r) for r in motion[k]]
               for k in ("body_t", "body_a", "body_b")})
    c["params"] = pd
    meta = dict(case["meta"])
    meta.update({"n_fluid": int(((c["kind"] == 0)).sum()), "n_dummy": int((c["kind"] != 0).sum()),
                 "n_body": int(len(xb))})
    c["meta"] = meta
    return c


def with_free_body(case, lo, hi, density, v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0), layers=3):
    """Copy of `case` with a solid box body [lo, hi] of kind-2 dummies that
    moves under G(t) and the water's force and torque: mass density * volume
    (area in 2D), the inertia tensor of the solid box about its centre, the
    dummies given at the pose of the box, initial velocity v0 and angular
    velocity w0 (world frame; in 2D only w0[2] is used).  Fluid particles
    inside the box are removed."""
    dim = case["params"]["dim"]
    c = with_body(case, lo, hi, {"body_t": [], "body_a": [], "body_b": []}, layers=layers)
    pd = c["params"]
    for k in ("body_t", "body_a", "body_b"):
        pd.pop(k, None)
    ext = [float(b - a) for a, b in zip(lo[:dim], hi[:dim])] + [0.0] * (3 - dim)
    vol = float(np.prod(ext[:dim]))
    m = density * vol
    a, b, cc = ext
    inertia = [m * (b * b + cc * cc) / 12.0, m * (a * a + cc * cc) / 12.0, m * (a * a + b * b) / 12.0, 0.0, 0.0, 0.0]
    centre = [0.5 * (float(lo[k]) + float(hi[k])) for k in range(dim)] + [0.0] * (3 - dim)
    pd.update({"body_free": True, "body_mass": m, "body_inertia": inertia, "body_c0": centre})
    c["body"] = {"c": list(centre), "q": [1.0, 0.0, 0.0, 0.0], "v": list(v0) + [0.0] * (3 - len(v0)),
                 "w": list(w0) + [0.0] * (3 - len(w0))}
    c["meta"]["desc"] = c["meta"].get("desc", "") + f"; free box body {lo}-{hi}, density {density}"
    return c


def _body_cylinder(dim, centre, radius, length, dx, layers):
    """Dummy points of a solid horizontal cylinder (axis along y in 3D; a
    disc in 2D) on a lattice of spacing dx centred on it: the points within
    `layers` spacings of its surface, each with the outward normal of its
    nearest surface (lateral: radial; 3D end caps: axial; equidistant: the
    normalised sum)."""
    c = np.asarray(centre[:dim], dtype=np.float64)
    k = int(math.ceil(radius / dx))
    if dim == 2:
        pts = _lattice([-k, -k], [k, k], dx)
    else:
        m = int(math.ceil(0.5 * length / dx))
        pts = _lattice([-k, -m, -k], [k, m, k], dx)
    rad = np.stack([pts[:, 0], pts[:, dim - 1]], 1)
    r = np.linalg.norm(rad, axis=1)
    d_lat = radius - r
    if dim == 2:
        keep = (d_lat >= 0.0) & (d_lat < layers * dx)
        d_cap = np.full(len(pts), np.inf)
    else:
        d_cap = 0.5 * length - np.abs(pts[:, 1])
        keep = (d_lat >= 0.0) & (d_cap >= 0.0) & (np.minimum(d_lat, d_cap) < layers * dx)
    pts, rad, r, d_lat, d_cap = pts[keep], rad[keep], r[keep], d_lat[keep], d_cap[keep]
    nrm = np.zeros_like(pts)
    dmin = np.minimum(d_lat, d_cap)
    lat = d_lat <= dmin + 1e-9 * dx
    nrm[lat, 0] = rad[lat, 0] / r[lat]
    nrm[lat, dim - 1] = rad[lat, 1] / r[lat]
    if dim == 3:
        cap = d_cap <= dmin + 1e-9 * dx
        nrm[cap, 1] += np.sign(pts[cap, 1])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return pts + c, nrm


def with_free_cylinder(case, centre, diameter, density, length=0.0, v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0),
                       layers=3):
    """Copy of `case` with a free solid cylinder of kind-2 dummies (axis
    along y in 3D, of the given length; a disc in 2D) centred at `centre`:
    mass density * volume, the solid cylinder's inertia tensor about its
    centre, initial velocity v0 and angular velocity w0.  The dummies sit on
    a lattice of the case's spacing centred on the cylinder (it continues
    the fluid's lattice when the centre is a lattice node of it).  Fluid
    particles inside it are removed (and a given mass array dropped: the
    masses then follow from the potential)."""
    pd = dict(case["params"])
    dim = pd["dim"]
    dx = pd["dx"]
    R = 0.5 * diameter
    xb, nb = _body_cylinder(dim, centre, R, length, dx, layers)
    x = case["x"]
    c3 = np.asarray(centre[:dim], dtype=np.float64)
    rad = np.stack([x[:, 0] - c3[0], x[:, dim - 1] - c3[dim - 1]], 1)
    # removed: the fluid points inside the solid (closed), no wider shell,
    # so that a body whose lattice continues the fluid's leaves no void
    # between them (a void of a quarter spacing costs a quarter of the
    # buoyancy at ten spacings per radius)
    inside = np.linalg.norm(rad, axis=1) <= R
    if dim == 3:
        inside &= np.abs(x[:, 1] - c3[1]) <= 0.5 * length
    keep = ~(inside & (case["kind"] == 0))
    G = np.asarray(pd["gravity"][:dim], dtype=np.float64)
    gmag = float(np.linalg.norm(pd["gravity"]))
    H = case["meta"]["H"]
    c = dict(case)
    c["x"] = np.concatenate([x[keep], xb])
    c["u"] = np.concatenate([case["u"][keep], np.zeros_like(xb)])
    c["phi"] = np.concatenate([case["phi"][keep], xb @ G + H * gmag])
    c["kind"] = np.concatenate([case["kind"][keep], np.full(len(xb), 2, np.uint8)])
    c["normal"] = np.concatenate([case["normal"][keep], nb])
    if case.get("mass") is not None:
        c["mass"] = None
    if dim == 2:
        m = density * math.pi * R * R
        inertia = [0.25 * m * R * R, 0.25 * m * R * R, 0.5 * m * R * R, 0.0, 0.0, 0.0]
    else:
        m = density * math.pi * R * R * length
        ia = m * (3.0 * R * R + length * length) / 12.0
        inertia = [ia, 0.5 * m * R * R, ia, 0.0, 0.0, 0.0]
    cen = [float(v) for v in centre[:dim]] + [0.0] * (3 - dim)
    pd.update({"body_free": True, "body_mass": m, "body_inertia": inertia, "body_c0": cen})
    c["params"] = pd
    c["body"] = {"c": list(cen), "q": [1.0, 0.0, 0.0, 0.0], "v": list(v0) + [0.0] * (3 - len(v0)),
                 "w": list(w0) + [0.0] * (3 - len(w0))}
    meta = dict(case["meta"])
    meta.update({"n_fluid": int((c["kind"] == 0).sum()), "n_dummy": int((c["kind"] != 0).sum()),
                 "n_body": int(len(xb))})
    c["meta"] = meta
    return c


def cylinder_entry(dim=3, dx=0.0025, tank=(1.0, 0.4), depth=0.6, diameter=0.05, length=0.2, v0=-6.22,
                   density=1370.0, wall_height=1.585, ceiling=1.6, gap=None, layers=3, **kw):
    """Water entry of a free horizontal cylinder (Sec. 4): a tank of length
    tank[0] (x) and width tank[1] (y, 3D) with water of depth `depth`, and a
    solid cylinder of the given diameter and length (axis along y, centred in
    the tank; a disc in 2D, the vertical section) of the given density,
    released with its lowest point `gap` (default dx / 2) above the still
    surface at vertical velocity v0; it then moves under gravity and the
    water's force and torque.  C0 = 30 m/s and every stabiliser on by
    default.  The paper gives neither the tank's height nor its wall layout:
    the default wall height makes the dummy count match its 2.37M (3D at
    the defaults: 15,360,000 fluid + 2,368,988 dummies, of which 13,736 are
    the cylinder's; the paper counts 15.16M + 2.37M = 17.53M)."""
    kw.setdefault("c0", 30.0)
    for k in ("delta_sph", "pst", "tic", "fs_project", "cont_uncorr"):
        kw.setdefault(k, True)
    kw.setdefault("fs_mode", "exact")
    kw.setdefault("depth", depth)
    gap = 0.5 * dx if gap is None else gap
    R = 0.5 * diameter
    if dim == 2:
        nx, nz, nw = round(tank[0] / dx), round(depth / dx), round(wall_height / dx)
        params = base_params(2, dx, domain_lo=[-layers * dx, -layers * dx, 0.0],
                             domain_hi=[tank[0] + layers * dx, ceiling, 0.0], **kw)
        xf = _lattice([0, 0], [nx, nz], dx)
        xd, nd = _box_walls(2, dx, [nx, nw], layers, open_top_cells=nw)
        centre = [0.5 * tank[0], depth + gap + R]
    else:
        nx, ny, nz, nw = round(tank[0] / dx), round(tank[1] / dx), round(depth / dx), round(wall_height / dx)
        params = base_params(3, dx, domain_lo=[-layers * dx] * 3,
                             domain_hi=[tank[0] + layers * dx, tank[1] + layers * dx, ceiling], **kw)
        xf = _lattice([0, 0, 0], [nx, ny, nz], dx)
        xd, nd = _box_walls(3, dx, [nx, ny, nw], layers, open_top_cells=nw)
        centre = [0.5 * tank[0], 0.5 * tank[1], depth + gap + R]
    case = _assemble(params, xf, xd, nd, depth, {"name": f"cylinder_entry{dim}d", "desc": ""})
    v = [0.0, 0.0, 0.0]
    v[dim - 1] = float(v0)
    c = with_free_cylinder(case, centre, diameter, density, length=length, v0=v, layers=layers)
    c["meta"]["desc"] = (f"{dim}D water entry of a free cylinder D={diameter} m"
                         + (f" L={length} m" if dim == 3 else "")
                         + f", density {density}, V0={v0} m/s into water {tank[:dim - 1]}x{depth} m, dx={dx}")
    return c


def entry2d(dx=0.01, width=0.6, depth=0.3, body=(0.25, 0.35, 0.27, 0.33), speed=(-0.5, -1.0), **kw):
    """2D tank with a rectangular body (x0, x1, y0, y1) cutting the free
    surface, moving with `speed` for 0.1 s and then decelerating linearly to
    rest at 0.3 s (a ditching-style history: a constant piece, then an affine
    one)."""
    case = tank2d(dx=dx, width=width, depth=depth, wall_height=depth + 0.2, **kw)
    vx, vy = speed
    motion = {"body_t": [0.0, 0.1, 0.3],
              "body_a": [[vx, vy, 0.0], [1.5 * vx, 1.5 * vy, 0.0]],
              "body_b": [[0.0, 0.0, 0.0], [-5.0 * vx, -5.0 * vy, 0.0]]}
    c = with_body(case, (body[0], body[2]), (body[1], body[3]), motion)
    c["meta"]["name"] = "entry2d"
    c["meta"]["desc"] = f"2D tank {width}x{depth} m with a body {body} moving at {speed} m/s, dx={dx}"
    return c


def ditch3d(dx=0.005, tank=(2.0, 0.8, 0.6), depth=0.3, body=((1.4, 0.25, 0.28), (1.8, 0.55, 0.38)),
            motion=None, **kw):
    """3D tank with a box body cutting the free surface (draft 2 cm at the
    defaults) and moving with the ditching velocity history of the paper by
    default.  At dx = 0.005: 3.84M fluid; all stabilisers, exact detection."""
    for k, v in (("c0", 10.0 * math.sqrt(G_EARTH * depth)), ("delta_sph", True), ("pst", True), ("tic", True),
                 ("fs_project", True), ("cont_uncorr", True), ("fs_mode", "exact")):
        kw.setdefault(k, v)
    case = box3d(dx, tank, (tank[0], tank[1], depth), name="ditch3d", **kw)
    c = with_body(case, body[0], body[1], motion or ditching_motion())
    c["meta"]["name"] = "ditch3d"
    c["meta"]["desc"] = (f"3D tank {tank} m, depth {depth} m, box body {body[0]}-{body[1]} m on the ditching "
                         f"velocity history, dx={dx}")
    return c


def cloud(n, dim, box=1.0, h=0.05, seed=0):
    """n uniform random fluid points in [0, box]^dim (no walls)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box, size=(n, dim))
    dx = h / 1.3
    params = base_params(dim, dx, domain_lo=[0.0] * 3, domain_hi=[box] * 3, depth=box)
    params["h"] = h
    params["cell_size"] = 2.0 * h
    case = _assemble(params, x, np.zeros((0, dim)), np.zeros((0, dim)), box,
                     {"name": "cloud", "desc": f"{n} random points in [0,{box}]^{dim}"})
    return case
