"""Pins of the oracle's individual terms of Eq. (sph) and Sec. 2.3, each
against a closed form that follows from the term's definition and the
geometry of the case, not from retyping the oracle's arithmetic:

* delta-SPH (Sec. 2.3): for phi = a/2 |x - x_i|^2 centred on particle i,
  Phi_ij . grad W = a r . grad W for the radial kernel, so D_i = delta h C0 a
  tr(L_i) exactly, at any particle of any configuration (tr L from the
  oracle's eigenvalues);
* the Lax-Friedrichs term of Eq. (lfsover): a symmetric lattice interior
  (L = l I) at rest except one neighbour j moving with w gives
  a_i = C0 (w . e) |dW/ds| V_j e / l, e = (x_j - x_i)/|x_j - x_i|, with dW/ds
  from central differences of W;
* particle shifting (Sec. 2.3): the same interior with neighbour j removed
  gives sum [1 + R (W/W(dx))^n] grad W V = -(that of j), so the shifting
  velocity points towards the vacancy with magnitude 2 h U_max [1 + R
  (W(s)/W(dx))^n] |dW/ds| V_j (below the U_max/2 clamp);
* the conservative (TIC) branch: phi linear and zero at x_i gives
  S_C = L^T b = l b at a symmetric interior, a_i = -l b + G; a uniform phi0
  gives S_C = 2 phi0 sum grad W V (brute-force sum) at edges and corners;
* the uncorrected continuity at TIC particles: U = A (x - x_i) gives
  N = A L, so -C0^2 tr N = -C0^2 l tr A (against -C0^2 tr A corrected);
* the free-surface projection: at flagged surface particles the shifting
  velocity has no normal component.

Each check is a plain function so that test_oracle_mutations.py can run it
against variants of the oracle with planted mistakes.
"""
import numpy as np

import oracle
import workloads as wl

DX = 0.01


def _block(dim, n_side, c0=10.0, gravity=None, **flags):
    """Square (cubic) lattice block of fluid, no walls, spacing DX."""
    g = [0.0, 0.0, 0.0] if gravity is None else gravity
    pd = wl.base_params(dim, DX, c0=c0, gravity=g, domain_lo=[-2 * DX] * dim + [0.0] * (3 - dim),
                        domain_hi=[(n_side + 2) * DX] * dim + [0.0] * (3 - dim), **flags)
    x = wl._lattice([0] * dim, [n_side] * dim, DX)
    n = len(x)
    return {"params": pd, "x": x, "u": np.zeros((n, dim)), "phi": np.zeros(n), "kind": np.zeros(n, np.uint8),
            "normal": np.zeros((n, dim)), "mass": None, "t": 0.0}


def _uniform_volume(case):
    """Masses that make every V = m / rho(phi) equal to dx^d."""
    c = dict(case)
    c["mass"] = oracle.mass_from_phi(c["params"], c["phi"])
    return c


def _centre(case):
    n_side = round(len(case["x"]) ** (1.0 / case["params"]["dim"]))
    mid = n_side // 2
    dim = case["params"]["dim"]
    idx = sum(mid * n_side ** (dim - 1 - a) for a in range(dim))  # lattice() is 'ij' ordered
    assert np.allclose(case["x"][idx], (mid + 0.5) * DX)
    return idx


def _dwds(dim, h, s):
    """dW/ds by central differences of the oracle's W (pinned elsewhere by
    quadrature and by its own finite-difference check of grad W)."""
    e = 1e-7 * h
    return (oracle.W(dim, h, (s + e) / h) - oracle.W(dim, h, (s - e) / h)) / (2.0 * e)


def check_delta_sph_closed_form(dim):
    a = 37.0
    rng = np.random.default_rng(40 + dim)
    base = wl.jitter(_block(dim, 9 if dim == 2 else 6, delta_sph=True), 0.12, seed=41 + dim)
    h, c0, delta = base["params"]["h"], base["params"]["c0"], base["params"]["delta"]
    n = len(base["x"])
    # centre particles: interior, edge and corner rows of a disordered block
    for i in sorted(set(rng.integers(0, n, 5).tolist()) | {0, n - 1, n // 2}):
        c = dict(base)
        d = base["x"] - base["x"][i]
        c["phi"] = 0.5 * a * (d * d).sum(1) + 3.0
        c = _uniform_volume(c)
        r = oracle.eval_rates(c)
        trL = r["lam"][i, :dim].sum()
        want = delta * h * c0 * a * trL
        got = r["dphi"][i]
        assert want > 0.0
        assert abs(got - want) <= 1e-10 * abs(want), (i, got, want)


def check_riemann_term_magnitude(dim):
    case = _uniform_volume(_block(dim, 9 if dim == 2 else 7))
    h, c0 = case["params"]["h"], case["params"]["c0"]
    i = _centre(case)
    d = case["x"] - case["x"][i]
    s = np.sqrt((d * d).sum(1))
    nbr = np.nonzero((s > 0) & (s <= 2 * h))[0]
    rng = np.random.default_rng(50 + dim)
    for j in nbr[rng.permutation(len(nbr))[:4]]:
        c = dict(case)
        w = rng.normal(size=dim)
        c["u"] = np.zeros_like(case["u"])
        c["u"][j] = w
        r = oracle.eval_rates(c)
        lam = r["lam"][i, :dim]
        assert lam.max() - lam.min() < 1e-12 * lam.max()  # L = l I at the symmetric interior
        e = d[j] / s[j]
        V = DX ** dim
        want = c0 * (w @ e) * abs(_dwds(dim, h, s[j])) * V * e / lam[0]
        got = r["acc"][i]
        assert np.abs(got - want).max() <= 1e-7 * np.abs(want).max() + 1e-12, (j, got, want)


def check_shifting_toward_vacancy(dim):
    full = _block(dim, 9 if dim == 2 else 7, pst=True)
    h = full["params"]["h"]
    R, npow = full["params"]["pst_R"], full["params"]["pst_n"]
    i = _centre(full)
    d = full["x"] - full["x"][i]
    s = np.sqrt((d * d).sum(1))
    far = int(np.argmax(s))  # corner particle outside i's support carries U_max
    assert s[far] > 2 * h
    nbr = np.nonzero((s > 0) & (s <= 2 * h))[0]
    umax = 1.3
    w0 = oracle.W(dim, h, DX / h)

    def expected(j):
        weight = 1.0 + R * (oracle.W(dim, h, s[j] / h) / w0) ** npow
        return weight, 2.0 * h * umax * weight * abs(_dwds(dim, h, s[j])) * DX ** dim

    # the nearest vacancy (largest shifting weight) and the farthest one; in
    # 2D the nearest one is clamped to U_max/2 and checked as such, and the
    # nearest unclamped one (the diagonal) carries the magnitude check
    near = nbr[np.argmin(s[nbr])]
    unclamped = [j for j in nbr[np.argsort(s[nbr])] if expected(j)[1] < 0.45 * umax]
    for j in sorted({int(near), int(unclamped[0]), int(nbr[np.argmax(s[nbr])])}):
        keep = np.arange(len(full["x"])) != j
        c = {k: (v[keep] if isinstance(v, np.ndarray) else v) for k, v in full.items()}
        c["u"] = np.zeros_like(c["u"])
        far_k = far - (1 if far > j else 0)
        c["u"][far_k, 0] = umax
        c = _uniform_volume(c)
        ii = i - (1 if i > j else 0)
        r = oracle.eval_rates(c)
        weight, mag = expected(j)
        e = d[j] / s[j]
        want = min(mag, 0.5 * umax) * e
        got = r["dushift"][ii]
        assert np.abs(got - want).max() <= 1e-7 * np.abs(want).max(), (j, got, want, weight)


def check_conservative_branch_linear_phi(dim):
    case = _block(dim, 9 if dim == 2 else 7, tic=True, gravity=[0.3, -9.81, 0.2][:dim] + [0.0] * (3 - dim))
    case["params"]["lambda_tic"] = 2.0  # every particle takes the conservative branch
    i = _centre(case)
    rng = np.random.default_rng(60 + dim)
    b = rng.normal(size=dim) * 5.0
    case["phi"] = (case["x"] - case["x"][i]) @ b
    case = _uniform_volume(case)
    r = oracle.eval_rates(case)
    assert r["tic"][i] == 1
    lam = r["lam"][i, :dim]
    assert lam.max() - lam.min() < 1e-12 * lam.max()
    G = np.asarray(case["params"]["gravity"][:dim])
    want = -lam[0] * b + G
    assert np.abs(r["acc"][i] - want).max() <= 1e-11 * np.abs(want).max(), (r["acc"][i], want)
    # the corrected branch at the same state reproduces the linear potential
    c2 = dict(case)
    c2["params"] = dict(case["params"], tic=False)
    r2 = oracle.eval_rates(c2)
    assert np.abs(r2["acc"][i] - (-b + G)).max() <= 1e-11 * np.abs(b).max()


def check_conservative_branch_uniform_phi(dim):
    """The conservative form is not zeroth-order consistent: with a uniform
    phi0 it gives S_C = 2 phi0 sum grad W V, non-zero at the block's edges
    and corners (sum taken here by brute force, dW/ds by differences)."""
    case = _block(dim, 7 if dim == 2 else 5, tic=True)
    case["params"]["lambda_tic"] = 2.0
    phi0 = 5.0
    case["phi"] = np.full(len(case["x"]), phi0)
    case = _uniform_volume(case)
    h = case["params"]["h"]
    r = oracle.eval_rates(case)
    for i in (0, len(case["x"]) // 2, 3):
        d = case["x"] - case["x"][i]
        s = np.sqrt((d * d).sum(1))
        g = np.zeros(dim)
        size = 0.0  # sum of the terms' magnitudes: the scale of the differences' error
        for j in np.nonzero((s > 0) & (s <= 2 * h))[0]:
            term = abs(_dwds(dim, h, s[j])) * DX ** dim
            g += term * d[j] / s[j]
            size += term
        want = -2.0 * phi0 * g
        assert r["tic"][i] == 1
        assert np.abs(r["acc"][i] - want).max() <= 1e-7 * 2.0 * phi0 * size, (i, r["acc"][i], want)
        if i == 0:  # the corner: far from zero
            assert np.abs(want).max() > 0.1 * 2.0 * phi0 * size


def check_uncorrected_continuity_at_tic(dim):
    rng = np.random.default_rng(70 + dim)
    A = rng.normal(size=(dim, dim))
    out = {}
    for cu in (True, False):
        case = _block(dim, 9 if dim == 2 else 7, tic=True, cont_uncorr=cu)
        case["params"]["lambda_tic"] = 2.0
        i = _centre(case)
        case["u"] = (case["x"] - case["x"][i]) @ A.T
        case = _uniform_volume(case)
        r = oracle.eval_rates(case)
        lam = r["lam"][i, :dim]
        assert lam.max() - lam.min() < 1e-12 * lam.max()
        out[cu] = (r["dphi"][i], lam[0])
    c0 = 10.0
    got_u, l = out[True]
    got_c, _ = out[False]
    assert abs(got_u - (-c0 * c0 * l * np.trace(A))) <= 1e-11 * c0 * c0 * np.abs(A).max(), (got_u, l)
    assert abs(got_c - (-c0 * c0 * np.trace(A))) <= 1e-11 * c0 * c0 * np.abs(A).max(), got_c


def check_free_surface_projection():
    base = wl.random_velocity(wl.tank2d(dx=0.02, pst=True, fs_mode="exact"), 0.2, seed=81)
    res = {}
    for proj in (True, False):
        c = wl.with_params(base, fs_project=proj)
        res[proj] = oracle.eval_rates(c)
    f = base["kind"] == 0
    fs = (res[True]["fs"] == 1) & f
    assert fs.sum() > 20
    du, n = res[True]["dushift"][fs], res[True]["normal"][fs]
    scale = np.abs(res[True]["dushift"][f]).max()
    assert scale > 0
    assert np.abs((du * n).sum(1)).max() <= 1e-14 * scale
    # without the projection the same particles do have normal components,
    # and the tangential parts agree
    du0 = res[False]["dushift"][fs]
    dn0 = (du0 * n).sum(1)
    assert np.abs(dn0).max() > 1e-3 * scale
    assert np.abs(du - (du0 - dn0[:, None] * n)).max() <= 1e-14 * scale
    # interior particles are untouched by it
    inner = f & (res[True]["fs"] == 0)
    assert np.array_equal(res[True]["dushift"][inner], res[False]["dushift"][inner])


CHECKS = {
    "delta_sph_2d": lambda: check_delta_sph_closed_form(2),
    "delta_sph_3d": lambda: check_delta_sph_closed_form(3),
    "riemann_2d": lambda: check_riemann_term_magnitude(2),
    "riemann_3d": lambda: check_riemann_term_magnitude(3),
    "shifting_2d": lambda: check_shifting_toward_vacancy(2),
    "shifting_3d": lambda: check_shifting_toward_vacancy(3),
    "conservative_2d": lambda: check_conservative_branch_linear_phi(2),
    "conservative_3d": lambda: check_conservative_branch_linear_phi(3),
    "conservative_uniform_2d": lambda: check_conservative_branch_uniform_phi(2),
    "conservative_uniform_3d": lambda: check_conservative_branch_uniform_phi(3),
    "cont_uncorr_2d": lambda: check_uncorrected_continuity_at_tic(2),
    "cont_uncorr_3d": lambda: check_uncorrected_continuity_at_tic(3),
    "fs_projection": check_free_surface_projection,
}


def test_delta_sph_closed_form(orc):
    check_delta_sph_closed_form(2)
    check_delta_sph_closed_form(3)


def test_riemann_term_magnitude(orc):
    check_riemann_term_magnitude(2)
    check_riemann_term_magnitude(3)


def test_shifting_toward_vacancy(orc):
    check_shifting_toward_vacancy(2)
    check_shifting_toward_vacancy(3)


def test_conservative_branch_linear_phi(orc):
    check_conservative_branch_linear_phi(2)
    check_conservative_branch_linear_phi(3)


def test_conservative_branch_uniform_phi(orc):
    check_conservative_branch_uniform_phi(2)
    check_conservative_branch_uniform_phi(3)


def test_uncorrected_continuity_at_tic(orc):
    check_uncorrected_continuity_at_tic(2)
    check_uncorrected_continuity_at_tic(3)


def test_free_surface_projection(orc):
    check_free_surface_projection()
