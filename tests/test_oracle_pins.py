"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: quadrature,
finite differences, brute force, LAPACK, closed forms, invariants of the
discrete operators, or hand-built geometry whose answer is known.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------------ kernel
@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_integrates_to_one(orc, dim):
    """Sec. 2.1 kernel: int W dV = 1 (2D with the printed 7/(4 pi h^2); 3D with
    the normalisation the oracle uses)."""
    h = 0.37
    if dim == 2:
        f = lambda r: orc.W(2, h, r / h) * 2.0 * math.pi * r
    else:
        f = lambda r: orc.W(3, h, r / h) * 4.0 * math.pi * r * r
    val, _ = integrate.quad(f, 0.0, 2.0 * h, epsabs=1e-14, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_gradient_matches_finite_difference(orc, dim):
    """grad_i W_ij = K(q) (x_j - x_i), checked by central differences of W."""
    rng = np.random.default_rng(3)
    h = 0.1
    for _ in range(20):
        xi = rng.uniform(-0.1, 0.1, dim)
        xj = rng.uniform(-0.1, 0.1, dim)
        r = xj - xi
        q = np.linalg.norm(r) / h
        if q > 1.95 or q < 0.05:
            continue
        ana = orc.K(dim, h, q) * r
        eps = 1e-6
        fd = np.zeros(dim)
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = eps
            fp = orc.W(dim, h, np.linalg.norm(xj - (xi + e)) / h)
            fm = orc.W(dim, h, np.linalg.norm(xj - (xi - e)) / h)
            fd[a] = (fp - fm) / (2 * eps)
        assert np.allclose(ana, fd, rtol=1e-6, atol=1e-6 * np.abs(ana).max())


def test_kernel_compact_support(orc):
    for dim in (2, 3):
        assert orc.W(dim, 0.2, 2.0) == 0.0
        assert orc.K(dim, 0.2, 2.0) == 0.0
        assert orc.W(dim, 0.2, 2.0 + 1e-12) == 0.0
        assert orc.W(dim, 0.2, 1.999) > 0.0


# -------------------------------------------------------------- neighbours
def _adversarial_cloud(dim, n, seed):
    """Random points plus points on cell faces and pairs at exactly 2h (h=0.5,
    2h=1: integer coordinates make the distances exact)."""
    c = wl.cloud(n, dim, box=8.0, h=0.5, seed=seed)
    rng = np.random.default_rng(seed + 100)
    extra = []
    for _ in range(60):
        p = rng.integers(1, 7, size=dim).astype(float)
        extra.append(p)
        q = p.copy()
        q[rng.integers(dim)] += 1.0  # exactly 2h away, on a cell face
        extra.append(q)
        r = p.copy()
        r[0] = np.nextafter(p[0] + 1.0, 10.0)  # one ulp beyond 2h
        extra.append(r)
    x = np.concatenate([c["x"], np.array(extra)])
    _, keep = np.unique(x, axis=0, return_index=True)
    x = x[np.sort(keep)]
    return c["params"], x


@pytest.mark.parametrize("dim,cell", [(2, 1.0), (3, 1.0), (2, 0.5), (3, 1.0 / 3.0)])
def test_cell_neighbors_equal_brute_force(orc, dim, cell):
    """Cell-list sets equal brute force, at R = 2h (Algorithm 1) and at R = h,
    2h/3 (wider stencil)."""
    pd, x = _adversarial_cloud(dim, 1500, seed=dim)
    pd = dict(pd, cell_size=cell)
    ob, ib = orc.neighbors(pd, x, mode="brute")
    oc, ic = orc.neighbors(pd, x, mode="cells")
    assert np.array_equal(ob, oc)
    for i in range(len(x)):
        assert np.array_equal(np.sort(ib[ob[i]:ob[i + 1]]), np.sort(ic[oc[i]:oc[i + 1]]))
    # symmetry of the relation
    pairs = set()
    for i in range(len(x)):
        for j in ib[ob[i]:ob[i + 1]]:
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)
    # the exact-2h pairs are in, the one-ulp-beyond pairs are out
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    assert (d <= 1.0).sum() == ob[-1]


def test_cells_closed_form(orc):
    """Eq. (ixyz): a point at lo + (k + 1/2) R is in cell k; the point at the
    upper domain corner is in the last cell, N = floor((hi - lo)/R) + 1."""
    pd = wl.base_params(3, 0.1, domain_lo=[-1.0, 0.0, 2.0], domain_hi=[1.0, 0.7, 3.1])
    R = pd["cell_size"]
    N = [int(math.floor((pd["domain_hi"][a] - pd["domain_lo"][a]) / R)) + 1 for a in range(3)]
    ks = np.array([[0, 0, 0], [3, 1, 2], [N[0] - 2, N[1] - 2, N[2] - 2]])
    x = np.array(pd["domain_lo"]) + (ks + 0.5) * R
    x = np.concatenate([x, [pd["domain_hi"]]])
    c3, hsh = orc.cells(pd, x)
    assert np.array_equal(c3[:3], ks)
    assert list(c3[3]) == [N[0] - 1, N[1] - 1, N[2] - 1]
    assert hsh[3] == (N[0] - 1) + (N[1] - 1) * N[0] + (N[2] - 1) * N[0] * N[1]
    with pytest.raises(orc.OracleError):
        orc.cells(pd, np.array([[pd["domain_hi"][0] + 1e-9, 0.1, 2.5]]))


# ------------------------------------------------------------- eigenvalues
def test_eigenvalues_match_lapack(orc):
    """Eigenvalues of sym(L) (Sec. 3) equal LAPACK's to a few ulps of |S|,
    also for repeated and nearly repeated eigenvalues (lattice rows by a wall
    give L = diag(a, a, b) up to round-off), negative and zero spectra."""
    rng = np.random.default_rng(5)
    mats = []
    for _ in range(300):
        for d in (2, 3):
            A = rng.normal(size=(d, d))
            mats.append(A @ A.T)
            mats.append(np.diag(rng.normal(size=d)))
            Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
            ev = rng.normal(size=d)
            ev[-1] = ev[0]  # repeated eigenvalue
            mats.append(Q @ np.diag(ev) @ Q.T)
            E = rng.normal(size=(d, d)) * 1e-16
            a, b = 1.0 + 0.1 * rng.normal(), 0.7 + 0.1 * rng.normal()
            mats.append(np.diag([a, a, b][:d]) + E + E.T)  # nearly repeated
            mats.append(np.full((d, d), rng.normal()))  # rank one, zeros
    for S in mats:
        d = S.shape[0]
        ref = np.linalg.eigvalsh(S)
        got = orc.eigvals(d, S)[:d]
        assert np.all(np.diff(got) >= 0)
        assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    # asymmetric input: its symmetric part is what is diagonalised
    S = rng.normal(size=(3, 3))
    assert np.abs(orc.eigvals(3, S) - np.linalg.eigvalsh(0.5 * (S + S.T))).max() <= 1e-14 * 4


# ---------------------------------------------- first-order consistency
def _fluid_block(dim, n_side, dx, seed, sigma=0.15):
    """A jittered fluid block with free surfaces on all sides, no walls."""
    hi = [n_side * dx] * dim + [0.0] * (3 - dim)
    pd = wl.base_params(dim, dx, domain_lo=[-dx] * dim + [0.0] * (3 - dim),
                        domain_hi=[n_side * dx + dx] * dim + [0.0] * (3 - dim), gravity=[0.0, 0.0, 0.0])
    x = wl._lattice([0] * dim, [n_side] * dim, dx)
    rng = np.random.default_rng(seed)
    x = x + rng.normal(0.0, sigma * dx, size=x.shape)
    n = len(x)
    return {"params": pd, "x": x, "u": np.zeros((n, dim)), "phi": np.zeros(n),
            "kind": np.zeros(n, np.uint8), "normal": np.zeros((n, dim)), "mass": None, "t": 0.0}


@pytest.mark.parametrize("dim,n_side", [(2, 24), (3, 10)])
def test_corrected_gradient_reproduces_linear_potential(orc, dim, n_side):
    """Eq. (parGrad) with Eq. (renorm): exact for linear phi on a disordered
    set with truncated supports (Sec. 2.2.2).  G = 0, U = 0 -> a = -c."""
    case = _fluid_block(dim, n_side, 0.01, seed=11)
    rng = np.random.default_rng(12)
    c = rng.normal(size=dim) * 3.0
    case["phi"] = case["x"] @ c + 0.7
    case["mass"] = np.full(len(case["x"]), 1000.0 * 0.01 ** dim)
    r = orc.eval_rates(case)
    assert r["n_singular"] == 0
    err = np.abs(r["acc"] + c).max()
    assert err <= 1e-12 * np.abs(c).max(), err
    # the truncated supports really are truncated (free-surface particles present)
    assert (r["lam"][:, 0] < 0.75).sum() > 0


@pytest.mark.parametrize("dim,n_side", [(2, 24), (3, 10)])
def test_corrected_divergence_reproduces_linear_velocity(orc, dim, n_side):
    """Continuity of Eq. (sph): sum (U_j - U_i).L^-T grad W V = tr(A) exactly
    for U = A x + b (delta-SPH off)."""
    case = _fluid_block(dim, n_side, 0.01, seed=13)
    rng = np.random.default_rng(14)
    A = rng.normal(size=(dim, dim))
    b = rng.normal(size=dim)
    case["u"] = case["x"] @ A.T + b
    case["mass"] = np.full(len(case["x"]), 1000.0 * 0.01 ** dim)
    r = orc.eval_rates(case)
    c0 = case["params"]["c0"]
    want = -c0 * c0 * np.trace(A)
    err = np.abs(r["dphi"] - want).max()
    assert err <= 1e-12 * abs(want) + 1e-12, err


# --------------------------------------------------------------- hydrostatic
def _hydro_cases():
    return [
        ("tank2d", wl.tank2d()),
        ("rect", wl.bump2d("rect", dx=0.01, width=1.0, depth=1.0, amp=0.5, bump_width=0.4)),
        ("tri", wl.bump2d("tri", dx=0.01, width=1.0, depth=1.0, amp=0.5, bump_width=0.4)),
        ("gauss", wl.bump2d("gauss", dx=0.005, width=1.0, depth=0.3, amp=0.1, sigma=0.1)),
        ("box3d", wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2))),
    ]


@pytest.mark.parametrize("name,case", _hydro_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_hydrostatic_state_is_discrete_equilibrium(orc, name, case):
    """Sec. 2.5: the hydrostatic solution satisfies the discrete system; with
    dummies mirrored by Eq. (phiBn) the accelerations vanish to round-off over
    flat, rectangular, triangular and Gaussian bottoms."""
    r = orc.eval_rates(case)
    f = case["kind"] == 0
    g = 9.81
    assert np.abs(r["acc"][f]).max() <= 1e-13 * g
    assert np.abs(r["dphi"][f]).max() == 0.0  # U = 0 exactly -> no compression
    # mirrored wall potential equals the hydrostatic field at the dummy (linear phi)
    d = (case["kind"] == 1) & (r["mir_src"] >= 0)
    assert np.allclose(r["mir_phi"][d], case["phi"][d], rtol=0, atol=1e-13)


def test_hydrostatic_window_stays_at_rest(orc):
    """2D tank (5,000 fluid), FP64, no stabilisers: spurious velocity stays at
    round-off over the first 100 steps (the literal scheme then grows from
    round-off through a free-surface mode; see the design notes)."""
    case = wl.tank2d()
    out = orc.step(case, 100)
    f = case["kind"] == 0
    assert np.abs(out["u"][f]).max() <= 1e-12
    assert np.abs(out["x"] - case["x"]).max() <= 1e-12


def test_free_surface_mode_growth_rate_is_acoustic(orc):
    """The literal scheme's free-surface mode grows at a fixed rate in physical
    time, of order C0/dx (independent of the CFL number)."""
    rates = []
    for cfl in (0.2, 0.1):
        c = wl.tank2d(cfl=cfl)
        f = c["kind"] == 0
        a = orc.step(c, int(60 * 0.2 / cfl))
        b = orc.step(a, int(60 * 0.2 / cfl))
        ua, ub = np.abs(a["u"][f]).max(), np.abs(b["u"][f]).max()
        rates.append(math.log(ub / ua) / (b["t"] - a["t"]))
    c0dx = c["params"]["c0"] / c["params"]["dx"]
    assert abs(rates[0] - rates[1]) < 0.15 * rates[0]
    assert 0.2 * c0dx < rates[0] < 1.0 * c0dx


# ------------------------------------------------------------- invariants
def test_conservative_branch_conserves_momentum(orc):
    """TIC branch (Sec. 2.3): sum_i V_i (a_i - G) = 0 by pair antisymmetry of
    (phi_i + phi_j) grad_i W_ij V_i V_j."""
    case = _fluid_block(2, 20, 0.01, seed=21)
    rng = np.random.default_rng(22)
    case["phi"] = rng.normal(size=len(case["x"]))
    case["params"] = dict(case["params"], tic=True, lambda_tic=1e9)
    m = np.full(len(case["x"]), 1000.0 * 1e-4)
    case["mass"] = m
    r = orc.eval_rates(case)
    assert r["tic"].all()
    V = m / (1000.0 * np.exp(case["phi"] / case["params"]["c0"] ** 2))
    tot = (V[:, None] * r["acc"]).sum(0)
    scale = (V[:, None] * np.abs(r["acc"])).sum(0)
    assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_delta_sph_term_is_conservative(orc):
    """delta-SPH (Sec. 2.3): sum_i V_i D_i = 0 (antisymmetric in i, j)."""
    case = _fluid_block(3, 8, 0.01, seed=23)
    rng = np.random.default_rng(24)
    case["phi"] = rng.normal(size=len(case["x"]))
    case["params"] = dict(case["params"], delta_sph=True)
    m = np.full(len(case["x"]), 1000.0 * 1e-6)
    case["mass"] = m
    r = orc.eval_rates(case)
    V = m / (1000.0 * np.exp(case["phi"] / case["params"]["c0"] ** 2))
    tot = (V * r["dphi"]).sum()
    assert abs(tot) <= 1e-13 * (V * np.abs(r["dphi"])).sum()
    assert np.abs(r["dphi"]).max() > 0


def test_riemann_term_galilean_and_dissipative(orc):
    """Eq. (lfsover): the dissipation depends on velocity differences only
    (uniform U adds nothing), and opposes an interior particle's motion
    relative to its neighbours."""
    case = _fluid_block(2, 20, 0.01, seed=25, sigma=0.0)
    case["mass"] = np.full(len(case["x"]), 0.1)
    r0 = orc.eval_rates(case)
    cu = dict(case)
    cu["u"] = np.tile([0.3, -0.2], (len(case["x"]), 1))
    ru = orc.eval_rates(cu)
    assert np.abs(ru["acc"] - r0["acc"]).max() <= 1e-12
    # one interior particle moving: LF acceleration opposes its velocity
    i = int(np.argmin(np.linalg.norm(case["x"] - case["x"].mean(0), axis=1)))
    cm = dict(case)
    u = np.zeros_like(case["u"])
    u[i] = [0.5, 0.2]
    cm["u"] = u
    rm = orc.eval_rates(cm)
    assert np.dot(rm["acc"][i] - r0["acc"][i], u[i]) < 0


def test_particle_shifting_bounds(orc):
    """Sec. 2.3 PST: |dU| <= U_max / 2; dU = 0 when U_max = 0; ~0 in the
    interior of a regular lattice (symmetric support)."""
    case = wl.tank2d(pst=True)
    r0 = orc.eval_rates(case)
    assert np.abs(r0["dushift"]).max() == 0.0
    cu = wl.random_velocity(wl.jitter(case, 0.1, seed=3), amp=0.05, seed=4)
    r = orc.eval_rates(cu)
    umax = r["umax"]
    f = case["kind"] == 0
    assert np.linalg.norm(r["dushift"][f], axis=1).max() <= 0.5 * umax * (1 + 1e-14)
    # regular lattice, interior: shifting vanishes by symmetry
    cl = dict(case)
    cl["u"] = np.where(f[:, None], 0.05, 0.0) * np.ones_like(case["u"])
    rl = orc.eval_rates(cl)
    y = case["x"][:, 1]
    xx = case["x"][:, 0]
    interior = f & (y > 0.1) & (y < 0.4) & (xx > 0.1) & (xx < 0.9)
    assert np.abs(rl["dushift"][interior]).max() <= 1e-12 * 0.05


def test_free_fall_is_exact_under_ssp_rk2(orc):
    """An isolated particle (L singular -> conservative branch, no neighbours)
    falls as x0 + U0 t + G t^2 / 2: SSP-RK2 is exact for constant acceleration."""
    pd = wl.base_params(2, 0.01, domain_lo=[-10, -10, 0], domain_hi=[10, 10, 0])
    case = {"params": pd, "x": np.array([[0.3, 0.4]]), "u": np.array([[0.7, 1.1]]),
            "phi": np.array([0.2]), "kind": np.zeros(1, np.uint8), "normal": np.zeros((1, 2)),
            "mass": None, "t": 0.0}
    out = orc.step(case, 50)
    t = out["t"]
    G = np.array([0.0, -9.81])
    want = case["x"][0] + case["u"][0] * t + 0.5 * G * t * t
    assert np.allclose(out["x"][0], want, rtol=0, atol=1e-14)
    assert np.allclose(out["u"][0], case["u"][0] + G * t, rtol=0, atol=1e-13)


def test_time_step_rule(orc):
    """Sec. 2.3: dt = CFL min(dx/(C0+|U|), dx^2/(2 nu), sqrt(2 dx/|G|)); at the
    2D tank (dx 0.01, C0 = 10 sqrt(g 0.5)) the acoustic limit binds."""
    case = wl.tank2d()
    assert abs(orc.dt(case) - 0.2 * 0.01 / (10 * math.sqrt(9.81 * 0.5))) < 1e-18
    c2 = wl.tank2d(nu=1.0)  # viscous limit: dx^2 / (2 nu)
    assert abs(orc.dt(c2) - 0.2 * 1e-4 / 2.0) < 1e-18


# ------------------------------------------------------- lattice values
def test_interior_correction_matrix_on_lattice(orc):
    """Interior of a regular lattice: L is isotropic, close to I (the continuum
    value of sum r (x) grad W V), and its value matches the direct lattice sum
    0.974 (2D) / 0.979 (3D) at h = 1.3 dx; the flat top layer has
    lambda_min ~ 0.487 (2D) / 0.489 (3D)."""
    for dim, want_int, want_top, case in (
            (2, 0.974, 0.487, wl.tank2d()),
            (3, 0.979, 0.489, wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2)))):
        r = orc.eval_rates(case)
        f = case["kind"] == 0
        x = case["x"]
        top = x[f, dim - 1].max()
        lam = r["lam"]
        # walls are completed by lattice dummies of equal volume: every fluid
        # particle deeper than 2h below the surface has a full, regular support
        interior = f & (x[:, dim - 1] < top - 2.0 * case["params"]["h"] - 0.1 * case["params"]["dx"])
        li = lam[interior][:, :dim]
        assert len(li) > 100
        assert np.allclose(li, li[0, 0], atol=1e-12)
        assert abs(li[0, 0] - want_int) < 5e-4
        surf = f & (x[:, dim - 1] == top)
        for a in range(dim - 1):
            surf &= (x[:, a] > 0.1) & (x[:, a] < x[f][:, a].max() - 0.1)
        assert abs(lam[surf, 0].mean() - want_top) < 5e-4


def test_neighbour_counts_on_lattice(orc):
    """|N(i)| in the lattice interior equals the number of lattice points within
    2h = 2.6 dx (counted by enumeration)."""
    for dim, case in ((2, wl.tank2d()), (3, wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2)))):
        k = np.arange(-3, 4)
        grid = np.stack(np.meshgrid(*([k] * dim), indexing="ij"), -1).reshape(-1, dim)
        cnt = int(((grid ** 2).sum(1) <= 2.6 ** 2).sum()) - 1
        r = orc.eval_rates(case)
        assert r["nnb"].max() == cnt
    assert cnt == 80


# ----------------------------------------------------------- free surface
def _fs_case(points, dx=0.01):
    pts = np.asarray(points, dtype=float)
    n = len(pts)
    pd = wl.base_params(2, dx, domain_lo=[-1, -1, 0], domain_hi=[1, 1, 0], fs_mode="exact",
                        gravity=[0, -9.81, 0])
    return {"params": pd, "x": pts, "u": np.zeros((n, 2)), "phi": np.zeros(n),
            "kind": np.zeros(n, np.uint8), "normal": np.zeros((n, 2)), "mass": np.full(n, 0.1),
            "t": 0.0}


def test_scan_region_hand_built(orc):
    """Scan-region test around T = x_i + h n (free-surface detection)."""
    dx = 0.01
    lat = wl._lattice([0, 0], [20, 10], dx)  # flat free surface at the top row
    top = np.argmax(np.where(np.abs(lat[:, 0] - 0.105) < 1e-12, lat[:, 1], -1))
    r = orc.eval_rates(_fs_case(lat))
    assert 0.2 < r["lam"][top, 0] <= 0.75  # a candidate, decided by the scan
    assert r["fs"][top] == 1
    assert np.allclose(r["normal"][top], [0.0, 1.0], atol=1e-12)
    below = top - 1
    assert r["fs"][below] == 0  # lambda > 0.75
    # a particle straight above inside the scan cone hides the top particle
    above = lat[top] + np.array([0.0, 1.0 * dx])
    r2 = orc.eval_rates(_fs_case(np.concatenate([lat, [above]])))
    assert r2["fs"][top] == 0 and r2["fs"][-1] == 1
    # farther out (s >= sqrt2 h) but within h of T: still hides it
    above2 = lat[top] + np.array([0.0, 1.9 * dx])
    r3 = orc.eval_rates(_fs_case(np.concatenate([lat, [above2]])))
    assert r3["fs"][top] == 0
    # isolated particle and a droplet of three: all on the surface
    assert orc.eval_rates(_fs_case([[0.0, 0.0]]))["fs"][0] == 1
    d3 = orc.eval_rates(_fs_case([[0.0, 0.0], [dx, 0.0], [0.5 * dx, 0.8 * dx]]))
    assert d3["fs"].all()


def test_mirror_dummy_hand_built(orc):
    """Eq. (phiBn) and the slip condition on a two-particle case; ties go to the
    lower index; a dummy beyond 2h of every fluid particle is inactive."""
    dx = 0.01
    pd = wl.base_params(2, dx, domain_lo=[-1, -1, 0], domain_hi=[1, 1, 0])
    x = np.array([[0.0, 0.01], [0.02, 0.01], [0.01, -0.005], [0.5, 0.5]])
    kind = np.array([0, 0, 1, 1], np.uint8)
    u = np.array([[0.3, -0.4], [1.0, 1.0], [0, 0], [0, 0]], float)
    nd = np.array([[0, 0], [0, 0], [0.0, 1.0], [0.0, 1.0]])
    phi = np.array([2.0, 3.0, 0.0, 0.0])
    case = {"params": pd, "x": x, "u": u, "phi": phi, "kind": kind, "normal": nd,
            "mass": np.full(4, 0.1), "t": 0.0}
    r = orc.eval_rates(case)
    assert r["mir_src"][2] == 0  # equidistant from both fluid particles: lower index
    assert r["mir_phi"][2] == pytest.approx(2.0 + (-9.81) * (-0.005 - 0.01), abs=1e-15)
    assert np.allclose(r["mir_u"][2], [0.3, 0.0])
    assert r["mir_src"][3] == -1


def test_sampled_rows_equal_full_evaluation(orc):
    """Evaluating a sample of rows (lists built for those rows and the dummies
    they touch) gives bit for bit the full evaluation's values on the sample:
    the sampled mode used against the GPU at full size drops no term."""
    case = wl.box3d(0.03, (0.6, 0.3, 0.45), (0.3, 0.3, 0.3))
    case = wl.with_params(case, delta_sph=True, pst=True, tic=True, fs_mode="exact")
    case = wl.random_velocity(wl.jitter(case, 0.05, 3), 0.05, 4)
    full = orc.eval_rates(case)
    f = np.nonzero(case["kind"] == 0)[0]
    rng = np.random.default_rng(5)
    top = f[np.argsort(case["x"][f, 2])[-20:]]
    rows = np.unique(np.concatenate([rng.choice(f, 60, replace=False), top]))
    sub = orc.eval_rates(case, rows=rows)
    for k in ("acc", "dphi", "dushift", "lam", "normal", "fs", "tic", "nnb", "feat", "fs_margin"):
        assert np.array_equal(sub[k][rows], full[k][rows]), k
    assert full["fs"][top].any()
    other = np.setdiff1d(f, rows)
    assert not sub["nnb"][other].any()
