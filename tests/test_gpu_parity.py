"""GPU (HIP, FP64 path) against the CPU oracle on the same seeded inputs.

Bars: cell indices and neighbour sets bit-exact; FP64 fields within 1e-12 of
the field's scale (see _scale); flags exact except particles whose decision
sits within a tie margin in the oracle (at most MAX_TIES rows per case; none
occur in the cases here); trajectories within 1e-12 of their scale.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

TOL = 1e-12
MAX_TIES = 2


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


def _flags_all(**kw):
    return dict(delta_sph=True, pst=True, tic=True, fs_project=True, cont_uncorr=True, fs_mode="exact", **kw)


def _cases():
    t2 = wl.tank2d(dx=0.01)
    dyn2 = wl.random_potential(wl.random_velocity(wl.jitter(wl.tank2d(dx=0.01, **_flags_all()), 0.1, 3), 0.05, 4),
                               0.05, 5)
    box = wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2), **_flags_all())
    dyn3 = wl.random_velocity(wl.jitter(box, 0.1, 6), 0.05, 7)
    gauss = wl.bump2d("gauss", dx=0.005, width=1.0, depth=0.3, amp=0.1, sigma=0.1)
    fine = wl.with_params(dyn3, cell_size=dyn3["params"]["h"])            # reach 2
    finer = wl.with_params(dyn2, cell_size=2.0 * dyn2["params"]["h"] / 3.0)  # reach 3
    slosh = wl.slosh3d(dx=0.02, tank=(0.4, 0.2, 0.3), depth=0.14)
    slosh = wl.random_velocity(wl.jitter(slosh, 0.1, 8), 0.02, 9)
    slosh["t"] = 0.37  # forcing phase != 0
    return [("tank2d-hydro", t2), ("tank2d-dyn", dyn2), ("box3d-dyn", dyn3), ("gauss2d", gauss),
            ("box3d-R=h", fine), ("tank2d-R=2h/3", finer), ("slosh3d-forced", slosh)]


CASES = _cases()


def _rel(a, b, scale):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / scale) if np.size(a) else 0.0


def compare_rates(sim, case, ref, tol=TOL):
    """Element-wise comparison of every output of one right-hand side."""
    f = case["kind"] == 0
    d = case["kind"] != 0
    pd = case["params"]
    gmag = float(np.linalg.norm(pd["gravity"])) or 1.0
    acc = sim.field("dudt")
    s_acc = max(gmag, np.abs(ref["acc"][f]).max())
    assert _rel(acc[f], ref["acc"][f], s_acc) <= tol
    dphi = sim.field("dphidt")
    s_dphi = max(np.abs(ref["dphi"][f]).max(), pd["c0"] * gmag * pd["h"])
    assert _rel(dphi[f], ref["dphi"][f], s_dphi) <= tol
    dus = sim.field("delta_u")
    s_dus = max(np.abs(ref["dushift"][f]).max(), 1e-3 * max(ref["umax"], 1e-30))
    # shifting is projected at free-surface particles: compare where the FS flags agree
    lam = sim.field("lambda")
    assert np.abs(lam[f] - ref["lam"][f]).max() <= tol * max(1.0, np.abs(ref["lam"][f]).max())
    nnb = sim.field("nnb")
    assert np.array_equal(nnb[f], ref["nnb"][f])
    # flags: exact except ties within the oracle's own decision margin
    lmin = ref["lam"][f, 0]
    near = np.zeros(f.sum(), bool)
    for thr in (pd["lambda_tic"], pd["lambda_fs_lo"], pd["lambda_fs_hi"], pd["lambda_singular"]):
        near |= np.abs(lmin - thr) < 1e-10
    tic = sim.field("tic")
    assert np.array_equal(tic[f][~near], ref["tic"][f][~near])
    fs = sim.field("fs")
    tie = near | (ref["fs_margin"][f] < 1e-9 * pd["h"] ** 2)
    # the rows left out of the flag comparison: at most MAX_TIES per case
    assert tie.sum() <= MAX_TIES, (int(near.sum()), int(tie.sum()))
    assert np.array_equal(fs[f][~tie], ref["fs"][f][~tie])
    agree = (fs[f] == ref["fs"][f])
    assert _rel(dus[f][agree], ref["dushift"][f][agree], s_dus) <= tol
    # normals where they are defined (|L^-T g| h well above round-off)
    nrm = sim.field("normal")
    defined = ref["feat"][f, 11] > 1e-6
    if defined.any():
        assert np.abs(nrm[f][defined] - ref["normal"][f][defined]).max() <= 1e-9
    # dummy mirror: source, potential, velocity
    if d.any():
        src = sim.field("mirror_src")
        assert np.array_equal(src[d], ref["mir_src"][d])
        act = d & (ref["mir_src"] >= 0)
        phi = sim.field("phi")
        s_phi = max(np.abs(ref["mir_phi"][act]).max(), 1.0) if act.any() else 1.0
        assert _rel(phi[act], ref["mir_phi"][act], s_phi) <= tol
        u = sim.field("u")
        if act.any():
            s_u = max(np.abs(ref["mir_u"][act]).max(), 1e-3)
            assert _rel(u[act], ref["mir_u"][act], s_u) <= tol
    return {"acc": _rel(acc[f], ref["acc"][f], s_acc), "dphi": _rel(dphi[f], ref["dphi"][f], s_dphi)}


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_cells_bit_exact(Sim, name, case):
    sim = Sim(case)
    cell = sim.field("cell")
    c3, _ = oracle.cells(case["params"], case["x"])
    assert np.array_equal(cell, c3)


@pytest.mark.parametrize("name,case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_neighbors_bit_exact(Sim, name, case):
    sim = Sim(case)
    off, ids = sim.neighbors()
    ro, ri = oracle.neighbors(case["params"], case["x"], mode="brute")
    f = np.nonzero(case["kind"] == 0)[0]
    for i in f:
        assert np.array_equal(ids[off[i]:off[i + 1]], ri[ro[i]:ro[i + 1]]), i
    d = np.nonzero(case["kind"] == 1)[0]
    assert all(off[i + 1] == off[i] for i in d)


def test_neighbors_adversarial_cloud(Sim):
    """Random cloud plus pairs at exactly 2h and one ulp beyond, on cell faces."""
    from tests.test_oracle_pins import _adversarial_cloud
    for dim in (2, 3):
        pd, x = _adversarial_cloud(dim, 1200, seed=10 + dim)
        n = len(x)
        case = {"params": pd, "x": x, "u": np.zeros((n, dim)), "phi": np.zeros(n), "kind": np.zeros(n, np.uint8),
                "normal": np.zeros((n, dim)), "mass": None, "t": 0.0}
        sim = Sim(case)
        off, ids = sim.neighbors()
        ro, ri = oracle.neighbors(pd, x, mode="brute")
        assert np.array_equal(off, ro)
        assert np.array_equal(ids, ri)
        assert np.array_equal(sim.field("cell"), oracle.cells(pd, x)[0])


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_rates_parity(Sim, name, case):
    sim = Sim(case)
    sim.eval_rates()
    ref = oracle.eval_rates(case)
    compare_rates(sim, case, ref)


def test_features_parity(Sim):
    case = wl.with_params(CASES[2][1], features=True)
    sim = Sim(case)
    sim.eval_rates()
    ref = oracle.eval_rates(case)
    f = case["kind"] == 0
    ft = sim.field("features")[f].astype(np.float64)
    rf = ref["feat"][f]
    defined = rf[:, 11] > 1e-6
    for k in range(16):
        rows = defined if k in (7, 8, 9, 10, 12) else np.ones(len(rf), bool)
        scale = max(np.abs(rf[rows, k]).max(), 1e-6)
        assert np.abs(ft[rows, k] - rf[rows, k]).max() <= 2e-6 * scale, k


def test_hydrostatic_tank_gpu(Sim):
    """2D tank (5,000 fluid), FP64, no stabilisers: discrete equilibrium and
    spurious velocity <= 1e-12 over 100 steps, matching the oracle."""
    case = wl.tank2d()
    sim = Sim(case)
    sim.eval_rates()
    f = case["kind"] == 0
    assert np.abs(sim.field("dudt")[f]).max() <= 1e-13 * 9.81
    sim.step(100)
    u = sim.field("u")
    assert np.abs(u[f]).max() <= 1e-12
    ref = oracle.step(case, 100)
    assert np.abs(sim.field("x") - ref["x"]).max() <= 1e-13
    st = sim.stats()
    assert abs(st["t"] - ref["t"]) <= 1e-15 and st["steps"] == 100


def test_hydrostatic_tank_200_steps_surface_mode(Sim):
    """The 2D tank's 200 steps (5,000 fluid, FP64, no stabilisers), stated as
    they come out.  The tank is an exact discrete equilibrium and stays below
    1e-12 m/s through step 100; then the literal scheme's free-surface mode
    grows from round-off: the linearised right-hand side has a real
    eigenvalue of 0.605 C0/dx in the top particle layer (pinned on the CPU in
    test_oracle_surface_mode.py), so max |U| passes 1e-12 between steps 100
    and 150 and the 1e-12 target does not hold at 200 steps under this
    reading.  Asserted: the window, the growth rate between steps 150 and 200
    within 10% of what SSP-RK2 gives that eigenvalue, and max |U| at step 200
    within a factor 10 of the oracle's (each grows from its own round-off)."""
    import math
    from tests.test_oracle_surface_mode import rk2_rate
    case = wl.tank2d()
    f = case["kind"] == 0
    sim = Sim(case)
    sim.step(100)
    assert np.abs(sim.field("u")[f]).max() <= 1e-12
    sim.step(50)
    u150, t150 = np.abs(sim.field("u")[f]).max(), sim.stats()["t"]
    sim.step(50)
    u200, t200 = np.abs(sim.field("u")[f]).max(), sim.stats()["t"]
    dt = sim.stats()["dt"]
    print(f"max |U|: step 150 {u150:.3e}, step 200 {u200:.3e}")
    assert u200 > 1e-12  # the mode, not a pass of the target
    c0dx = case["params"]["c0"] / case["params"]["dx"]
    rate, want = math.log(u200 / u150) / (t200 - t150), rk2_rate(0.605 * c0dx, dt)
    assert abs(rate - want) <= 0.10 * want, (rate, want)
    ref = oracle.step(case, 200)
    u_ref = np.abs(ref["u"][f]).max()
    assert 0.1 * u_ref <= u200 <= 10.0 * u_ref, (u200, u_ref)


@pytest.mark.parametrize("name,case,nsteps", [
    ("tank2d-dyn", CASES[1][1], 10),
    ("dambreak3d-mini", wl.dambreak3d(dx=0.04, tank=(0.8, 0.4, 0.4), column=(0.3, 0.4, 0.22)), 10),
], ids=["tank2d-dyn", "dambreak3d-mini"])
def test_trajectory_parity(Sim, name, case, nsteps):
    sim = Sim(case)
    sim.step(nsteps)
    ref = oracle.step(case, nsteps)
    f = case["kind"] == 0
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    assert np.abs(sim.field("x")[f] - ref["x"][f]).max() <= 1e-12 * L
    umax = max(np.abs(ref["u"][f]).max(), 1e-3)
    assert np.abs(sim.field("u")[f] - ref["u"][f]).max() <= 1e-12 * umax
    pmax = np.abs(ref["phi"][f]).max()
    assert np.abs(sim.field("phi")[f] - ref["phi"][f]).max() <= 1e-12 * pmax
    assert abs(sim.stats()["t"] - ref["t"]) <= 1e-15


def test_single_particle_free_fall(Sim):
    pd = wl.base_params(2, 0.01, domain_lo=[-10, -10, 0], domain_hi=[10, 10, 0])
    case = {"params": pd, "x": np.array([[0.3, 0.4]]), "u": np.array([[0.7, 1.1]]), "phi": np.array([0.2]),
            "kind": np.zeros(1, np.uint8), "normal": np.zeros((1, 2)), "mass": None, "t": 0.0}
    sim = Sim(case)
    sim.step(50)
    ref = oracle.step(case, 50)
    assert np.abs(sim.field("x") - ref["x"]).max() <= 1e-14
    assert np.abs(sim.field("u") - ref["u"]).max() <= 1e-13


def test_out_of_domain_is_reported(Sim):
    """A particle pushed out of the hashed box by its own velocity is reported
    as SPH_EDOMAIN at the next synchronising call; the context then refuses
    further steps but still serves fields."""
    from paper_2608_22269_amd import _lib as L
    pd = wl.base_params(2, 0.01, domain_lo=[0, 0, 0], domain_hi=[1, 1, 0], gravity=[0, 0, 0])
    case = {"params": pd, "x": np.array([[0.5, 0.5], [0.9995, 0.5]]), "u": np.array([[0.0, 0.0], [50.0, 0.0]]),
            "phi": np.zeros(2), "kind": np.zeros(2, np.uint8), "normal": np.zeros((2, 2)), "mass": None, "t": 0.0}
    sim = Sim(case)
    sim.step(2, dt=1e-4)
    with pytest.raises(L.SphError) as e:
        sim.sync()
    assert e.value.code == L.SPH_EDOMAIN
    with pytest.raises(L.SphError) as e:
        sim.step(1)
    assert e.value.code == L.SPH_ESTATE
