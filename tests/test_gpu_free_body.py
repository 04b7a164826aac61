"""The free rigid body (kind-2 dummies moving under G(t) and the water's force
and torque; the cylinder water entry of Sec. 4) on the GPU.

Against the oracle on the same seeded inputs: one right-hand side at a turned,
shifted, moving pose (fluid rates and the wall mirror at the bars of the
fixed-wall cases, neighbour counts and mirror sources exact, the dummies'
placed positions to rounding, force and torque), and trajectories of the
body's state and of the fluid over several steps, 2D and 3D.  Against closed
forms: free flight (c = c0 + v0 t + G t^2 / 2, v = v0 + G t: SSP-RK2 is exact
for them) and a torque-free spin of an isotropic body.  The force and torque
are sums over the body's dummies taken in another order than the oracle's
(sorted rows, a fixed block tree), so they agree to the rounding of those
sums: the bars are relative to the sum of the magnitudes of the terms.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from test_gpu_parity import _flags_all, compare_rates
from test_oracle_free_body import _far_fluid_case, _immersed, _qmat, _quat

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


def _posed(dim, seed=3):
    """The immersed box at a turned (0.37 rad) and shifted pose, moving and
    turning, with jittered, moving water and every stabiliser on."""
    c = wl.random_velocity(wl.jitter(_immersed(dim, **_flags_all()), 0.1, seed), 0.05, seed + 1)
    shift = np.array([0.013, -0.021, 0.008][:dim])
    v = [0.4, -0.7, 0.2][:dim] + [0.0] * (3 - dim)
    w = [0.0, 0.0, 1.3] if dim == 2 else [0.5, -0.9, 1.3]
    c["body"] = dict(c["body"], q=_quat(dim, 0.37), v=v, w=w,
                     c=list(np.asarray(c["body"]["c"][:dim]) + shift) + [0.0] * (3 - dim))
    return c


def _placed(case):
    """x = c + R (x_ref - c0) of the body's rows."""
    dim = case["params"]["dim"]
    b = case["kind"] == 2
    R = _qmat(case["body"]["q"])[:dim, :dim]
    c0 = np.asarray(case["params"]["body_c0"][:dim])
    cc = np.asarray(case["body"]["c"][:dim])
    return cc + (case["x"][b] - c0) @ R.T


def _term_scale(case, ref):
    """Sum over the body's active dummies of m_d |a_d| (the magnitude the
    force's rounding scales with), from the oracle's mirror and a plain
    pass over the dummies' neighbours."""
    dim = case["params"]["dim"]
    pd = case["params"]
    h = pd["h"]
    b = np.flatnonzero((case["kind"] == 2) & (ref["mir_src"] >= 0))
    f = case["kind"] == 0
    xb = _placed(case)
    idx = {k: j for j, k in enumerate(np.flatnonzero(case["kind"] == 2))}
    xf, phif = case["x"][f], case["phi"][f]
    mass = case["mass"] if case.get("mass") is not None else oracle.mass_from_phi(pd, case["phi"])
    V = mass[f] / (pd["rho0"] * np.exp(phif / pd["c0"] ** 2))
    alpha = 7.0 / (4.0 * math.pi * h * h) if dim == 2 else 21.0 / (16.0 * math.pi * h ** 3)
    tot = 0.0
    for d in b:
        r = xf - xb[idx[d]]
        s = np.sqrt((r * r).sum(1))
        near = s <= 2.0 * h
        t = 1.0 - 0.5 * s[near] / h
        K = 5.0 * alpha / (h * h) * t ** 3
        tot += mass[d] * (np.abs(phif[near] + ref["mir_phi"][d]) * K * s[near] * V[near]).sum()
    return tot


@pytest.mark.parametrize("dim", [2, 3])
def test_free_body_rates_parity(Sim, dim):
    case = _posed(dim)
    case["mass"] = oracle.mass_from_phi(case["params"], case["phi"])
    sim = Sim(case)
    sim.eval_rates()
    ref = oracle.eval_rates(case)
    print(dim, compare_rates(sim, case, ref))
    b = case["kind"] == 2
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    xb = sim.field("x")[b]
    assert np.abs(xb - _placed(case)).max() <= 4e-16 * L
    assert (ref["mir_src"][b] >= 0).sum() > 20
    st = sim.body_state()
    scale = _term_scale(case, ref)
    ef = np.abs(st["force"][:dim] - ref["body_force"][:dim]).max() / scale
    arm = np.abs(xb - np.asarray(case["body"]["c"][:dim])).max()
    et = np.abs(st["torque"] - ref["body_torque"]).max() / (scale * arm)
    print(f"force {st['force']} vs {ref['body_force']}: {ef:.2e}; torque {et:.2e} (term scale {scale:.3g})")
    assert ef <= 1e-14
    assert et <= 1e-14
    # the state itself is untouched by a right-hand side
    for k in ("c", "q", "v", "w"):
        assert np.array_equal(st[k], np.asarray(case["body"][k], dtype=float)), k


def _trajectory_errors(sim, case, ref):
    """Relative differences of the body's state and the fluid fields after
    a run (positions relative to the domain size, the rest to their
    maxima; the angular velocity to at least |v| / l, l the body's reach
    from its centre, the spin its speed would give: a symmetric entry has
    no spin but rounding)."""
    st = sim.body_state()
    rb = ref["body"]
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    dim = case["params"]["dim"]
    reach = np.linalg.norm(case["x"][case["kind"] == 2] - np.asarray(case["params"]["body_c0"][:dim]), axis=1).max()
    vmax = max(np.abs(rb["v"]).max(), 1e-3)
    errs = {
        "c": np.abs(st["c"] - rb["c"]).max() / L,
        "q": np.abs(st["q"] - rb["q"]).max(),
        "v": np.abs(st["v"] - rb["v"]).max() / vmax,
        "w": np.abs(st["w"] - rb["w"]).max() / max(np.abs(rb["w"]).max(), vmax / reach),
    }
    f = case["kind"] == 0
    errs["x"] = np.abs(sim.field("x")[f] - ref["x"][f]).max() / L
    errs["u"] = np.abs(sim.field("u")[f] - ref["u"][f]).max() / max(np.abs(ref["u"][f]).max(), 1e-3)
    errs["phi"] = np.abs(sim.field("phi")[f] - ref["phi"][f]).max() / np.abs(ref["phi"][f]).max()
    assert abs(sim.stats()["t"] - ref["t"]) <= 1e-15
    return st, errs


@pytest.mark.parametrize("dim,nsteps", [(2, 10), (3, 10), (2, 40)])
def test_free_body_trajectory_parity(Sim, dim, nsteps):
    """A body released at a turned pose with velocity and spin in moving
    water: the body's state and the fluid after nsteps SSP-RK2 steps."""
    case = _posed(dim, seed=13)
    case["mass"] = oracle.mass_from_phi(case["params"], case["phi"])
    sim = Sim(case)
    sim.step(nsteps)
    ref = oracle.step(case, nsteps)
    st, errs = _trajectory_errors(sim, case, ref)
    print(dim, nsteps, {k: f"{v:.2e}" for k, v in errs.items()})
    for k in ("c", "q", "v", "w", "x", "u", "phi"):
        assert errs[k] <= 1e-12, (k, errs[k])
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    # it moved and turned: far beyond the bars
    assert np.abs(st["c"] - np.asarray(case["body"]["c"])).max() > 1e-4
    assert np.abs(st["q"] - np.asarray(case["body"]["q"])).max() > 1e-4
    # the dummies sit at the pose of the final state
    moved = dict(case, body={k: list(v) for k, v in st.items() if k in ("c", "q", "v", "w")})
    sim.eval_rates()
    b = case["kind"] == 2
    assert np.abs(sim.field("x")[b] - _placed(moved)).max() <= 4e-16 * L


def _entry(dim):
    """Small cylinder water entries (V0 = -6.22 m/s, density 1370, C0 = 30):
    2D, a disc of D = 0.05 m into 0.3 x 0.15 m of water at dx = 0.0025 (7,200
    fluid); 3D, a cylinder of D = 0.05 m and L = 0.06 m into 0.2 x 0.1 x 0.1 m
    of water at dx = 0.005 (16,000 fluid)."""
    if dim == 2:
        return wl.cylinder_entry(2, dx=0.0025, tank=(0.3,), depth=0.15, wall_height=0.2, ceiling=0.25)
    return wl.cylinder_entry(3, dx=0.005, tank=(0.2, 0.1), depth=0.1, length=0.06, wall_height=0.15, ceiling=0.2)


@pytest.mark.parametrize("dim,nsteps", [(2, 40), (3, 8)])
def test_cylinder_entry_parity(Sim, dim, nsteps):
    """The impact of the water-entry case: the cylinder meets the surface
    and the water brakes it; its state and the fluid against the oracle."""
    case = _entry(dim)
    case["mass"] = oracle.mass_from_phi(case["params"], case["phi"])
    sim = Sim(case)
    sim.step(nsteps)
    ref = oracle.step(case, nsteps)
    st, errs = _trajectory_errors(sim, case, ref)
    print(dim, nsteps, st["v"], st["force"], {k: f"{v:.2e}" for k, v in errs.items()})
    for k in ("c", "q", "v", "w", "x", "u", "phi"):
        assert errs[k] <= 1e-12, (k, errs[k])
    # the water pushes up on the cylinder, beyond its weight
    m = case["params"]["body_mass"]
    assert st["force"][dim - 1] > m * 9.81


@pytest.mark.parametrize("dim", [2, 3])
def test_free_flight_on_the_gpu_is_exact(Sim, dim):
    """No water within 2h of the body: c and v follow the closed forms of a
    body under gravity alone (SSP-RK2 is exact for them), q stays put."""
    v0 = [0.3, 1.7, -0.4][:dim]
    case = _far_fluid_case(dim, v0, [0.0, 0.0, 0.0])
    sim = Sim(case)
    sim.step(50, dt=1e-3)
    st = sim.body_state()
    t = sim.stats()["t"]
    G = np.asarray(case["params"]["gravity"][:dim])
    c0 = np.asarray(case["body"]["c"][:dim])
    assert np.abs(st["c"][:dim] - (c0 + np.asarray(v0) * t + 0.5 * G * t * t)).max() <= 1e-13
    assert np.abs(st["v"][:dim] - (np.asarray(v0) + G * t)).max() <= 1e-13
    assert np.array_equal(st["q"], [1.0, 0.0, 0.0, 0.0])
    assert np.array_equal(st["force"], np.zeros(3)) and np.array_equal(st["torque"], np.zeros(3))


def test_torque_free_spin_on_the_gpu(Sim):
    """An isotropic body spinning without torque or gravity: omega constant,
    q(t) = (cos(|w| t / 2), sin(|w| t / 2) w / |w|) to the SSP-RK2 error,
    unit norm to rounding."""
    w0 = np.array([0.8, -1.1, 2.3])
    case = _far_fluid_case(3, [0.0, 0.0, 0.0], list(w0), inertia=[0.7, 0.7, 0.7, 0.0, 0.0, 0.0])
    case["params"]["gravity"] = [0.0, 0.0, 0.0]
    sim = Sim(case)
    sim.step(500, dt=2e-4)
    st = sim.body_state()
    t = sim.stats()["t"]
    assert np.abs(st["w"] - w0).max() <= 1e-13
    wn = np.linalg.norm(w0)
    want = np.concatenate([[math.cos(0.5 * wn * t)], math.sin(0.5 * wn * t) * w0 / wn])
    assert np.abs(st["q"] - want).max() <= 1e-7
    assert abs(np.linalg.norm(st["q"]) - 1.0) <= 1e-15


def test_body_state_needs_a_free_body(Sim):
    from paper_2608_22269_amd import _lib as L
    sim = Sim(wl.tank2d(dx=0.02))
    with pytest.raises(L.SphError) as e:
        sim.body_state()
    assert e.value.code == L.SPH_ESTATE
    sim.eval_rates()  # the context stays usable


def test_cylinder_entry_full_size_sampled(Sim):
    """The bench's cylinder entry at the paper's size (15.36M fluid + 2.37M
    dummies, R = h), the cylinder half submerged (centre at the still
    surface, the water inside it removed) and entering at 6.22 m/s, at its
    first right-hand side: the body's force and torque against the oracle's,
    summed over all 13,736 of its dummies, and 1,500 sampled fluid rows next
    to the cylinder plus 500 elsewhere, element by element at the parity
    bar."""
    from test_gpu_fullsize import _compare_rows
    from test_gpu_parity import TOL
    case = wl.cylinder_entry(3, dx=0.0025, gap=-0.025)
    case = wl.with_params(case, cell_size=case["params"]["h"])
    case["mass"] = oracle.mass_from_phi(case["params"], case["phi"])
    rng = np.random.default_rng(41)
    f = np.nonzero(case["kind"] == 0)[0]
    c = np.asarray(case["body"]["c"])
    xf = case["x"][f]
    h = case["params"]["h"]
    near = f[(np.abs(xf[:, 0] - c[0]) < 0.025 + 3 * h) & (np.abs(xf[:, 1] - c[1]) < 0.1 + 3 * h)
             & (xf[:, 2] > c[2] - 0.025 - 3 * h)]
    rows = np.unique(np.concatenate([rng.choice(near, 1500, replace=False), rng.choice(f, 500, replace=False)]))
    sim = Sim(case)
    sim.eval_rates()
    ref = oracle.eval_rates(case, rows=rows)
    nnb = _compare_rows(sim, case, ref, rows, TOL, TOL)
    assert np.array_equal(nnb, ref["nnb"][rows])
    st = sim.body_state()
    F, T = ref["body_force"], ref["body_torque"]
    print("force", st["force"], F, "torque", st["torque"], T)
    # the hydrostatic part: the buoyancy of the submerged half, to 2%
    assert abs(F[2] / (1000.0 * 9.81 * 0.5 * math.pi * 0.025 ** 2 * 0.2) - 1.0) <= 0.02, F
    # the lateral components and the torque cancel by symmetry
    assert np.abs(st["force"] - F).max() <= 1e-12 * abs(F[2])
    assert np.abs(st["torque"] - T).max() <= 1e-12 * abs(F[2]) * 0.1
    sim.close()


@pytest.mark.parametrize("dim,nsteps", [(2, 40), (3, 8)])
def test_mixed_free_body_tracks_fp64(Sim, dim, nsteps):
    """The mixed path (cell + FP32 offset storage, FP32 pair terms, FP64 sums;
    the body's force summed in FP64 from its records) against the FP64 path on
    the cylinder entry: the body's state and the fluid after nsteps steps,
    at the mixed path's bars (positions 1e-7 m, velocities and potentials
    1e-4 of their maxima); the body's velocity to 1e-6 of its speed and its
    force to 1e-5 (FP64 sums over records whose offsets carry the FP32
    rounding, about 1e-7 of a cell)."""
    case = _entry(dim)
    sm = Sim(wl.with_params(case, precision="mixed"))
    sd = Sim(case)
    sm.step(nsteps)
    sd.step(nsteps)
    bm, bd = sm.body_state(), sd.body_state()
    f = case["kind"] == 0
    speed = np.abs(bd["v"]).max()
    err = {"c": np.abs(bm["c"] - bd["c"]).max(), "v": np.abs(bm["v"] - bd["v"]).max() / speed,
           "F": np.abs(bm["force"] - bd["force"]).max() / np.abs(bd["force"]).max(),
           "x": np.abs(sm.field("x")[f] - sd.field("x")[f]).max(),
           "u": np.abs(sm.field("u")[f] - sd.field("u")[f]).max() / np.abs(sd.field("u")[f]).max(),
           "phi": np.abs(sm.field("phi")[f] - sd.field("phi")[f]).max() / np.abs(sd.field("phi")[f]).max()}
    print(dim, nsteps, {k: f"{v:.2e}" for k, v in err.items()})
    assert err["c"] <= 1e-7 and err["x"] <= 1e-7
    assert err["u"] <= 1e-4 and err["phi"] <= 1e-4
    assert err["v"] <= 1e-6 and err["F"] <= 1e-5
