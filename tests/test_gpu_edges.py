"""Edge cases of the FP64 path on the GPU: an empty context, walls without
water, water without walls, particle counts around the wave and block sizes
(a ragged last wave, a single particle) against the oracle at the parity bar,
and coincident particles reported as SPH_ENONFINITE."""
import numpy as np
import pytest

import oracle
import workloads as wl
from test_gpu_parity import compare_rates

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


def _rows(case, keep):
    c = dict(case)
    for k in ("x", "u", "phi", "kind", "normal"):
        c[k] = case[k][keep]
    if case.get("mass") is not None:
        c["mass"] = case["mass"][keep]
    return c


def test_empty_context(Sim):
    """No particles at all: a context is created and steps; time advances by
    the rule's dt (no velocity, so dx / C0 times CFL and the gravity term)."""
    case = _rows(wl.tank2d(dx=0.02), np.zeros(0, bool))
    sim = Sim(case)
    sim.eval_rates()
    sim.step(3)
    st = sim.stats()
    assert st["n_fluid"] == 0 and st["n_dummy"] == 0 and st["steps"] == 3
    pd = case["params"]
    dt = pd["cfl"] * min(pd["dx"] / pd["c0"], pd["dx"] ** 2 / (2 * pd["nu"]), np.sqrt(2 * pd["dx"] / 9.81))
    assert abs(st["t"] - 3 * dt) <= 1e-15
    sim.close()


def test_walls_without_water(Sim):
    """Only wall dummies: every dummy is inactive (no fluid within 2h), keeps
    its given potential and a zero velocity, and stepping changes nothing."""
    case = wl.tank2d(dx=0.02)
    case = _rows(case, case["kind"] != 0)
    sim = Sim(case)
    sim.step(2)
    assert np.array_equal(sim.field("mirror_src"), np.full(len(case["kind"]), -1, np.int32))
    assert np.array_equal(sim.field("phi"), case["phi"])
    assert np.array_equal(sim.field("x"), case["x"])
    assert not sim.field("u").any()
    sim.close()


def _block(n, dx=0.02, seed=0):
    """The first n points of a k^3 lattice (k^3 >= n) of spacing dx, jittered
    by 0.1 dx, in the middle of a 1 m box without walls: water without walls
    whose particle count is not a multiple of anything."""
    k = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
    g = (np.stack(np.meshgrid(*[np.arange(k)] * 3, indexing="ij"), -1).reshape(-1, 3)[:n] + 0.5) * dx
    rng = np.random.default_rng(seed)
    x = 0.5 - 0.5 * k * dx + g + rng.normal(0.0, 0.1 * dx, g.shape)
    pd = wl.base_params(3, dx, domain_lo=[0.0] * 3, domain_hi=[1.0] * 3, depth=k * dx, delta_sph=True, pst=True,
                        tic=True, fs_project=True, cont_uncorr=True, fs_mode="exact")
    phi = 9.81 * (x[:, 2].max() - x[:, 2])
    return {"params": pd, "x": x, "u": rng.normal(0.0, 0.05, x.shape), "phi": phi,
            "kind": np.zeros(n, np.uint8), "normal": np.zeros((n, 3)), "mass": None, "t": 0.0,
            "meta": {"H": float(x[:, 2].max()), "name": "block"}}


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 257, 3001])
def test_water_without_walls_ragged_sizes(Sim, n):
    """A jittered block of water without walls, counts around the wave (64)
    and block (256) sizes: one right-hand side and two steps against the
    oracle."""
    case = _block(n, seed=n)
    sim = Sim(case)
    sim.eval_rates()
    ref = oracle.eval_rates(case)
    print(n, compare_rates(sim, case, ref))
    sim.step(2)
    out = oracle.step(case, 2)
    L = 1.0
    assert np.abs(sim.field("x") - out["x"]).max() <= 1e-12 * L
    umax = max(np.abs(out["u"]).max(), 1e-3)
    assert np.abs(sim.field("u") - out["u"]).max() <= 1e-12 * umax
    sim.close()


def _two_blocks_at_the_limit(axis, precision, seed):
    """A 3D domain with the largest cell count the library accepts along
    `axis` (2047, 2047, 1023 cells of 2h; 14 on the others) and two jittered
    3 x 3 x 3 water blocks, one in its first cells and one in its last."""
    dx = 0.01
    pd = wl.base_params(3, dx, delta_sph=True, pst=True, tic=True, fs_project=True, cont_uncorr=True,
                        fs_mode="exact", precision=precision)
    R = pd["cell_size"]
    ncell = [14, 14, 14]
    ncell[axis] = (2047, 2047, 1023)[axis]
    pd["domain_lo"] = [0.0, 0.0, 0.0]
    pd["domain_hi"] = [(nc - 0.5) * R for nc in ncell]
    g = (np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) * dx
    lo = np.full(3, 0.5 * R)
    hi = np.full(3, 0.5 * R)
    hi[axis] = pd["domain_hi"][axis] - 2.75 * dx  # the top layer 0.25 dx inside the last (half) cell
    rng = np.random.default_rng(seed)
    x = np.concatenate([lo + g, hi + g]) + rng.normal(0.0, 0.05 * dx, (54, 3))
    pd["depth"] = 3 * dx
    phi = 9.81 * (x[:, 2].max() - x[:, 2])
    return {"params": pd, "x": x, "u": rng.normal(0.0, 0.05, x.shape), "phi": phi, "kind": np.zeros(54, np.uint8),
            "normal": np.zeros((54, 3)), "mass": None, "t": 0.0, "meta": {"name": "limit"}}


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_water_in_the_last_cells_of_the_largest_grid(Sim, axis):
    """Cells at the largest index along each axis (the mixed path packs
    them in 11, 11 and 10 bits): FP64 against the oracle at the parity bars
    over one right-hand side and two steps; the mixed path's cells and
    neighbour counts exact."""
    case = _two_blocks_at_the_limit(axis, "fp64", 80 + axis)
    c3, _ = oracle.cells(case["params"], case["x"])
    assert c3[:, axis].max() == (2046, 2046, 1022)[axis]
    sim = Sim(case)
    sim.eval_rates()
    assert np.array_equal(sim.field("cell"), c3)
    ref = oracle.eval_rates(case)
    print(axis, compare_rates(sim, case, ref))
    sim.step(2)
    out = oracle.step(case, 2)
    L = max(case["params"]["domain_hi"])
    assert np.abs(sim.field("x") - out["x"]).max() <= 1e-12 * L
    assert np.abs(sim.field("u") - out["u"]).max() <= 1e-12 * np.abs(out["u"]).max()
    sim.close()
    mixed = _two_blocks_at_the_limit(axis, "mixed", 80 + axis)
    sm = Sim(mixed)
    sm.eval_rates()
    assert np.array_equal(sm.field("cell"), c3)
    assert np.array_equal(sm.field("nnb"), ref["nnb"])
    sm.close()


def test_coincident_particles_are_reported(Sim):
    """Two fluid particles at one position (r = 0 has no kernel gradient
    direction): the right-hand side flags it and the next synchronising call
    returns SPH_ENONFINITE."""
    from paper_2608_22269_amd import _lib as L
    case = wl.tank2d(dx=0.02)
    f = np.flatnonzero(case["kind"] == 0)
    k = f[len(f) // 2]
    dup = np.concatenate([np.arange(len(case["kind"])), [k]])
    case = _rows(case, dup)
    sim = Sim(case)
    sim.eval_rates()
    with pytest.raises(L.SphError) as e:
        sim.sync()
    assert e.value.code == L.SPH_ENONFINITE
