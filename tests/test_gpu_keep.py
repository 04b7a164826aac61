"""Right-hand sides run from kept candidate lists (SPH_F_KEEP_LISTS): a
right-hand side that sorts searches to 2h + s, s the cells' room, and keeps
its candidates; the step's second stage (with SPH_F_KEEP_ACROSS_STEPS, any
later stage) tests only those, over the cells and order of the build, while
twice the bound on any particle's move since the build fits s.

The neighbour sets are those of a fresh search, so trajectories match the
oracle to the bars of the rebuilding path, and fields match the rebuilding
path to summation order.  Steps that move particles too far for the room, or
whose lists overflow, rebuild every stage, and then equal the rebuilding
path bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from test_gpu_parity import _flags_all

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


def _room(case, factor):
    """Cells a factor wider than 2h / reach: room for a skin of about
    (factor - 1) 2h."""
    h = case["params"]["h"]
    return wl.with_params(case, cell_size=factor * h, keep_lists=True)


def _cases():
    dyn2 = wl.random_potential(wl.random_velocity(wl.jitter(wl.tank2d(dx=0.01, **_flags_all()), 0.1, 3), 0.05, 4),
                               0.05, 5)
    dam = wl.dambreak3d(dx=0.04, tank=(0.8, 0.4, 0.4), column=(0.3, 0.4, 0.22))
    dam = wl.random_velocity(dam, 0.3, 11)
    slosh = wl.slosh3d(dx=0.02, tank=(0.4, 0.2, 0.3), depth=0.14)
    slosh = wl.random_velocity(wl.jitter(slosh, 0.1, 8), 0.02, 9)
    slosh["t"] = 0.37
    return [("tank2d-dyn R=2.1h", _room(dyn2, 2.1)), ("dambreak3d-mini R=1.05h", _room(dam, 1.05)),
            ("slosh3d-forced R=1.01h", _room(slosh, 1.01))]


CASES = _cases()
CASES_X = [(name + " across steps", wl.with_params(case, keep_across_steps=True)) for name, case in CASES]


def _traj_close(sim, case, ref):
    f = case["kind"] == 0
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    assert np.abs(sim.field("x")[f] - ref["x"][f]).max() <= 1e-12 * L
    umax = max(np.abs(ref["u"][f]).max(), 1e-3)
    assert np.abs(sim.field("u")[f] - ref["u"][f]).max() <= 1e-12 * umax
    pmax = np.abs(ref["phi"][f]).max()
    assert np.abs(sim.field("phi")[f] - ref["phi"][f]).max() <= 1e-12 * pmax


@pytest.mark.parametrize("name,case", CASES + CASES_X, ids=[c[0] for c in CASES + CASES_X])
def test_kept_lists_trajectory_parity(Sim, name, case):
    """10 steps against the oracle (which searches afresh at every stage):
    every second stage from the kept lists, and with the lists kept across
    steps most first stages too."""
    sim = Sim(case)
    sim.step(10)
    st = sim.stats()
    print(name, {k: st[k] for k in ("n_kept", "n_rebuilt", "tests", "pairs")})
    if case["params"].get("keep_across_steps"):
        assert st["n_kept"] + st["n_rebuilt"] == 20 and st["n_kept"] > 10
    else:
        assert st["n_kept"] == 10 and st["n_rebuilt"] == 10
    ref = oracle.step(case, 10)
    _traj_close(sim, case, ref)
    assert abs(st["t"] - ref["t"]) <= 1e-15


@pytest.mark.parametrize("name,case", CASES + CASES_X, ids=[c[0] for c in CASES + CASES_X])
def test_kept_lists_match_rebuilding_path(Sim, name, case):
    """The second stage's rates from the kept lists against a rebuild and a
    fresh search of the same state: neighbour counts and flags exact, fields
    to summation order."""
    a = Sim(case)
    b = Sim(wl.with_params(case, keep_lists=False, keep_across_steps=False))
    a.step(3)
    b.step(3)
    assert a.stats()["n_kept"] >= 3
    f = case["kind"] == 0
    assert np.array_equal(a.field("nnb")[f], b.field("nnb")[f])
    assert np.array_equal(a.field("fs")[f], b.field("fs")[f])
    assert np.array_equal(a.field("tic")[f], b.field("tic")[f])
    for name_, tol in (("x", 1e-13), ("u", 1e-12), ("phi", 1e-12), ("dudt", 1e-12), ("dphidt", 1e-12)):
        va, vb = a.field(name_)[f], b.field(name_)[f]
        scale = max(np.abs(vb).max(), 1e-30)
        assert np.abs(va - vb).max() <= tol * scale, name_
    assert a.stats()["pairs"] == b.stats()["pairs"]


def test_no_room_for_the_skin_rebuilds(Sim):
    """Steps too long for the cells' room: every stage rebuilds, bit for bit
    as without the flag."""
    base = CASES[1][1]
    case = wl.with_params(base, cell_size=1.0005 * base["params"]["h"], keep_across_steps=True)
    dt = 2e-4
    a = Sim(case)
    b = Sim(wl.with_params(case, keep_lists=False, keep_across_steps=False))
    a.step(3, dt)
    b.step(3, dt)
    st = a.stats()
    assert st["n_kept"] == 0 and st["n_rebuilt"] == 6
    for name_ in ("x", "u", "phi", "dudt", "nnb"):
        assert np.array_equal(a.field(name_), b.field(name_)), name_


def test_list_overflow_rebuilds(Sim):
    """h = 4.5 dx in 2D (about 250 neighbours): every build overflows the kept
    chunks, every stage rebuilds, bit for bit as without the flag, and the
    trajectory matches the oracle."""
    case = wl.tank2d(dx=0.02, width=0.6, depth=0.3, wall_height=0.4, layers=10, h_factor=4.5, **_flags_all())
    case = wl.random_velocity(wl.jitter(case, 0.1, 12), 0.05, 13)
    case = wl.with_params(_room(case, 2.1), keep_across_steps=True)
    a = Sim(case)
    b = Sim(wl.with_params(case, keep_lists=False, keep_across_steps=False))
    a.step(2)
    b.step(2)
    st = a.stats()
    assert st["n_kept"] == 0 and st["n_rebuilt"] == 4
    for name_ in ("x", "u", "phi", "dudt", "nnb"):
        assert np.array_equal(a.field(name_), b.field(name_)), name_
    _traj_close(a, case, oracle.step(case, 2))


@pytest.mark.parametrize("name,case", CASES[1:] + CASES_X[1:], ids=[c[0] for c in CASES[1:] + CASES_X[1:]])
def test_mixed_kept_lists_match_rebuilding_path(Sim, name, case):
    """Mixed path: the kept lists (skin padded for the FP32 positions and
    test) give the second stage the neighbour sets of a rebuild; fields differ
    only by the grouping of the FP32 chunk sums."""
    case = wl.with_params(case, precision="mixed")
    a = Sim(case)
    b = Sim(wl.with_params(case, keep_lists=False, keep_across_steps=False))
    a.step(10)
    b.step(10)
    st = a.stats()
    assert st["n_kept"] + st["n_rebuilt"] == 20 and st["n_kept"] >= 10
    f = case["kind"] == 0
    assert np.array_equal(a.field("nnb")[f], b.field("nnb")[f])
    assert a.stats()["pairs"] == b.stats()["pairs"]
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    assert np.abs(a.field("x")[f] - b.field("x")[f]).max() <= 1e-9 * L
    for name_ in ("u", "phi", "dudt", "dphidt"):
        va, vb = a.field(name_)[f], b.field(name_)[f]
        assert np.abs(va - vb).max() <= 1e-5 * max(np.abs(vb).max(), 1e-30), name_
