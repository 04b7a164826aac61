"""The single-precision form (SPH_FP32, the paper's GPU design of Sec. 3:
single precision in the particle interactions) against the oracle.

Storage is the mixed path's; the pair terms are formed from the absolute FP32
positions and FP32 potentials and summed in FP32 per list fill.  The oracle
(FP64) evaluates the state the GPU stores.  Bar: a relative position error
of up to 2^-24 |x| in each of x_i, x_j gives r a relative error up to
eps_r = 2^-23 X / s_min (X the largest coordinate, s_min the closest pair,
about half a spacing after jitter), the FP32 potentials add 2^-23 |phi|max /
(|G| s_min) to phi_j - phi_i relative to G.r; the accelerations take both
through L^-T (condition up to 1 / lambda_tic where the corrected form is
used), so |a - a_ref| <= 4 (eps_r + eps_phi) |G| / lambda_tic, 0.5-2e-4 of
|G| at these sizes; the same bar holds for D(phi)/Dt on its scale.  Ten
steps track the FP64 path to the mixed path's bars.
Neighbour sets come from the same FP32 test as the mixed path's.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from test_gpu_mixed import _own_state_case, _with_mass
from test_gpu_parity import _flags_all

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


CASES = [
    ("tank2d-dyn", wl.random_potential(wl.random_velocity(wl.jitter(wl.tank2d(dx=0.01, **_flags_all()), 0.1, 3),
                                                          0.05, 4), 0.05, 5)),
    ("box3d-dyn", wl.random_velocity(wl.jitter(wl.box3d(0.02, (0.4, 0.3, 0.4), (0.4, 0.3, 0.2), **_flags_all()),
                                               0.1, 6), 0.05, 7)),
    ("tank2d-hydro", wl.tank2d(dx=0.01)),
]


def _bar(case):
    pd = case["params"]
    f = case["kind"] == 0
    x = case["x"]
    X = np.abs(x).max()
    d2 = ((x[f][:, None, :] - x[None, :, :]) ** 2).sum(-1)
    d2[d2 == 0] = np.inf
    smin = np.sqrt(d2.min())
    gmag = float(np.linalg.norm(pd["gravity"]))
    eps_r = 2.0 ** -23 * X / smin
    eps_phi = 2.0 ** -23 * np.abs(case["phi"]).max() / (gmag * smin)
    return 4.0 * (eps_r + eps_phi) / pd["lambda_tic"]


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_fp32_rates_vs_oracle(Sim, name, case):
    case = _with_mass(case)
    sim = Sim(wl.with_params(case, precision="fp32"))
    sim.eval_rates()
    ref = oracle.eval_rates(_own_state_case(sim, case))
    f = case["kind"] == 0
    gmag = 9.81
    bar = _bar(case)
    acc = sim.field("dudt")
    s_acc = max(gmag, np.abs(ref["acc"][f]).max())
    err_acc = np.abs(acc[f] - ref["acc"][f]).max() / s_acc
    dphi = sim.field("dphidt")
    s_dphi = max(np.abs(ref["dphi"][f]).max(), case["params"]["c0"] * gmag * case["params"]["h"])
    err_dphi = np.abs(dphi[f] - ref["dphi"][f]).max() / s_dphi
    bad_nnb = int((sim.field("nnb")[f] != ref["nnb"][f]).sum())
    print(f"{name}: bar {bar:.2e} acc {err_acc:.2e} dphi {err_dphi:.2e} nnb mismatches {bad_nnb}")
    assert err_acc <= bar
    assert err_dphi <= bar
    assert bad_nnb <= max(1, 1e-4 * f.sum())


def test_fp32_hydrostatic_tank_is_not_well_balanced(Sim):
    """The 2D tank at rest: the FP64 and mixed forms balance gravity to
    round-off of their sums; the single-precision form leaves an imbalance of
    the size its position rounding predicts (it is the form the mixed
    storage is designed to avoid)."""
    case = wl.tank2d()
    f = case["kind"] == 0
    out = {}
    for prec in ("fp64", "mixed", "fp32"):
        sim = Sim(wl.with_params(case, precision=prec))
        sim.eval_rates()
        out[prec] = np.abs(sim.field("dudt")[f]).max()
    print({k: f"{v:.2e}" for k, v in out.items()})
    assert out["fp64"] <= 1e-13 * 9.81
    assert out["mixed"] <= 1e-5 * 9.81
    assert out["fp32"] <= _bar(case) * 9.81
    assert out["fp32"] > 10.0 * out["mixed"]


def test_fp32_trajectory_tracks_fp64(Sim):
    case = CASES[0][1]
    f = case["kind"] == 0
    s32 = Sim(wl.with_params(case, precision="fp32"))
    sd = Sim(case)
    s32.step(10)
    sd.step(10)
    dx = np.abs(s32.field("x")[f] - sd.field("x")[f]).max()
    du = np.abs(s32.field("u")[f] - sd.field("u")[f]).max() / np.abs(sd.field("u")[f]).max()
    dp = np.abs(s32.field("phi")[f] - sd.field("phi")[f]).max() / np.abs(sd.field("phi")[f]).max()
    print(f"10 steps: |dx| {dx:.2e} m, rel |dU| {du:.2e}, rel |dphi| {dp:.2e}")
    assert dx <= 1e-7
    assert du <= 1e-4
    assert dp <= 1e-4
    # dt follows max |U| (rel. difference below 1e-4 of U_max / C0 per step)
    assert abs(s32.stats()["t"] - sd.stats()["t"]) <= 1e-9


def test_fp32_kept_lists_match_rebuilding_path(Sim):
    """The single-precision form with the second stages from kept lists: the
    neighbour sets of a rebuild (counts and pair totals exact), fields equal
    up to the grouping of the FP32 chunk sums."""
    from test_gpu_keep import CASES_X
    name, case = CASES_X[1]
    case = wl.with_params(case, precision="fp32")
    a = Sim(case)
    b = Sim(wl.with_params(case, keep_lists=False, keep_across_steps=False))
    a.step(10)
    b.step(10)
    st = a.stats()
    assert st["n_kept"] + st["n_rebuilt"] == 20 and st["n_kept"] >= 10
    f = case["kind"] == 0
    assert np.array_equal(a.field("nnb")[f], b.field("nnb")[f])
    assert st["pairs"] == b.stats()["pairs"]
    L = max(case["params"]["domain_hi"]) - min(case["params"]["domain_lo"])
    assert np.abs(a.field("x")[f] - b.field("x")[f]).max() <= 1e-9 * L
    for name_ in ("u", "phi", "dudt", "dphidt"):
        va, vb = a.field(name_)[f], b.field(name_)[f]
        assert np.abs(va - vb).max() <= 1e-5 * max(np.abs(vb).max(), 1e-30), name_
