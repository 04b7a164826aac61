"""Pins of the oracle's moving body (kind-2 dummies with a prescribed
velocity history, the aircraft-ditching case of Sec. 4).

* the displacement and velocity against the paper's printed history
  (tests/golden/ditching_velocity.txt) integrated by adaptive quadrature;
* the mirrored velocity of the body's dummies: the wall's normal velocity
  and the source fluid particle's tangential velocity (the slip condition of
  Sec. 2.4 taken relative to the moving wall);
* neighbour counts against brute force with the body placed from the
  quadrature's displacement;
* Galilean invariance: a body moving with U_w in fluid moving with U equals
  a fixed body at the same place in fluid moving with U - U_w (rates that
  depend on velocity differences only).
"""
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ditching_velocity.txt")


def _paper_history():
    """U(T) of the golden file, built from its printed forms only."""
    pieces = []
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if not line:
            continue
        lo, hi, form = float(line[0]), float(line[1]), line[2]
        par = [float(v) for v in line[3:]]
        pieces.append((lo, hi, form, par))

    def U(T):
        for k, (lo, hi, form, par) in enumerate(pieces):
            inside = (lo <= T <= hi) if k == 0 else (lo < T <= hi)
            if inside:
                return par[0] if form == "const" else par[0] * (T - par[1])
        return 0.0

    return pieces, U


def test_ditching_motion_matches_the_printed_history():
    pieces, U = _paper_history()
    pd = dict(wl.base_params(3, 0.03), **wl.ditching_motion())
    breaks = sorted({p[0] for p in pieces} | {p[1] for p in pieces})
    for T in [0.0, 0.3, 0.8, 0.8 + 1e-9, 1.2, 2.0, 2.8, 3.0, 4.0]:
        D, Ur = oracle.body_motion(pd, T)
        assert Ur[0] == pytest.approx(U(T), abs=1e-13), T
        assert Ur[1] == 0.0 and Ur[2] == 0.0
        pts = [b for b in breaks if 0.0 < b < T]
        ref, _ = integrate.quad(U, 0.0, T, points=pts or None, epsabs=1e-14, epsrel=1e-14) if T > 0 else (0.0, 0)
        assert D[0] == pytest.approx(ref, abs=1e-12), T
        assert D[1] == 0.0 and D[2] == 0.0
    # the body glides to x = -4 - 6 = -10 m and stays
    assert oracle.body_motion(pd, 10.0)[0][0] == pytest.approx(-10.0, abs=1e-13)
    # before the history starts it rests at its reference position
    D, Ur = oracle.body_motion(pd, -1.0)
    assert not D.any() and not Ur.any()


def _entry(seed=0, t=0.0):
    case = wl.entry2d(delta_sph=True, pst=True, tic=True, fs_project=True, cont_uncorr=True, fs_mode="exact")
    case = wl.random_velocity(wl.jitter(case, 0.1, seed), 0.2, seed + 1)
    case["t"] = t
    return case


def _quad_disp(pd, t):
    """Displacement of the body from the pieces a + b s by quadrature."""
    D = np.zeros(3)
    T = pd["body_t"]
    for k in range(len(T) - 1):
        for c in range(3):
            a, b = pd["body_a"][k][c], pd["body_b"][k][c]
            if t > T[k]:
                D[c] += integrate.quad(lambda s: a + b * s, T[k], min(t, T[k + 1]), epsabs=1e-15)[0]
    return D


def test_body_mirror_keeps_wall_normal_velocity():
    case = _entry(3, t=0.004)
    pd = case["params"]
    dim = pd["dim"]
    r = oracle.eval_rates(case)
    _, Uw = oracle.body_motion(pd, case["t"])
    Uw = Uw[:dim]
    assert np.abs(Uw).max() > 0.4
    for kind, wall in ((2, Uw), (1, np.zeros(dim))):
        rows = np.nonzero((case["kind"] == kind) & (r["mir_src"] >= 0))[0]
        assert len(rows) > 10
        n = case["normal"][rows]
        ud = r["mir_u"][rows]
        uf = case["u"][r["mir_src"][rows]]
        # normal part: the wall's; tangential part: the source fluid's
        assert np.abs((ud * n).sum(1) - n @ wall).max() <= 1e-14
        tang = lambda v: v - (v * n).sum(1)[:, None] * n
        assert np.abs(tang(ud) - tang(uf)).max() <= 1e-14


def test_body_neighbours_brute_force():
    case = _entry(5, t=0.02)
    pd = case["params"]
    dim = pd["dim"]
    x = case["x"].copy()
    b = case["kind"] == 2
    x[b] += _quad_disp(pd, case["t"])[:dim]
    two_h = 2.0 * pd["h"]
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    cnt = (d2 <= two_h ** 2).sum(1)
    r = oracle.eval_rates(case)
    f = case["kind"] == 0
    assert np.array_equal(r["nnb"][f], cnt[f])
    # the test sees the motion: counts differ from those of the body at rest
    r0 = oracle.eval_rates(dict(case, t=0.0))
    assert (r0["nnb"][f] != cnt[f]).sum() > 10


def test_moving_body_galilean_invariance():
    """Fluid velocities u with every wall (the body and the tank) moving at
    U_w, against u - U_w with the walls fixed (kind 1) at their displaced
    positions: velocity differences, mirrored potentials and positions are
    the same, so are accelerations, potential rates, eigenvalues, flags and
    neighbour counts.  Shifting is off (its scale U_max is not Galilean
    invariant)."""
    case = wl.with_params(_entry(7, t=0.012), pst=False, domain_lo=[-0.1, -0.1, 0.0])
    case["kind"] = np.where(case["kind"] != 0, 2, 0).astype(np.uint8)
    pd = case["params"]
    dim = pd["dim"]
    _, Uw = oracle.body_motion(pd, case["t"])
    Uw = Uw[:dim].copy()
    assert np.abs(Uw).max() > 0.4
    b = case["kind"] == 2
    fixed = dict(case)
    fixed["x"] = case["x"].copy()
    fixed["x"][b] += _quad_disp(pd, case["t"])[:dim]
    fixed["kind"] = np.where(b, 1, case["kind"]).astype(np.uint8)
    fixed["u"] = case["u"] - Uw
    fixed["params"] = {k: v for k, v in pd.items() if not k.startswith("body_")}
    fixed["mass"] = oracle.mass_from_phi(pd, case["phi"])
    moving = dict(case, mass=fixed["mass"])
    rm = oracle.eval_rates(moving)
    rf = oracle.eval_rates(fixed)
    f = case["kind"] == 0
    assert np.array_equal(rm["nnb"][f], rf["nnb"][f])
    assert np.array_equal(rm["mir_src"], rf["mir_src"])
    sa = max(9.81, np.abs(rf["acc"][f]).max())
    assert np.abs(rm["acc"][f] - rf["acc"][f]).max() <= 1e-12 * sa
    sp = max(np.abs(rf["dphi"][f]).max(), 1.0)
    assert np.abs(rm["dphi"][f] - rf["dphi"][f]).max() <= 1e-12 * sp
    assert np.abs(rm["lam"][f] - rf["lam"][f]).max() <= 1e-12
    assert np.array_equal(rm["fs"][f], rf["fs"][f])
    act = (case["kind"] != 0) & (rm["mir_src"] >= 0)
    assert np.abs(rm["mir_u"][act] - Uw - rf["mir_u"][act]).max() <= 1e-13
    # and the motion matters: without the wall velocity the rates differ
    still = dict(fixed, u=case["u"])
    rs = oracle.eval_rates(still)
    assert np.abs(rs["acc"][f] - rm["acc"][f]).max() > 1e-3 * sa


def test_body_steps_keep_reference_rows():
    """Steps leave the body's rows at their reference positions (the body is
    placed from its history at every right-hand side); fixed walls stay."""
    case = _entry(9)
    out = oracle.step(case, 3)
    d = case["kind"] != 0
    assert np.array_equal(out["x"][d], case["x"][d])
    assert out["t"] > 0.0
