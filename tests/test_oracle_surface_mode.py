"""The free-surface mode of the literal scheme, pinned on the CPU from the
linearisation of the oracle's right-hand side about the hydrostatic state.

The state of a small 2D tank is y = (x, U, phi) of its fluid particles (the
dummies are fixed and mirrored at every evaluation, Sec. 2.4); the oracle's
right-hand side f(y) = (U + dU_shift, DU/Dt, Dphi/Dt) of Eq. (sph) is
differentiated by central differences about the hydrostatic state (an exact
discrete equilibrium, Sec. 2.5), and the spectrum of the Jacobian is taken
with LAPACK.  Two independent computations then have to agree:

* the largest real part of the spectrum (an eigenvalue on the real axis,
  of order C0/dx, whose eigenvector sits in the top particle layer) and
* the growth rate the SSP-RK2 time stepping of the same tank shows once
  round-off has excited the mode, |1 + z + z^2/2| per step with z = lambda dt.

A tank closed by a lid (no free surface) has no such eigenvalue: the mode
belongs to the free surface.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def small_tank(lid=False, **kw):
    """0.2 x 0.1 m of water, dx = 0.01 (200 fluid particles), walls to 0.12 m;
    with lid=True three dummy layers close the top at the still-water level."""
    case = wl.tank2d(dx=0.01, width=0.2, depth=0.1, wall_height=0.12, **kw)
    if lid:
        dx = 0.01
        nx = 20
        xs = (np.arange(-3, nx + 3) + 0.5) * dx
        top = [np.stack([xs, np.full_like(xs, 0.1 + (k + 0.5) * dx)], 1) for k in range(3)]
        xl = np.concatenate(top)
        # keep only lid points not already wall dummies
        old = case["x"][case["kind"] == 1]
        keep = np.array([np.min(np.abs(old - p).sum(1)) > 1e-9 for p in xl])
        xl = xl[keep]
        nl = len(xl)
        g = 9.81
        case = dict(case)
        case["x"] = np.concatenate([case["x"], xl])
        case["u"] = np.concatenate([case["u"], np.zeros((nl, 2))])
        case["phi"] = np.concatenate([case["phi"], g * (0.1 - xl[:, 1])])
        case["kind"] = np.concatenate([case["kind"], np.ones(nl, np.uint8)])
        nrm = np.zeros((nl, 2))
        nrm[:, 1] = -1.0
        case["normal"] = np.concatenate([case["normal"], nrm])
        case["params"] = dict(case["params"], domain_hi=[0.23, 0.2, 0.0])
    case["mass"] = oracle.mass_from_phi(case["params"], case["phi"])
    return case


def _rhs(case, f, y):
    dim = case["params"]["dim"]
    nf = int(f.sum())
    c = dict(case)
    x, u, phi = case["x"].copy(), case["u"].copy(), case["phi"].copy()
    x[f] = y[:nf * dim].reshape(nf, dim)
    u[f] = y[nf * dim:2 * nf * dim].reshape(nf, dim)
    phi[f] = y[2 * nf * dim:]
    c["x"], c["u"], c["phi"] = x, u, phi
    r = oracle.eval_rates(c)
    return np.concatenate([(u[f] + r["dushift"][f]).ravel(), r["acc"][f].ravel(), r["dphi"][f]])


def jacobian(case):
    f = case["kind"] == 0
    dim = case["params"]["dim"]
    nf = int(f.sum())
    y0 = np.concatenate([case["x"][f].ravel(), case["u"][f].ravel(), case["phi"][f]])
    eps = np.concatenate([np.full(nf * dim, 1e-6 * case["params"]["dx"]), np.full(nf * dim, 1e-6),
                          np.full(nf, 1e-6)])
    J = np.zeros((len(y0), len(y0)))
    nt = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        for k in range(len(y0)):
            yp, ym = y0.copy(), y0.copy()
            yp[k] += eps[k]
            ym[k] -= eps[k]
            J[:, k] = (_rhs(case, f, yp) - _rhs(case, f, ym)) / (2.0 * eps[k])
    finally:
        oracle.set_num_threads(nt)
    return J


def leading_mode(case):
    """(lambda, fraction of the eigenvector's potential and velocity held by
    the top particle layer) for the eigenvalue of largest real part."""
    J = jacobian(case)
    w, V = np.linalg.eig(J)
    k = int(np.argmax(w.real))
    f = case["kind"] == 0
    dim = case["params"]["dim"]
    nf = int(f.sum())
    yf = case["x"][f][:, dim - 1]
    top = yf > yf.max() - 0.5 * case["params"]["dx"]
    v = V[:, k]
    vu = np.abs(v[nf * dim:2 * nf * dim].reshape(nf, dim)) ** 2
    vp = np.abs(v[2 * nf * dim:]) ** 2 / case["params"]["c0"] ** 2  # energy-like weighting
    wgt = vu.sum(1) + vp
    return w[k], float(wgt[top].sum() / wgt.sum())


def stepping_growth(case, n0, n1):
    """Growth rate of max |U| between steps n0 and n1 of the oracle's SSP-RK2."""
    f = case["kind"] == 0
    a = oracle.step(case, n0)
    b = oracle.step(a, n1 - n0)
    ua, ub = np.abs(a["u"][f]).max(), np.abs(b["u"][f]).max()
    return math.log(ub / ua) / (b["t"] - a["t"]), a["dt"]


def rk2_rate(lam, dt):
    z = lam * dt
    return math.log(abs(1.0 + z + 0.5 * z * z)) / dt


@pytest.mark.slow
@pytest.mark.parametrize("label,kw", [
    ("literal", {}),
    ("paper constants", {"h_factor": 1.5, "c0": 30.0}),
], ids=["literal", "paper-constants"])
def test_surface_mode_eigenvalue_matches_time_stepping(orc, label, kw):
    case = small_tank(**kw)
    lam, top_frac = leading_mode(case)
    c0dx = case["params"]["c0"] / case["params"]["dx"]
    # a real, positive eigenvalue of order C0/dx, living in the top layer
    assert lam.real > 0.2 * c0dx, lam
    assert abs(lam.imag) <= 1e-6 * abs(lam.real), lam
    assert top_frac > 0.6, top_frac
    # the time stepping grows at the rate SSP-RK2 gives that eigenvalue
    rate, dt = stepping_growth(case, 150, 250)
    want = rk2_rate(lam.real, dt)
    assert abs(rate - want) <= 0.10 * want, (rate, want, lam.real / c0dx)


@pytest.mark.slow
def test_closed_tank_has_no_growing_mode(orc):
    """The same water under a lid of dummies (no free surface): no eigenvalue
    with a growing real part beyond the differences' noise."""
    case = small_tank(lid=True)
    lam, _ = leading_mode(case)
    c0dx = case["params"]["c0"] / case["params"]["dx"]
    assert lam.real <= 1e-4 * c0dx, lam
