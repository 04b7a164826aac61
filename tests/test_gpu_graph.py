"""SPH_F_GRAPH: pairs of steps replayed from one captured HIP graph give the
eager path's results bit for bit.  The graph is replayed many times with the
program's own eager work and synchronisations between the replays (field
reads, right-hand sides outside sph_step, odd step counts run eagerly, a
changed dt and classifier margin that force a new capture), and every replay
is checked against a context stepping eagerly."""
import numpy as np
import pytest

import workloads as wl
from test_gpu_parity import _flags_all

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

FIELDS = ("x", "u", "phi", "dudt", "dphidt", "delta_u", "nnb", "fs", "tic", "mirror_src")


@pytest.fixture(scope="module")
def Sim():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_22269_amd import Simulation
    return Simulation


def _same(a, b, names=FIELDS):
    for n in names:
        assert np.array_equal(a.field(n), b.field(n)), n
    sa, sb = a.stats(), b.stats()
    for k in ("t", "dt", "steps", "umax", "pairs", "n_fs"):
        assert sa[k] == sb[k], k


def _cases():
    t2 = wl.random_velocity(wl.jitter(wl.tank2d(dx=0.02, **_flags_all()), 0.1, 3), 0.05, 4)
    d3 = wl.random_velocity(wl.dambreak3d(dx=0.04), 0.05, 5)
    cyl = wl.cylinder_entry(2, dx=0.005, tank=(0.3,), depth=0.15, wall_height=0.2, ceiling=0.25)
    return [("tank2d", t2), ("dambreak3d-coarse", d3), ("tank2d-mixed", wl.with_params(t2, precision="mixed")),
            ("tank2d-fp32", wl.with_params(t2, precision="fp32")),
            ("dambreak3d-coarse-mixed", wl.with_params(d3, precision="mixed")),
            ("cylinder-entry-2d", cyl), ("cylinder-entry-2d-mixed", wl.with_params(cyl, precision="mixed")),
            ("entry2d-prescribed", wl.entry2d(dx=0.02, **_flags_all()))]


CASES = _cases()


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_graph_replays_equal_eager_steps(Sim, name, case):
    a = Sim(case)
    b = Sim(wl.with_params(case, graph=True))
    for n in (2, 4, 6):  # capture, then replays
        a.step(n)
        b.step(n)
        _same(a, b)
    a.step(3)  # one replay and an eager step
    b.step(3)
    _same(a, b)
    a.eval_rates()  # a right-hand side outside sph_step: the next step recaptures
    b.eval_rates()
    _same(a, b)
    a.step(4)
    b.step(4)
    _same(a, b)
    dt = 0.5 * a.stats()["dt"]  # a fixed step: a new capture
    a.step(4, dt=dt)
    b.step(4, dt=dt)
    _same(a, b)
    a.step(2)
    b.step(2)
    _same(a, b)
    if case.get("body") is not None:
        sa, sb = a.body_state(), b.body_state()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k


def test_graph_with_the_learned_detector(Sim):
    """Learned detection: a new classifier margin changes the launches and is
    followed by a new capture."""
    from bench import load_classifier
    clf = load_classifier()
    case = wl.with_params(wl.dambreak3d(dx=0.04), precision="mixed", fs_mode="learned")
    a = Sim(case)
    b = Sim(wl.with_params(case, graph=True))
    for s in (a, b):
        s.set_classifier(clf["params"], clf["mean"], clf["std"], float(clf["margin"]))
    for n in (2, 2, 4):
        a.step(n)
        b.step(n)
        _same(a, b)
    for s in (a, b):
        s.set_classifier(clf["params"], clf["mean"], clf["std"], float("inf"))
    a.step(4)
    b.step(4)
    _same(a, b)
