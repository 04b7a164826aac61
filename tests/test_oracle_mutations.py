"""Planted mistakes in the oracle's C source: each variant is compiled on
the CPU and must fail at least one of the term pins of
test_oracle_terms.py.  This shows that those pins see the mistakes a reader
of Eq. (sph), Eq. (lfsover) and Sec. 2.3 could plausibly make (a flipped
sign, a dropped factor or term, a branch that ignores its switch), and not
only that the oracle agrees with itself."""
import pytest

import oracle
from tests import test_oracle_free_body as fb
from tests import test_oracle_terms as terms

# (name, text in the oracle source, its replacement); each text occurs once
MUTATIONS = [
    ("delta-SPH sign", "if (p->flags & ORC_DELTA) dphi += p->delta * h * c0 * Dsum;",
     "if (p->flags & ORC_DELTA) dphi -= p->delta * h * c0 * Dsum;"),
    ("delta-SPH factor 2 dropped", "Dsum += 2.0 * (phiv[j] - phii) * rg / (s * s) * Vj;",
     "Dsum += (phiv[j] - phii) * rg / (s * s) * Vj;"),
    ("delta-SPH over |r| instead of |r|^2", "Dsum += 2.0 * (phiv[j] - phii) * rg / (s * s) * Vj;",
     "Dsum += 2.0 * (phiv[j] - phii) * rg / s * Vj;"),
    ("shifting direction", "dstar[a] = -2.0 * h * umax * P[a];", "dstar[a] = 2.0 * h * umax * P[a];"),
    ("shifting weight dropped", "double pw = 1.0 + p->pst_R * pow(wr, p->pst_n);", "double pw = 1.0;"),
    ("shifting factor 2 dropped", "dstar[a] = -2.0 * h * umax * P[a];", "dstar[a] = -h * umax * P[a];"),
    ("conservative branch sign", "for (int a = 0; a < dim; ++a) grad[a] = SC[a];",
     "for (int a = 0; a < dim; ++a) grad[a] = -SC[a];"),
    ("conservative sum as a difference", "SC[a] += (phiv[j] + phii) * gw[a] * Vj;",
     "SC[a] += (phiv[j] - phii) * gw[a] * Vj;"),
    ("Lax-Friedrichs coefficient halved", "double twophi = (phiv[j] - phii) - c0 * dun;",
     "double twophi = (phiv[j] - phii) - 0.5 * c0 * dun;"),
    ("Lax-Friedrichs sign", "double twophi = (phiv[j] - phii) - c0 * dun;",
     "double twophi = (phiv[j] - phii) + c0 * dun;"),
    ("free-surface projection dropped", "for (int a = 0; a < dim; ++a) dus[a] -= dn * nr[a];",
     "(void)nr;"),
    ("uncorrected continuity ignored", "int uncorr = singular || (tic_on && (p->flags & ORC_CONT_UNCORR));",
     "int uncorr = singular;"),
]


# the free body's pins (as plain checks)
BODY_CHECKS = {
    "flight_2d": lambda: fb.test_free_flight_is_exact(oracle, 2),
    "flight_3d": lambda: fb.test_free_flight_is_exact(oracle, 3),
    "spin": lambda: fb.test_torque_free_spin(oracle),
    "precession": lambda: fb.test_torque_free_precession_keeps_angular_momentum(oracle),
    "pose_3d": lambda: fb.test_pose_equals_explicit_walls(oracle, 3),
    "slip_2d": lambda: fb.test_slip_relative_to_moving_wall(oracle, 2),
    "slip_3d": lambda: fb.test_slip_relative_to_moving_wall(oracle, 3),
    "archimedes_2d": lambda: fb.test_archimedes(oracle, 2),
    "archimedes_3d": lambda: fb.test_archimedes(oracle, 3),
    "archimedes_cylinder_2d": lambda: fb.test_archimedes_cylinder(oracle, 2),
    "covariance_3d": lambda: fb.test_force_and_torque_rotate_with_the_scene(oracle, 3),
    "reference_point_3d": lambda: fb.test_torque_reference_point(oracle, 3),
}

BODY_MUTATIONS = [
    ("body force sign", "ad[a] -= (phiv[i] + phiv[d]) * Kq * r[a] * V[i];",
     "ad[a] += (phiv[i] + phiv[d]) * Kq * r[a] * V[i];"),
    ("body force without the volume", "ad[a] -= (phiv[i] + phiv[d]) * Kq * r[a] * V[i];",
     "ad[a] -= (phiv[i] + phiv[d]) * Kq * r[a];"),
    ("torque arm reversed", "arm[a] = x[d * dim + a] - body->c[a];", "arm[a] = body->c[a] - x[d * dim + a];"),
    ("wall velocity w x r reversed", "cross3(b->w, d, wr);", "cross3(d, b->w, wr);"),
    ("gyroscopic term sign", "rhs[a] = T[a] - gyro[a];", "rhs[a] = T[a] + gyro[a];"),
    ("gravity left out of the body", "rate->v[a] = F[a] / p->body_mass + G[a];", "rate->v[a] = F[a] / p->body_mass;"),
    ("quaternion rate in the body frame", "rate->q[1] = 0.5 * (w[0] * q[0] + w[1] * q[3] - w[2] * q[2]);",
     "rate->q[1] = 0.5 * (w[0] * q[0] - w[1] * q[3] + w[2] * q[2]);"),
]


def test_unmutated_oracle_passes_every_term_pin(orc):
    for name, fn in terms.CHECKS.items():
        fn()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(orc, tmp_path, name, old, new):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site of '{name}' not unique"
    lib = oracle.build_variant(src.replace(old, new), str(tmp_path))
    failed = []
    with oracle.using_library(lib):
        for check, fn in terms.CHECKS.items():
            try:
                fn()
            except AssertionError:
                failed.append(check)
    assert failed, f"no pin fails with the planted mistake '{name}'"


def test_unmutated_oracle_passes_every_body_pin(orc):
    for name, fn in BODY_CHECKS.items():
        fn()


@pytest.mark.parametrize("name,old,new", BODY_MUTATIONS, ids=[m[0] for m in BODY_MUTATIONS])
def test_planted_body_mistake_fails_a_pin(orc, tmp_path, name, old, new):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site of '{name}' not unique"
    lib = oracle.build_variant(src.replace(old, new), str(tmp_path))
    failed = []
    with oracle.using_library(lib):
        for check, fn in BODY_CHECKS.items():
            try:
                fn()
            except AssertionError:
                failed.append(check)
    assert failed, f"no pin fails with the planted mistake '{name}'"
