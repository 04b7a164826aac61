"""Planted mistakes in the oracle's C source: each variant is compiled on
the CPU and must fail at least one of the term pins of
test_oracle_terms.py.  This shows that those pins see the mistakes a reader
of Eq. (sph), Eq. (lfsover) and Sec. 2.3 could plausibly make (a flipped
sign, a dropped factor or term, a branch that ignores its switch), and not
only that the oracle agrees with itself."""
import pytest

import oracle
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
