"""The spread between correct FP64 implementations of the Newmark IMEX
scheme, from which the GPU trajectory tolerances are derived
(tests/tolerances.py).  Re-measured here with the oracle on the 16x16 plate
(200 steps) and the 128x128 plate (600 steps); the stored figures were
written by tests/golden/make_trajectory_spread.py."""
import os
import sys

import numpy as np
import pytest

import tolerances

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_trajectory_spread as mts  # noqa: E402


@pytest.mark.parametrize("name,steps", [("config1", 200), ("config2", 600)])
def test_spread_reproduced(name, steps):
    """Dense Cholesky against sparse LU, and K u cell by cell: the measured
    spreads match the stored ones (same rounding, same figures up to the
    platform's LAPACK), are far above machine precision in the c fields and
    tiny in u^d, as the ill-conditioned cut block makes them."""
    stored = tolerances.read_spreads()[(name, steps)]
    variants = {"chol": mts.VARIANTS["chol"], "sumfact": mts.VARIANTS["sumfact"]}
    got = mts.spreads(name, steps, variants)
    for v in variants:
        for f in tolerances.FIELDS:
            a, b = got[v][f], stored[v][f]
            assert 0.5 * b <= a <= 2.0 * b, (name, v, f, a, b)
    for v in variants:
        assert got[v]["ac"] > 1e-12 and got[v]["ud_prev"] < 1e-12


def test_tolerances_are_a_multiple_of_the_spread():
    tol = tolerances.trajectory_tolerances()
    m = tolerances.max_spread((("config1", 200), ("config2", 600)))
    assert tol["u"] == tolerances.SPREAD_FACTOR * m["u"]
    assert tol["u_prev_d"] == tolerances.SPREAD_FACTOR * m["ud_prev"]
    assert tol["v_c"] == tolerances.SPREAD_FACTOR * m["vc"]
    assert tol["a_c"] == tolerances.SPREAD_FACTOR * m["ac"]
    # the 5000-step horizon of the 128x128 plate has its own, larger spread
    t5 = tolerances.trajectory_tolerances((("config2", 5000),))
    assert t5["a_c"] >= tol["a_c"] / 10
    assert np.all(np.isfinite(list(t5.values())))
