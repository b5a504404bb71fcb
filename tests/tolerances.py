"""Trajectory tolerances of the FP64 GPU parity tests, derived from the
measured spread between correct FP64 implementations.

tests/golden/trajectory_spread.txt (written by make_trajectory_spread.py from
the oracle alone) holds, per workload and horizon, how far the oracle's
trajectory moves when only the rounding changes: dense Cholesky of S in
place of sparse LU, and/or every row of K summed in another order.  The
implicit block is ill-conditioned (alpha_f = 1e-5, cond(S) ~ 3e6 on the
16 x 16 plate), so such differences grow along a trajectory, mostly in the
c dofs.  A GPU trajectory is one more correct implementation with its own
rounding (fused multiply-adds, sum-factorised stiffness, dense inverses), so
it is held to SPREAD_FACTOR times the largest spread of each field.
"""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trajectory_spread.txt")
FIELDS = ("u", "ud_prev", "vc", "ac")
SPREAD_FACTOR = 20.0


def read_spreads(path=GOLDEN):
    """{(workload, steps): {variant: {field: spread}}}"""
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, steps, variant, *vals = line.split()
            out.setdefault((name, int(steps)), {})[variant] = dict(zip(FIELDS, map(float, vals)))
    return out


def max_spread(cases):
    """Largest spread of every field over the given (workload, steps) cases
    and all variants."""
    sp = read_spreads()
    return {f: max(v[f] for c in cases for v in sp[c].values()) for f in FIELDS}


def trajectory_tolerances(cases=(("config1", 200), ("config2", 600))):
    """Per-field bounds: SPREAD_FACTOR x the largest measured spread."""
    m = max_spread(cases)
    return {"u": SPREAD_FACTOR * m["u"], "u_prev_d": SPREAD_FACTOR * m["ud_prev"],
            "v_c": SPREAD_FACTOR * m["vc"], "a_c": SPREAD_FACTOR * m["ac"]}
