"""Writes tests/golden/trajectory_spread.txt: how far two correct FP64
implementations of the Newmark IMEX scheme drift apart along a trajectory.

Every run is the oracle (oracle/newmark.py) from rest with the Ricker load.
The reference run factorises S with SciPy's sparse LU and sums the products
with K in CSR column order.  Four variants change only the rounding:
  chol          dense Cholesky of each connected component of S (and M^cc);
  perm          every row of K summed in a seeded random column order;
  sumfact       K u cell by cell, uncut cells by sum factorisation of the 1D
                matrices (the form the device computes the uncut part in);
  chol_sumfact  dense Cholesky and the cell-by-cell K u.
For each variant and field the file holds the relative L2 difference from
the reference: u (all active dofs), u^d_{n-1}, v^c and a^c.  The GPU parity
tests take their trajectory tolerances as a fixed multiple of the largest
of these spreads (tests/tolerances.py).

Run from the repository root:  python tests/golden/make_trajectory_spread.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fcm, newmark  # noqa: E402
from paper_2310_14712_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trajectory_spread.txt")
FIELDS = ("u", "ud_prev", "vc", "ac")
VARIANTS = {
    "chol": {"solver": "dense_cholesky"},
    "perm": {"perm_seed": 7},
    "sumfact": {"sumfact": True},
    "chol_sumfact": {"solver": "dense_cholesky", "sumfact": True},
}
CASES = (("config1", 200), ("config2", 600), ("config2", 5000))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def spreads(name, n_steps, variants=VARIANTS):
    """{variant: {field: spread}} for the named workload after n_steps."""
    w = getattr(inputs, name)()
    d = fcm.assemble(w)
    ft = inputs.ft_table(d.dt, n_steps, w.source_freq)
    z = np.zeros(d.n_grid)

    def run(solver="splu", perm_seed=None, sumfact=False):
        perm = None if perm_seed is None else np.random.default_rng(perm_seed).permutation(d.n_grid)
        ka = fcm.sumfact_stiffness(w, d) if sumfact else None
        ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, d.dt, solver=solver, sum_perm=perm, k_apply=ka)
        return ig.run(ig.initial_state(z, z, ft[0]), ft, n_steps)

    ref = run()
    out = {}
    for v, kw in variants.items():
        st = run(**kw)
        out[v] = {f: rel(getattr(st, f), getattr(ref, f)) for f in FIELDS}
    return out


def main():
    lines = ["# Spread of FP64 Newmark IMEX trajectories between correct implementations",
             "# (written by tests/golden/make_trajectory_spread.py; oracle only)",
             "# workload steps variant " + " ".join(FIELDS)]
    for name, n in CASES:
        res = spreads(name, n)
        for v in VARIANTS:
            lines.append(f"{name} {n} {v} " + " ".join(f"{res[v][f]:.3e}" for f in FIELDS))
            print(lines[-1], flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
