"""The oracle's cut-cell quadrature against every eigenfrequency the paper
prints for a single cell cut by a horizontal line (Section "Critical time
step analysis of cut cells"), and its critical steps against the printed
ones.  These pin the basis, both quadrature rules, the alpha scaling and the
space-tree reading at once."""
import numpy as np
import pytest

from conftest import read_golden
from oracle import fcm

ROWS = [(int(p), float(eta), float(om)) for p, eta, om in read_golden("cut_cell_omega.txt")]
EXACT = [r for r in ROWS if r[1] in (0.0, 0.5, 1.0)]
SAMPLED = [r for r in ROWS if r[1] not in (0.0, 0.5, 1.0)][::4]


def omega(p, eta, depth=13):
    if eta == 1.0:
        Me, Ke = fcm.uncut_element_matrices(p, [1.0, 1.0], 1.0, 1.0)
    else:
        Me, Ke = fcm.cut_element_matrices(fcm.HalfSpace(1, eta), p, [0.0, 0.0], [1.0, 1.0],
                                          depth, 1.0, 1.0, 1e-6)
    return fcm.omega_max(Ke, Me)


@pytest.mark.parametrize("p,eta,om", EXACT)
def test_exactly_integrable_cuts(p, eta, om):
    """eta = 1 (uncut), 0 (all fictitious), 0.5 (cut on the first bisection):
    the tree integrates these exactly, so the printed value is reproduced to
    the printed digits."""
    assert abs(omega(p, eta) - om) / om < 1e-11


@pytest.mark.parametrize("p,eta,om", SAMPLED)
def test_tree_integrated_cuts(p, eta, om):
    """Generic cut positions integrated by the depth-13 quadtree."""
    assert abs(omega(p, eta) - om) / om < 2e-9


def test_uncut_p1_uses_exact_stiffness():
    """With the Gauss-Legendre stiffness the uncut p=1 cell has omega = 2; a
    GLL-collocated stiffness would give 2 sqrt(2)."""
    assert abs(omega(1, 1.0) - 2.0) < 1e-13


def test_wrong_tree_depth_is_detected():
    """A shallower tree moves generic values well outside the tolerance."""
    p, eta, om = 2, 0.3, [r[2] for r in ROWS if r[0] == 2 and r[1] == 0.3][0]
    assert abs(omega(p, eta, depth=4) - om) / om > 1e-6


CRIT = {r[0]: (float(r[1]), int(r[2])) for r in read_golden("critical_steps.txt")}


def test_plate_uncut_cellwise_step():
    """p = 5, h = 0.25 m, c = 1: 18.13 ms."""
    Me, Ke = fcm.uncut_element_matrices(5, [0.25, 0.25], 1.0, 1.0)
    dt = 2.0 / fcm.omega_max(Ke, Me)
    val, digits = CRIT["plate_uncut_cellwise"]
    assert float(f"{dt:.{digits}g}") == val


def test_pillar_cellwise_bound():
    """3D p = 4, h = 0.0625 m, c = 3000 m/s: the uncut cell-wise step is a
    lower bound of the printed global IMEX critical step (element eigenvalue
    inequality) and within 1% of it."""
    Me, Ke = fcm.uncut_element_matrices(4, [0.0625] * 3, 1.0, 3000.0 ** 2)
    dt = 2.0 / fcm.omega_max(Ke, Me)
    val, _ = CRIT["pillar_imex_global"]
    assert dt <= val and dt > 0.99 * val
