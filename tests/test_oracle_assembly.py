"""Pins of the oracle's classification, assembly and partition against
brute-force point sampling, exact integrals and algebraic invariants."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import basis, fcm
from paper_2310_14712_amd import inputs


@pytest.fixture(scope="module")
def c1():
    w = inputs.config1()
    return w, fcm.assemble(w)


def test_classification_matches_point_sampling(c1):
    """Every empty cell is fictitious at all of 41^2 sample points, every
    uncut cell physical at all of them, and every cut cell has both."""
    w, d = c1
    geom = fcm.geometry_of(w)
    s = np.linspace(0, 1, 41)[1:-1]
    S = np.array(np.meshgrid(s, s)).reshape(2, -1).T
    for cid, cidx in enumerate(fcm.all_cells(w.n_cells)):
        lo, h = fcm.cell_box(w, cidx)
        fic = geom.fictitious(lo + S * h)
        if d.flags[cid] == fcm.EMPTY:
            assert fic.all()
        elif d.flags[cid] == fcm.UNCUT:
            assert not fic.any()
        else:
            assert fic.any() and not fic.all()


def test_config1_counts(c1):
    _, d = c1
    assert (d.flags == fcm.CUT).sum() == 28
    assert (d.flags == fcm.EMPTY).sum() == 24
    assert len(d.active) == 3888 and len(d.Ic) == 560 and len(d.Id) == 3328


def test_mass_and_stiffness_invariants(c1):
    """K annihilates constants (rows sum to 0), K and M are symmetric, M is
    block diagonal over (d, c) with a diagonal d block, and the total mass is
    the integral of alpha rho over the non-empty cells (to the tree's
    accuracy)."""
    w, d = c1
    one = np.zeros(d.n_grid)
    one[d.active] = 1.0
    assert np.max(np.abs(d.K @ one)) < 1e-11
    assert abs(d.K - d.K.T).max() < 1e-13
    assert abs(d.M - d.M.T).max() < 1e-16
    Mdc = d.M[d.Id][:, d.Ic]
    assert Mdc.count_nonzero() == 0
    Mdd = d.M[d.Id][:, d.Id]
    assert (Mdd - sp.diags(Mdd.diagonal())).count_nonzero() == 0
    # total mass: non-empty cell area minus (1 - alpha_f) * hole area inside them
    ncell = (d.flags != fcm.EMPTY).sum()
    h2 = np.prod(w.h)
    empty_area = (d.flags == fcm.EMPTY).sum() * h2
    hole_area_nonempty = np.pi * 0.2 ** 2 - empty_area
    exact = ncell * h2 - (1 - w.alpha_f) * hole_area_nonempty
    assert abs(one @ d.M @ one - exact) / exact < 2e-3


def test_point_source_moments(c1):
    """f_x at a physical point: weights sum to 1 (partition of unity) and
    reproduce the source coordinates (linear reproduction)."""
    w, d = c1
    grid = d.grid
    nz = np.nonzero(d.fx)[0]
    assert abs(d.fx.sum() - 1.0) < 1e-13
    xl, _ = basis.gll(w.p)
    coords = np.concatenate([[e * w.h[0] + (xl[a] + 1) * w.h[0] / 2 for a in range(w.p)]
                             for e in range(w.n_cells[0])] + [[1.0]])
    ix = nz % grid[0]
    iy = nz // grid[0]
    assert abs(d.fx[nz] @ coords[ix] - w.source[0]) < 1e-13
    assert abs(d.fx[nz] @ coords[iy] - w.source[1]) < 1e-13


def test_uncut_element_is_exact_tensor_form():
    """The uncut element stiffness equals the Kronecker form
    kappa [(hy/hx) Kh x Mh + (hx/hy) Mh x Kh] with consistent 1D matrices
    (exact integration), in 2D and its 3D analogue."""
    p = 3
    xg, wg = basis.gauss_legendre(p + 1)
    Mh, Kh = fcm.quadrature_matrices(p, np.array([-1.0]), np.array([2.0]),
                                     xg[:, None], wg, np.ones(p + 1), np.ones(p + 1))
    hx, hy, hz = 0.3, 0.2, 0.45
    kappa = 2.5
    _, K2 = fcm.uncut_element_matrices(p, [hx, hy], 1.0, kappa)
    # local index a + n b: x fastest -> kron(y_op, x_op)
    ref2 = kappa * ((hy / hx) * np.kron(Mh, Kh) + (hx / hy) * np.kron(Kh, Mh))
    np.testing.assert_allclose(K2, ref2, rtol=1e-12, atol=1e-12)
    _, K3 = fcm.uncut_element_matrices(p, [hx, hy, hz], 1.0, kappa)
    ref3 = kappa * (hy * hz / (2 * hx) * np.kron(np.kron(Mh, Mh), Kh)
                    + hx * hz / (2 * hy) * np.kron(np.kron(Mh, Kh), Mh)
                    + hx * hy / (2 * hz) * np.kron(np.kron(Kh, Mh), Mh))
    np.testing.assert_allclose(K3, ref3, rtol=1e-12, atol=1e-12)


def test_small_3d_partition():
    w = inputs.small_3d()
    d = fcm.assemble(w)
    assert len(d.Ic) > 0 and len(d.Id) > 0
    one = np.zeros(d.n_grid)
    one[d.active] = 1.0
    assert np.max(np.abs(d.K @ one)) < 1e-11
    assert d.M[d.Id][:, d.Ic].count_nonzero() == 0
