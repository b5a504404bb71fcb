"""The C-ABI library without a GPU: it loads, exports every declared entry
point, and its C++ host setup (classification, partition, K^c, M^cc, S, the
critical step) agrees with the oracle, which shares no code with it."""
import dataclasses
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import ROOT
from oracle import fcm, newmark
from paper_2310_14712_amd import inputs

imex = pytest.importorskip("paper_2310_14712_amd.imex")


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "imex.h")).read()
    return sorted(set(re.findall(r"\b(imex_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    syms = declared_symbols()
    assert "imex_step" in syms and "imex_setup_mesh" in syms
    for s in syms:
        assert hasattr(imex._lib, s), s
    assert sorted(syms) == sorted(imex.EXPORTED)


CASES = {
    "config1": inputs.config1,
    "small2d": inputs.small_2d,
    "small2d_p1_two_holes": lambda: inputs.small_2d(n=(7, 5), p=1, holes=((0.3, 0.4, 0.2), (0.75, 0.6, 0.17)), depth=4),
    "small2d_p6": lambda: inputs.small_2d(n=(3, 4), p=6, holes=((0.6, 0.5, 0.3),), depth=2),
    "small3d": inputs.small_3d,
    "small3d_p3": lambda: inputs.small_3d(n=(3, 3, 4), p=3, holes=((0.5, 0.5, 0.5, 0.31), (0.1, 0.9, 0.9, 0.2)), depth=2),
    "forced": lambda: inputs.Workload(name="forced", dim=2, n_cells=(4, 4), p=3, tree_depth=0,
                                      source=(0.1, 0.1), forced_cut=np.array([5, 6, 9])),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    w = CASES[request.param]()
    lib = imex.Imex(w, device_mode=imex.HOST_ONLY)
    lib.assemble()
    return w, lib, fcm.assemble(w)


def test_classification_and_partition(pair):
    w, lib, d = pair
    inf = lib.info()
    assert np.array_equal(lib.export_index(imex.INDEX_CELL_FLAGS), d.flags)
    assert np.array_equal(np.sort(lib.export_index(imex.INDEX_C_NODES)), d.Ic)
    assert np.array_equal(lib.export_index(imex.INDEX_D_NODES), d.Id)
    assert inf["n_active"] == len(d.active)
    assert inf["n_grid"] == d.n_grid
    assert abs(inf["dt"] - d.dt) / d.dt < 1e-13
    assert abs(inf["dt_crit_uncut"] - d.dt_crit_uncut) / d.dt_crit_uncut < 1e-13


def test_implicit_block_matrices(pair):
    w, lib, d = pair
    cn = lib.export_index(imex.INDEX_C_NODES)
    nc = len(cn)
    if nc == 0:
        return
    dt = lib.info()["dt"]
    rp, cols, vals = lib.export_csr(imex.CSR_KC)
    Kc = sp.csr_matrix((vals, cols, rp), shape=(nc, d.n_grid))
    ref = d.K[cn]
    assert abs(Kc - ref).max() <= 1e-13 * abs(ref).max()
    rp, cols, vals = lib.export_csr(imex.CSR_MCC)
    Mcc = sp.csr_matrix((vals, cols, rp), shape=(nc, nc))
    Mref = d.M[cn][:, cn]
    assert abs(Mcc - Mref).max() <= 1e-13 * abs(Mref).max()
    rp, cols, vals = lib.export_csr(imex.CSR_S)
    S = sp.csr_matrix((vals, cols, rp), shape=(nc, nc))
    Sref = Mref + 0.25 * dt * dt * d.K[cn][:, cn]
    assert abs(S - Sref).max() <= 1e-13 * abs(Sref).max()
    # components are contiguous in c order and S has no coupling across them
    cp = lib.export_index(imex.INDEX_COMP_PTR)
    lab = np.searchsorted(cp, np.arange(nc), side="right") - 1
    coo = S.tocoo()
    assert np.all(lab[coo.row] == lab[coo.col])
    ncomp, _ = fcm.c_components(d)
    assert len(cp) - 1 == ncomp


def test_config2_counts_match_oracle():
    w = inputs.config2()
    lib = imex.Imex(w, device_mode=imex.HOST_ONLY)
    lib.assemble()
    d = fcm.assemble(w)
    inf = lib.info()
    assert np.array_equal(lib.export_index(imex.INDEX_CELL_FLAGS), d.flags)
    assert inf["n_c"] == len(d.Ic) and inf["n_d"] == len(d.Id)


def test_errors_are_reported():
    w = inputs.small_2d()
    w.p = 0
    with pytest.raises(imex.ImexError, match="EINVAL"):
        imex.Imex(w, device_mode=imex.HOST_ONLY)
    w = inputs.small_2d(holes=((0.1, 0.3, 0.25),))   # source inside a hole's empty cell
    with pytest.raises(imex.ImexError, match="empty cell"):
        imex.Imex(w, device_mode=imex.HOST_ONLY)
    lib = imex.Imex(inputs.small_2d(), device_mode=imex.HOST_ONLY)
    with pytest.raises(imex.ImexError, match="ESTATE"):
        lib.step(np.zeros(3))
    lib.assemble()
    with pytest.raises(imex.ImexError, match="ESTATE"):
        lib.set_initial()
    with pytest.raises(imex.ImexError, match="ESTATE"):   # failure detection needs a device state
        lib.set_check_finite(True)


@pytest.mark.parametrize("case", ["holed_2d", "holed_2d_hrz", "config1", "3d"])
def test_global_critical_step_matches_oracle(case):
    """The library's power iteration against Lanczos (SciPy eigsh) on the
    same pencil: approached from above, within 1e-4."""
    w = {"holed_2d": lambda: inputs.small_2d(n=(6, 5), p=3, holes=((0.55, 0.45, 0.23),), depth=2),
         "holed_2d_hrz": lambda: dataclasses.replace(
             inputs.small_2d(n=(6, 5), p=3, holes=((0.55, 0.45, 0.23),), depth=2), cut_mass="hrz"),
         "config1": inputs.config1,
         "3d": lambda: inputs.small_3d(n=(4, 3, 5), p=2)}[case]()
    d = fcm.assemble(w)
    ref = newmark.global_critical_step(d.M, d.K, d.active)
    lib = imex.Imex(w, device_mode=imex.HOST_ONLY)
    lib.assemble()
    g = lib.global_critical_step()
    assert g >= ref * (1 - 1e-12)
    assert g <= ref * (1 + 1e-4)


def test_newmark_beta_setter():
    lib = imex.Imex(inputs.small_2d(), device_mode=imex.HOST_ONLY)
    with pytest.raises(imex.ImexError, match="EINVAL"):
        lib.set_newmark_beta(0.7)
    with pytest.raises(imex.ImexError, match="ESTATE"):
        lib.global_critical_step()
    lib.set_newmark_beta(0.0)
    lib.assemble()
    with pytest.raises(imex.ImexError, match="ESTATE"):
        lib.set_newmark_beta(0.25)


def test_kc_and_s_rows_against_oracle_on_cube_replica():
    """The host assembly of the 24^3 replica of the voided cube: 100 sampled
    rows of K^c and S against rows summed from the oracle's element matrices
    of the cells around each node (tree-integrated cut cells, exact uncut
    stiffness, lumped uncut mass); the GPU test repeats this at full size."""
    import rowcheck
    w = inputs.config3_replica()
    lib = imex.Imex(w, device_mode=imex.HOST_ONLY)
    lib.assemble()
    inf = lib.info()
    rows = np.random.default_rng(3).choice(inf["n_c"], size=100, replace=False)
    err = rowcheck.max_row_error(w, lib, inf["dt"], rows)
    assert err <= 1e-12, err
