"""Pins of the oracle's time integrators: the ten spring-coupled masses
(closed-form eigenvalues, the paper's critical steps, second-order
convergence, the stability limit of the explicit subsystem), the exact
discrete energy of the unforced IMEX scheme, and a standing mode on an
uncut square with Neumann boundaries."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import read_golden
from oracle import fcm, newmark, springs
from paper_2310_14712_amd import inputs

CRIT = {r[0]: (float(r[1]), int(r[2])) for r in read_golden("critical_steps.txt")}


def run_springs(dt, n_steps, scheme="imex", u0=None, v0=None, force=True):
    M, K, fx, Id, Ic = springs.matrices()
    if not force:
        fx = 0.0 * fx
    _, vref = springs.reference(np.array([0.0]))
    u0 = np.zeros(10) if u0 is None else u0
    v0 = vref if v0 is None else v0
    ft = springs.ft(np.arange(n_steps + 1) * dt)
    if scheme == "cdm":
        return newmark.cdm_run(M, K, fx, ft, u0, v0, dt, n_steps)
    if scheme == "trap":
        return newmark.trapezoidal_run(M, K, fx, ft, u0, v0, dt, n_steps)
    ig = newmark.NewmarkImex(M, K, fx, Id, Ic, dt)
    st = ig.initial_state(u0, v0, ft[0])
    return ig.run(st, ft, n_steps).u


def test_spring_critical_steps():
    M, K, _, Id, _ = springs.matrices()
    dtg = springs.dt_crit(K, M)
    dte = springs.dt_crit(K[np.ix_(Id, Id)], M[np.ix_(Id, Id)])
    # closed form of the explicit subsystem: 8x8 tridiag(-1, 2, -1)
    assert abs(dte - 1.0 / np.sin(4 * np.pi / 9)) < 1e-13
    for name, val in (("springs_global", dtg), ("springs_explicit", dte)):
        ref, digits = CRIT[name]
        assert float(f"{val:.{digits}g}") == ref


@pytest.mark.parametrize("scheme", ["imex", "cdm", "trap"])
def test_spring_second_order(scheme):
    T = 50.0
    errs = []
    for nt in (2000, 4000, 8000) if scheme == "cdm" else (200, 400, 800):
        u = run_springs(T / nt, nt, scheme)
        ref, _ = springs.reference(np.array([T]))
        errs.append(np.linalg.norm(u - ref[0]))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.85) and np.all(rates < 2.15), (errs, rates)


def test_spring_imex_stable_up_to_explicit_limit():
    """Elastic energy 1/2 u^T K u stays bounded at 0.99 dt_crit^explicit and
    grows without bound at 1.01 (Section "Spring-coupled masses")."""
    M, K, _, Id, _ = springs.matrices()
    dte = springs.dt_crit(K[np.ix_(Id, Id)], M[np.ix_(Id, Id)])
    energies = {}
    for f in (0.99, 1.01):
        dt = f * dte
        u = run_springs(dt, int(200.0 / dt))
        energies[f] = 0.5 * u @ K @ u
    assert energies[0.99] < 10.0
    assert energies[1.01] > 1e20


def test_spring_cdm_unstable_beyond_global_limit():
    M, K, _, _, _ = springs.matrices()
    dtg = springs.dt_crit(K, M)
    u = run_springs(1.05 * dtg, 400, "cdm")
    assert np.linalg.norm(u) > 1e6


def _energy_series(w, n_steps, seed=7, dt_factor=1.0):
    d = fcm.assemble(w)
    ig = newmark.NewmarkImex(d.M, d.K, 0 * d.fx, d.Id, d.Ic, dt_factor * d.dt)
    rng = np.random.default_rng(seed)
    u0 = np.zeros(d.n_grid)
    v0 = np.zeros(d.n_grid)
    u0[d.active] = rng.standard_normal(len(d.active))
    v0[d.active] = rng.standard_normal(len(d.active))
    sts = [ig.initial_state(u0, v0, 0.0)]
    for _ in range(n_steps + 1):
        sts.append(ig.step(sts[-1], 0.0, 0.0))
    return np.array([ig.energy(sts[k - 1], sts[k], sts[k + 1]) for k in range(1, n_steps)]), ig


def test_discrete_energy_conserved_config1():
    """Unforced config-1 mesh from a random state: the discrete IMEX energy
    is constant to roundoff over 300 steps."""
    E, _ = _energy_series(inputs.config1(), 300)
    assert np.max(np.abs(E - E[0])) / E[0] < 1e-12


def test_energy_detects_wrong_beta(monkeypatch):
    """Planted mistake: beta = 0.3 in the predictor/corrector breaks the
    invariant by far more than roundoff."""
    monkeypatch.setattr(newmark, "BETA", 0.3)
    E, _ = _energy_series(inputs.small_2d(), 100)
    assert np.max(np.abs(E - E[0])) / E[0] > 1e-6


def test_energy_detects_wrong_coupling(monkeypatch):
    """Planted mistake: predicting the c dofs with u^d_n instead of u^d_{n+1}
    (dropping the flowchart's u^d_pred = u^d_{n+1}) breaks the invariant."""
    orig = newmark.NewmarkImex.step

    def bad_step(self, st, ft_n, ft_np1):
        new = orig(self, st, ft_n, ft_np1)
        # recompute the implicit part with the old d values
        Id, Ic, dt = self.Id, self.Ic, self.dt
        uc_pred = st.u[Ic] + dt * st.vc + 0.25 * dt * dt * st.ac
        vc_pred = st.vc + 0.5 * dt * st.ac
        up = st.u.copy()
        up[Ic] = uc_pred
        ac = self.solve_S(ft_np1 * self.fx[Ic] - self.Kc @ up)
        new.u[Ic] = uc_pred + 0.25 * dt * dt * ac
        new.vc = vc_pred + 0.5 * dt * ac
        new.ac = ac
        return new

    monkeypatch.setattr(newmark.NewmarkImex, "step", bad_step)
    E, _ = _energy_series(inputs.small_2d(), 100)
    assert np.max(np.abs(E - E[0])) / E[0] > 1e-6


def test_tiny_mesh_eigen_bound_and_stability():
    """Dense eigenvalues of (K^dd, M^dd) on a 4x4 p=2 mesh with one hole give
    dt_crit^explicit; it is >= the cell-wise uncut value, the scheme is
    bounded just below it and grows just above it."""
    import scipy.linalg
    w = inputs.small_2d(n=(4, 4), p=2, holes=((0.5, 0.5, 0.3),), depth=3)
    d = fcm.assemble(w)
    Kdd = d.K[d.Id][:, d.Id].toarray()
    Mdd = d.M[d.Id][:, d.Id].toarray()
    lam = scipy.linalg.eigh(Kdd, Mdd, eigvals_only=True)[-1]
    dte = 2.0 / np.sqrt(lam)
    assert dte >= d.dt_crit_uncut * (1 - 1e-12)
    out = {}
    for f in (0.99, 1.01):
        ig = newmark.NewmarkImex(d.M, d.K, 0 * d.fx, d.Id, d.Ic, f * dte)
        rng = np.random.default_rng(3)
        u0 = np.zeros(d.n_grid)
        u0[d.active] = rng.standard_normal(len(d.active))
        st = ig.initial_state(u0, np.zeros(d.n_grid), 0.0)
        st = ig.run(st, np.zeros(4001), 4000)
        out[f] = np.linalg.norm(st.u)
    assert out[0.99] < 1e2
    assert not np.isfinite(out[1.01]) or out[1.01] > 1e6


def _standing_mode_error(n, p, nsteps, T, forced=None):
    w = inputs.Workload(name="standing", dim=2, n_cells=(n, n), p=p, tree_depth=0,
                        source=(0.5, 0.5), forced_cut=forced)
    d = fcm.assemble(w)
    grid = d.grid
    xs = np.linspace(0, 1, grid[0])
    # node coordinates: GLL points within each cell
    from oracle import basis
    xl, _ = basis.gll(p)
    coords = np.concatenate([[e / n + (xl[a] + 1) / (2 * n) for a in range(p)] for e in range(n)] + [[1.0]])
    X, Y = np.meshgrid(coords, coords, indexing="xy")
    k, l = 1, 1
    om = np.pi * np.sqrt(k * k + l * l)
    u0 = (np.cos(k * np.pi * X) * np.cos(l * np.pi * Y)).ravel()
    dt = T / nsteps
    ig = newmark.NewmarkImex(d.M, d.K, 0 * d.fx, d.Id, d.Ic, dt)
    st = ig.run(ig.initial_state(u0, np.zeros_like(u0), 0.0), np.zeros(nsteps + 1), nsteps)
    exact = u0 * np.cos(om * T)
    return np.linalg.norm(st.u - exact) / np.linalg.norm(exact), d


@pytest.mark.parametrize("forced", [None, "ring"])
def test_standing_mode_second_order_in_time(forced):
    """cos(pi x) cos(pi y) cos(sqrt(2) pi t) on the uncut unit square; with
    p = 4 the spatial error is negligible and the nodal error falls by 4 per
    halving of dt.  With some uncut cells forced to the implicit (consistent
    mass) treatment the same limit and order hold."""
    n, p, T = 4, 4, 0.5
    ids = np.array([5, 6, 9, 10]) if forced else None
    errs = []
    for ns in (20, 40, 80):
        e, d = _standing_mode_error(n, p, ns, T, ids)
        errs.append(e)
    if forced:
        assert len(d.Ic) > 0
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8) and np.all(rates < 2.2), (errs, rates)


def test_fully_implicit_mode_is_trapezoidal_newmark():
    """Every cell forced into the implicit block: the IMEX step has no d dofs
    and is the trapezoidal Newmark rule on all dofs (the fully implicit
    comparator, Section "Time Integration"); the same trajectory as the
    plain trapezoidal loop on the assembled M and K of the active dofs."""
    w = inputs.fully_implicit(inputs.small_2d(n=(6, 5), p=3, holes=((0.55, 0.45, 0.23),), depth=2))
    d = fcm.assemble(w)
    assert len(d.Id) == 0 and np.array_equal(np.sort(d.Ic), np.sort(d.active))
    act = np.sort(d.active)
    rng = np.random.default_rng(11)
    u0 = np.zeros(d.n_grid)
    v0 = np.zeros(d.n_grid)
    u0[act] = rng.standard_normal(len(act))
    v0[act] = rng.standard_normal(len(act))
    n = 60
    ft = inputs.ft_table(d.dt, n, w.source_freq)
    ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, d.dt)
    st = ig.run(ig.initial_state(u0, v0, ft[0]), ft, n)
    Ma = d.M.tocsr()[act][:, act]
    Ka = d.K.tocsr()[act][:, act]
    u_trap = newmark.trapezoidal_run(Ma, Ka, d.fx[act], ft, u0[act], v0[act], d.dt, n)
    assert np.linalg.norm(st.u[act] - u_trap) <= 1e-12 * np.linalg.norm(u_trap)


def test_beta_zero_is_central_differences_springs():
    """beta = 0 on the c block turns the IMEX step into the explicit central
    difference method on all dofs (Newmark with beta = 0, gamma = 1/2 is the
    two-step CDM): the same trajectory as the textbook two-step loop."""
    M, K, fx, Id, Ic = springs.matrices()
    dtg = springs.dt_crit(K, M)
    dt, n = 0.5 * dtg, 400
    _, vref = springs.reference(np.array([0.0]))
    ft = springs.ft(np.arange(n + 1) * dt)
    ig = newmark.NewmarkImex(M, K, fx, Id, Ic, dt, beta=0.0)
    u = ig.run(ig.initial_state(np.zeros(10), vref, ft[0]), ft, n).u
    u_cdm = newmark.cdm_run(newmark.imex_mass(M, Id, Ic), K, fx, ft, np.zeros(10), vref, dt, n)
    assert np.linalg.norm(u - u_cdm) <= 1e-11 * np.linalg.norm(u_cdm)


def test_global_critical_step_springs():
    """Lanczos on the sparse pencil reproduces the dense generalised
    eigenvalue problem and the tabulated global critical step."""
    M, K, _, _, _ = springs.matrices()
    dtg = newmark.global_critical_step(M, K, np.arange(10))
    assert abs(dtg - springs.dt_crit(K, M)) <= 1e-10 * dtg
    ref, digits = CRIT["springs_global"]
    assert float(f"{dtg:.{digits}g}") == ref


def test_cdm_comparator_stability_limit_on_mesh():
    """The central difference comparator (beta = 0) on a holed mesh: bounded
    (relative to the start) at 0.98 of the global critical step, unbounded
    at 1.02; the global step is below the uncut-cell step that the IMEX
    scheme runs at."""
    w = inputs.small_2d(n=(6, 5), p=3, holes=((0.55, 0.45, 0.23),), depth=2)
    d = fcm.assemble(w)
    dtg = newmark.global_critical_step(d.M, d.K, d.active)
    assert dtg < d.dt
    out = {}
    for f in (0.98, 1.02):
        ig = newmark.NewmarkImex(d.M, d.K, 0 * d.fx, d.Id, d.Ic, f * dtg, beta=0.0)
        u0 = np.zeros(d.n_grid)
        u0[d.active] = np.random.default_rng(3).standard_normal(len(d.active))
        st = ig.run(ig.initial_state(u0, np.zeros(d.n_grid), 0.0), np.zeros(3001), 3000)
        out[f] = np.linalg.norm(st.u) / np.linalg.norm(u0)
    assert out[0.98] < 1e2
    assert not np.isfinite(out[1.02]) or out[1.02] > 1e6


def test_hrz_lumping_of_cut_cells():
    """HRZ-lumped cut-cell masses: diagonal and positive, the total mass of
    every cell kept; on a bilinear square (p = 1, forced cut, no boundary)
    each node gets a quarter of the cell's mass, the row-sum lumping."""
    w = inputs.small_2d(n=(6, 5), p=3, holes=((0.55, 0.45, 0.23),), depth=2)
    d = fcm.assemble(w)
    w.cut_mass = "hrz"
    dh = fcm.assemble(w)
    cut = d.flags == fcm.CUT
    assert cut.any()
    Mcc = dh.M.tocsr()[dh.Ic][:, dh.Ic]
    off = Mcc - sp.diags(Mcc.diagonal())
    assert abs(off).max() == 0.0 and Mcc.diagonal().min() > 0
    assert abs(dh.M.sum() - d.M.sum()) <= 1e-12 * d.M.sum()
    sq = inputs.Workload(name="sq", dim=2, n_cells=(1, 1), p=1, tree_depth=0, source=(0.5, 0.5),
                         extent=(0.5, 0.25, 1.0), forced_cut=np.array([0]), cut_mass="hrz")
    ds = fcm.assemble(sq)
    assert np.allclose(ds.M.diagonal()[ds.active], 0.5 * 0.25 / 4, rtol=1e-14, atol=0)


@pytest.mark.parametrize("dim,p", [(2, 3), (2, 4), (3, 2)])
def test_point_sampling_reproduces_tensor_polynomials(dim, p):
    """Receiver sampling of the finite element field: nodal values of a
    polynomial of degree p in each variable are reproduced exactly at
    arbitrary points (the tensor GLL basis spans Q_p)."""
    from oracle import basis
    w = (inputs.small_2d(n=(5, 4), p=p, holes=((0.55, 0.45, 0.23),), depth=2) if dim == 2
         else inputs.small_3d(n=(4, 3, 5), p=p))
    xl, _ = basis.gll(p)
    coords = []
    for k in range(dim):
        n, h = w.n_cells[k], w.h[k]
        coords.append(np.concatenate([[e * h + (xl[a] + 1) * h / 2 for a in range(p)] for e in range(n)]
                                     + [[n * h]]))
    mesh = np.meshgrid(*coords, indexing="ij")          # mesh[k][i0, i1, ...]
    rng = np.random.default_rng(1)
    cf = rng.standard_normal((p + 1,) * dim)

    def f(X):                                            # sum_c cf[c] prod_k x_k^c_k
        val = 0.0
        for idx in np.ndindex(*cf.shape):
            term = cf[idx]
            for k in range(dim):
                term = term * X[k] ** idx[k]
            val = val + term
        return val
    u = f(mesh).transpose().ravel()                       # x fastest
    flags = fcm.classify(w)
    pts = []
    while len(pts) < 25:
        x = rng.uniform(0, 1, dim) * np.array(w.extent[:dim])
        cidx = [min(int(x[k] / w.h[k]), w.n_cells[k] - 1) for k in range(dim)]
        cid = sum(cidx[k] * int(np.prod(w.n_cells[:k])) for k in range(dim))
        if flags[cid] != fcm.EMPTY:
            pts.append(x)
    pts = np.array(pts)
    got = fcm.sample_points(w, u, pts)
    want = np.array([f(list(x)) for x in pts])
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))
