"""GPU parity of the FP32 explicit path (FP32 grid state in increment form,
FP64 arithmetic; FP64 implicit block) against the FP64 oracle.

Metric and tolerance: relative L2 error <= 1e-6 of the displacement field,
measured (a) as the nodal L2 norm over the d dofs and (b) as the L2 norm of
the finite-element field, ||e||_M / ||u||_M with the FCM mass matrix (which
weights the fictitious part of cut cells by alpha_f).  The nodal L2 norm over
all active dofs is reported but not gated: on cut cells with a small physical
fraction the basis functions centred in the fictitious part have almost no
mass and stiffness of their own, so their nodal values are extrapolations of
the physical field and magnify any perturbation of it by one to two orders
(on the 16x16 plate the largest errors sit on c nodes with M_ii ~ 1e-9
against ~1e-4 for a physical node).  FP32 storage of the state perturbs the
physical field by unit roundoffs (2^-24 ~ 6e-8) every step, so that nodal
error passes 1e-6 long before the field error does.  The field error itself
grows about linearly with the step count and stays below 1e-6 up to about a
thousand steps of the 128x128 plate; the tests keep to such horizons.
"""
import numpy as np
import pytest

from oracle import fcm, newmark
from paper_2310_14712_amd import inputs

pytestmark = pytest.mark.gpu
TOL_U = 1e-6
# The c state enters the next displacement through the predictor and the
# corrector as dt v^c and dt^2/4 a^c; its errors are gated in those
# displacement units (M^cc norm over the field's ||u||_M).  Relative to their
# own norms they are not meaningful: accelerations weight the white FP32
# roundoff by omega^2, up to (omega_max dt)^2 ~ 3 per step against the
# signal's (omega dt)^2 << 1.


def _imex():
    from paper_2310_14712_amd import imex
    return imex


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_m(M, a, b):
    e = a - b
    nb = np.sqrt(b @ (M @ b))
    return np.sqrt(e @ (M @ e)) / (nb if nb > 0 else 1.0)


def errors(lib, d, st, dt):
    imex = _imex()
    cn = lib.export_index(imex.INDEX_C_NODES)
    pos = np.searchsorted(d.Ic, cn)
    u = lib.read(imex.FIELD_U)
    out = {"u_d": rel(u[d.Id], st.u[d.Id]), "u_field": rel_m(d.M, u, st.u),
           "u_prev_d": rel(lib.read(imex.FIELD_UPREV)[d.Id], st.ud_prev),
           "u_nodal_all": rel(u, st.u)}
    if len(cn):
        Mcc = d.M[d.Ic][:, d.Ic]
        u_norm = np.sqrt(st.u @ (d.M @ st.u))
        vc = np.empty(len(d.Ic))
        ac = np.empty(len(d.Ic))
        vc[pos] = lib.read(imex.FIELD_VC)
        ac[pos] = lib.read(imex.FIELD_AC)
        ev, ea = vc - st.vc, ac - st.ac
        out["v_c"] = dt * np.sqrt(ev @ (Mcc @ ev)) / u_norm
        out["a_c"] = 0.25 * dt * dt * np.sqrt(ea @ (Mcc @ ea)) / u_norm
    inactive = np.setdiff1d(np.arange(d.n_grid), d.active)
    assert np.all(u[inactive] == 0.0)
    return out


def check(errs, tol=TOL_U):
    for k, e in errs.items():
        if k == "u_nodal_all":
            continue  # reported only (see the module docstring)
        assert e <= tol, (k, e, errs)


def run_fp32(w, horizons, seed=None):
    """Run the FP32 library and the FP64 oracle side by side; return the
    errors at each horizon (steps from the start)."""
    imex = _imex()
    print(f"\n[case] fp32 {w.name} dim={w.dim} cells={tuple(w.n_cells)} p={w.p} horizons={horizons}",
          flush=True)
    d = fcm.assemble(w)
    lib = imex.Imex(w, explicit_fp=32)
    lib.assemble()
    dt = lib.info()["dt"]
    n = max(horizons)
    ft = inputs.ft_table(dt, n, w.source_freq)
    if seed is None:
        u0 = v0 = np.zeros(d.n_grid)
    else:
        rng = np.random.default_rng(seed)
        u0 = np.zeros(d.n_grid)
        v0 = np.zeros(d.n_grid)
        # smooth data (a random combination of low modes) so the FP32 input
        # rounding is not the dominant error
        x = [np.linspace(0, 1, k) for k in d.grid]
        X = np.meshgrid(*x, indexing="ij")
        for _ in range(3):
            kx = rng.integers(1, 4, size=w.dim)
            ph = np.prod([np.sin(np.pi * kk * XX) for kk, XX in zip(kx, X)], axis=0)
            u0 += rng.standard_normal() * ph.T.reshape(-1) if w.dim == 2 else \
                rng.standard_normal() * ph.transpose(2, 1, 0).reshape(-1)
        u0[np.setdiff1d(np.arange(d.n_grid), d.active)] = 0.0
    ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, dt)
    st = ig.initial_state(u0, v0, ft[0])
    lib.set_initial(u0, v0, ft[0])
    out = {}
    k = 0
    for h in sorted(horizons):
        lib.step(ft[k:h + 1])
        st = ig.run(st, ft[k:], h - k)
        k = h
        out[h] = errors(lib, d, st, dt)
        print(f"[case] fp32 {w.name} step {h}: {out[h]}", flush=True)
    return out


def test_fp32_config1_200_steps():
    errs = run_fp32(inputs.config1(), [50, 200])
    for e in errs.values():
        check(e)


def test_fp32_cube_replica_1000_steps():
    """The 24^3 replica of the 64^3 p = 3 voided cube from rest, FP32 state:
    <= 1e-6 at 200 and 1000 steps.  (At 2000 steps, the cube's horizon, the
    field error is 1.1e-6, so the cube benchmarks keep the FP64 state.)"""
    errs = run_fp32(inputs.config3_replica(), [200, 1000])
    for e in errs.values():
        check(e)


def test_fp32_config2_1000_steps():
    """The 128x128 p=4 perforated plate, FP32 explicit part: <= 1e-6 at
    200 and 1000 steps."""
    errs = run_fp32(inputs.config2(), [200, 1000])
    for e in errs.values():
        check(e)


@pytest.mark.parametrize("p", [2, 3, 5, 7])
def test_fp32_2d_orders(p):
    w = inputs.small_2d(n=(9, 7), p=p, holes=((0.55, 0.45, 0.23), (0.2, 0.8, 0.12)), depth=2,
                        source=(0.05, 0.3))
    errs = run_fp32(w, [33, 100], seed=p)
    for e in errs.values():
        check(e)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_fp32_3d_orders(p):
    w = inputs.small_3d(n=(6, 5, 7), p=p, holes=((0.5, 0.45, 0.55, 0.3), (0.1, 0.9, 0.1, 0.25)), depth=1)
    errs = run_fp32(w, [40, 100], seed=10 + p)
    for e in errs.values():
        check(e)


def test_fp32_large_tiles_2d():
    w = inputs.small_2d(n=(70, 37), p=4, holes=((0.5, 0.5, 0.11), (0.8, 0.2, 0.05)), depth=3,
                        source=(0.1, 0.5))
    check(run_fp32(w, [64])[64])


def test_fp32_one_step_explicit_part():
    """One step from an injected state, compared with the oracle's step from
    the same state rounded to FP32: the d part of u_{n+1} and its increment
    within a few FP32 roundoffs of the state, and a^c_{n+1} solving the
    oracle's system with the library's own u^d_{n+1} (normwise backward
    error <= 1e-14, FP64 solve)."""
    imex = _imex()
    w = inputs.small_2d(n=(7, 5), p=4, holes=((0.55, 0.45, 0.23),), depth=2, source=(0.2, 0.3))
    d = fcm.assemble(w)
    lib = imex.Imex(w, explicit_fp=32)
    lib.assemble()
    dt = lib.info()["dt"]
    ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, dt)
    ft = inputs.ft_table(dt, 40, w.source_freq) + 0.3
    st = ig.run(ig.initial_state(np.zeros(d.n_grid), np.zeros(d.n_grid), ft[0]), ft, 30)
    # the oracle state as the library holds it: u and u_{n-1} in FP32
    st.u = st.u.astype(np.float32).astype(np.float64)
    st.ud_prev = st.ud_prev.astype(np.float32).astype(np.float64)
    cn = lib.export_index(imex.INDEX_C_NODES)
    pos = np.searchsorted(d.Ic, cn)
    up = np.zeros(d.n_grid)
    up[d.Id] = st.ud_prev
    lib.set_initial(None, None, 0.0)
    lib.set_state(imex.FIELD_U, st.u)
    lib.set_state(imex.FIELD_UPREV, up)
    lib.set_state(imex.FIELD_VC, st.vc[pos])
    lib.set_state(imex.FIELD_AC, st.ac[pos])
    lib.step(ft[30:32])
    st1 = ig.step(st, ft[30], ft[31])
    u = lib.read(imex.FIELD_U)
    e_ud = rel(u[d.Id], st1.u[d.Id])
    # the FP32 increment u_{n+1} - u_n before u_{n+1} is rounded: its error
    # is that of the FP32 apply, a few roundoffs of the state
    inc = lib.read(imex.FIELD_DELTA)[d.Id]
    e_inc = np.linalg.norm(inc - (st1.u[d.Id] - st.u[d.Id])) / np.linalg.norm(st1.u[d.Id])
    a = np.empty(len(d.Ic))
    a[pos] = lib.read(imex.FIELD_AC)
    Ic = d.Ic
    u_pred = u.copy()
    u_pred[Ic] = st.u[Ic] + dt * st.vc + 0.25 * dt * dt * st.ac
    r = ft[31] * ig.fx[Ic] - ig.Kc @ u_pred
    import scipy.sparse.linalg as spla
    be = np.linalg.norm(ig.S @ a - r) / (spla.norm(ig.S) * np.linalg.norm(a) + np.linalg.norm(r))
    print(f"[case] fp32 one step: u_d {e_ud:.3e} increment {e_inc:.3e} a_c backward {be:.3e}", flush=True)
    assert e_ud <= 2e-7, e_ud
    assert e_inc <= 2e-7, e_inc
    assert be <= 1e-14, be


def test_fp32_checkpoint_resume_bitwise():
    """U, UPREV, the FP64 u^c, VC, AC and the FP32 increment restore a run
    bit for bit."""
    imex = _imex()
    w = inputs.small_2d(n=(6, 6), p=4, depth=3)
    a = imex.Imex(w, explicit_fp=32)
    a.assemble()
    dt = a.info()["dt"]
    ft = inputs.ft_table(dt, 80, 10.0)
    a.set_initial(None, None, ft[0])
    a.step(ft[:41])
    keys = (imex.FIELD_U, imex.FIELD_UPREV, imex.FIELD_UC, imex.FIELD_VC, imex.FIELD_AC, imex.FIELD_DELTA)
    snap = {k: a.read(k) for k in keys}
    a.step(ft[40:])
    b = imex.Imex(w, explicit_fp=32)
    b.assemble()
    b.set_initial(None, None, 0.0)
    for k in keys:
        b.set_state(k, snap[k])
    b.step(ft[40:])
    for k in keys:
        assert np.array_equal(a.read(k), b.read(k)), k


def test_fp32_graph_independent():
    import os
    imex = _imex()
    w = inputs.config1()
    outs = []
    for no_graph in ("0", "1"):
        os.environ["IMEX_NO_GRAPH"] = no_graph
        try:
            lib = imex.Imex(w, explicit_fp=32)
            lib.assemble()
            ft = inputs.ft_table(lib.info()["dt"], 70, 10.0)
            lib.set_initial(None, None, ft[0])
            lib.step(ft)
            outs.append(lib.read(imex.FIELD_U))
            lib.close()
        finally:
            os.environ.pop("IMEX_NO_GRAPH", None)
    assert np.array_equal(outs[0], outs[1])


def test_increment_field_rejected_in_fp64():
    imex = _imex()
    lib = imex.Imex(inputs.config1())
    lib.assemble()
    lib.set_initial(None, None, 0.0)
    with pytest.raises(imex.ImexError):
        lib.read(imex.FIELD_DELTA)
