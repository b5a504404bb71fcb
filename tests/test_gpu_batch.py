"""Batched instances and the tile autotuner, through the C ABI.

A batch steps independent contexts together.  The default form launches each
kernel type once per step over all instances (per-instance argument tables,
32-step chunks captured in one graph); the other forms replay the instances'
own 32-step graphs over several streams, or one graph per 32 steps with a
branch per instance.  Instances share no data, so a batched run must
reproduce every instance's own run bit for bit; the autotuner only changes
the launch shape of the explicit kernel, whose per-node summation order is
fixed, so tuned and untuned runs are bitwise equal too.  Eight FP64
instances of orders 2 to 6 are also checked against the oracle.  The
per-kernel timing events sit between launches that the stream orders
anyway, so timed runs (steps launched one by one) and untimed ones (captured
chunks) are bitwise equal as well.
"""
import numpy as np
import pytest

import tolerances
from oracle import fcm, newmark
from paper_2310_14712_amd import inputs

pytestmark = pytest.mark.gpu


def _imex():
    from paper_2310_14712_amd import imex
    return imex


def small_instances(k, fp, orders=None):
    """k uneven 2D instances in the style of the batched workload, shrunk
    (N ~ U{6..20}) so the oracle can follow them; orders: the p of every
    instance (else p ~ U{2..6})."""
    out = []
    for i in range(k):
        rng = np.random.default_rng(700 + i)
        n = int(rng.integers(6, 21))
        p = int(rng.integers(2, 7))
        if orders is not None:
            p = orders[i]
        nh = int(rng.integers(1, 4))
        c = np.stack([rng.uniform(0.3, 1.0, nh), rng.uniform(0.0, 1.0, nh)], axis=1)
        r = rng.uniform(0.08, 0.2, nh)
        src = (float(rng.uniform(0.02, 0.1)), float(rng.uniform(0.1, 0.9)))
        out.append(inputs.Workload(name=f"inst{i}_n{n}_p{p}", dim=2, n_cells=(n, n + i % 3), p=p, tree_depth=2,
                                   hole_centers=c, hole_radii=r, source=src, explicit_fp=fp))
    return out


def make(ws, tune=False):
    imex = _imex()
    libs = []
    for w in ws:
        lib = imex.Imex(w)
        lib.assemble()
        if tune:
            lib.autotune_tiles(5)
        libs.append(lib)
    return libs


@pytest.mark.parametrize("fp,lanes", [(64, None), (32, None), (64, "16"), (32, "16"), (64, "0"), (32, "3")])
def test_batch_equals_individual_runs(fp, lanes, monkeypatch):
    """Every batch form (batched kernels, streams lanes, or one graph with a
    branch per instance) against the instances stepped alone."""
    imex = _imex()
    if lanes is not None:
        monkeypatch.setenv("IMEX_BATCH_LANES", lanes)
    else:
        monkeypatch.delenv("IMEX_BATCH_LANES", raising=False)
    ws = small_instances(6, fp)
    print(f"\n[case] batch fp{fp} lanes {lanes}: " + ", ".join(w.name for w in ws), flush=True)
    n_steps = 70                      # two graph chunks and an eager tail
    tabs = []
    solo = make(ws)
    for w, lib in zip(ws, solo):
        ft = inputs.ft_table(lib.info()["dt"], n_steps, w.source_freq)
        tabs.append(ft)
        lib.set_initial(None, None, ft[0])
        lib.step(ft)
    bat = make(ws, tune=True)
    for lib, ft in zip(bat, tabs):
        lib.set_initial(None, None, ft[0])
    b = imex.Batch(bat)
    assert b.form() == (imex.BATCH_KERNELS if lanes is None else
                        imex.BATCH_GRAPH if lanes == "0" else imex.BATCH_LANES)
    b.step(40, tables=[t[:41] for t in tabs])
    b.step(30, tables=[t[40:] for t in tabs])
    b.close()
    for w, s, t in zip(ws, solo, bat):
        assert np.linalg.norm(s.read(imex.FIELD_U)) > 0, w.name   # the source has acted
        for k in (imex.FIELD_U, imex.FIELD_UPREV, imex.FIELD_UC, imex.FIELD_VC, imex.FIELD_AC):
            assert np.array_equal(s.read(k), t.read(k)), (w.name, k)
        assert t.info()["steps_taken"] == n_steps


def test_autotuned_tiles_bitwise():
    imex = _imex()
    w = inputs.small_2d(n=(37, 23), p=4, holes=((0.5, 0.5, 0.11), (0.8, 0.2, 0.05)), depth=3, source=(0.1, 0.5))
    a, b = make([w, w])
    tiles = b.autotune_tiles(10)
    print(f"\n[case] autotuned tiles {tiles}", flush=True)
    ft = inputs.ft_table(a.info()["dt"], 45, 10.0)
    for lib in (a, b):
        lib.set_initial(None, None, ft[0])
        lib.step(ft)
    assert np.linalg.norm(a.read(imex.FIELD_U)) > 0
    assert np.array_equal(a.read(imex.FIELD_U), b.read(imex.FIELD_U))


def test_autotune_3d_bitwise():
    imex = _imex()
    w = inputs.small_3d(n=(9, 7, 11), p=3, holes=((0.5, 0.5, 0.5, 0.2),), depth=1)
    a, b = make([w, w])
    tiles = b.autotune_tiles(3)
    print(f"\n[case] autotuned 3D tiles {tiles}", flush=True)
    ft = inputs.ft_table(a.info()["dt"], 12, 10.0)
    for lib in (a, b):
        lib.set_initial(None, None, ft[0])
        lib.step(ft)
    assert np.linalg.norm(a.read(imex.FIELD_U)) > 0
    assert np.array_equal(a.read(imex.FIELD_U), b.read(imex.FIELD_U))


@pytest.mark.parametrize("dim", [2, 3])
def test_step_timing_events_bitwise(dim):
    imex = _imex()
    if dim == 2:
        w = inputs.small_2d(n=(37, 23), p=4, holes=((0.5, 0.5, 0.11),), depth=3, source=(0.1, 0.5))
    else:
        w = inputs.small_3d(n=(9, 7, 11), p=3, holes=((0.5, 0.5, 0.5, 0.2),), depth=1)
    a, b = make([w, w])
    b.set_step_timing(True)
    with pytest.raises(imex.ImexError):
        b.step_timing()  # no chunk has run yet
    n = 70  # untimed: two captured 32-step chunks and 6 single steps; timed: 70 single steps
    ft = inputs.ft_table(a.info()["dt"], n, 10.0)
    for lib in (a, b):
        lib.set_initial(None, None, ft[0])
        lib.step(ft)
    ms = b.step_timing()
    print(f"\n[case] {dim}D step timing (ms): {ms}", flush=True)
    assert set(ms) == {"explicit", "rhs", "solve"}
    assert all(0.0 < v < 1e3 for v in ms.values())
    assert np.linalg.norm(a.read(imex.FIELD_U)) > 0
    for f in (imex.FIELD_U, imex.FIELD_UPREV, imex.FIELD_UC, imex.FIELD_VC, imex.FIELD_AC):
        assert np.array_equal(a.read(f), b.read(f))
    b.set_step_timing(False)
    with pytest.raises(imex.ImexError):
        b.step_timing()


def test_batch_against_oracle():
    """Eight FP64 instances of orders p = 2..6 through the batched kernels,
    against the oracle (the FP64 trajectory tolerance of the plain path)."""
    imex = _imex()
    ws = small_instances(8, 64, orders=[2, 3, 4, 5, 6, 4, 3, 2])
    libs = make(ws, tune=True)
    n_steps = 64
    tabs = []
    for w, lib in zip(ws, libs):
        ft = inputs.ft_table(lib.info()["dt"], n_steps, w.source_freq)
        tabs.append(ft)
        lib.set_initial(None, None, ft[0])
    b = imex.Batch(libs)
    assert b.form() == imex.BATCH_KERNELS
    b.step(n_steps, tables=tabs)
    b.close()
    for w, lib, ft in zip(ws, libs, tabs):
        d = fcm.assemble(w)
        ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, lib.info()["dt"])
        st = ig.run(ig.initial_state(np.zeros(d.n_grid), np.zeros(d.n_grid), ft[0]), ft, n_steps)
        u = lib.read(imex.FIELD_U)
        err = np.linalg.norm(u - st.u) / np.linalg.norm(st.u)
        print(f"[case] batch {w.name}: rel L2 {err:.2e}", flush=True)
        assert err <= tolerances.trajectory_tolerances()["u"], (w.name, err)


def test_batched_workload_slice_bitwise():
    """The first eight instances of the 64-instance workload at full size
    (33^2 .. 128^2 cells, p = 2..6, FP32 state), 64 steps batched against the
    same instances stepped one by one."""
    imex = _imex()
    ws = inputs.config4_instances(8)
    print("\n[case] config4 slice " + ", ".join(f"{w.n_cells[0]}^2 p{w.p}" for w in ws), flush=True)
    solo, bat = make(ws), make(ws, tune=True)
    tabs = []
    for w, lib in zip(ws, solo):
        ft = inputs.ft_table(lib.info()["dt"], 64, w.source_freq)
        tabs.append(ft)
        lib.set_initial(None, None, ft[0])
        lib.step(ft)
    for lib, ft in zip(bat, tabs):
        lib.set_initial(None, None, ft[0])
    b = imex.Batch(bat)
    b.step(64, tables=tabs)
    b.close()
    for w, s, t in zip(ws, solo, bat):
        assert np.linalg.norm(s.read(imex.FIELD_U)) > 0, w.name
        assert np.array_equal(s.read(imex.FIELD_U), t.read(imex.FIELD_U)), w.name
