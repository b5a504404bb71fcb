"""The allocation-free sampling entry point (imex_sample_field_noalloc)
against the allocating one (imex_sample_field), through the C ABI.

Both evaluate the finite element field of the same library state at the
same physical points.  The allocation-free call stages points and values in
the library's device scratch array and evaluates the cell basis on the
device; the allocating one evaluates it on the host.  FP64 results agree to
rounding (bound 1e-14 of the field's maximum).  Two calls in a row, the
second with fewer points, check that the scratch's leftover contents from
the first call do not leak into the second; a third call of more points than
the scratch holds is refused on the host.
"""
import numpy as np
import pytest

from oracle import fcm
from paper_2310_14712_amd import inputs

pytestmark = pytest.mark.gpu


def _points(w, n, seed):
    """n seeded points of active (non-empty) cells."""
    flags = fcm.classify(w)
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(0, 1, w.dim) * np.array(w.extent[:w.dim])
        cidx = [min(int(x[k] / w.h[k]), w.n_cells[k] - 1) for k in range(w.dim)]
        cid = sum(cidx[k] * int(np.prod(w.n_cells[:k])) for k in range(w.dim))
        if flags[cid] != fcm.EMPTY:
            pts.append(x)
    return np.array(pts)


CASES = {
    "2d_p4_fp64": lambda: inputs.small_2d(n=(9, 7), p=4, holes=((0.55, 0.45, 0.23),), depth=2),
    "3d_p3_fp32": lambda: inputs.small_3d(n=(5, 4, 6), p=3, holes=((0.5, 0.45, 0.55, 0.3),), depth=1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_noalloc_sampling_matches(name):
    from paper_2310_14712_amd import imex
    w = CASES[name]()
    if name.endswith("fp32"):
        w.explicit_fp = 32
    print(f"\n[case] noalloc sampling {name} cells={tuple(w.n_cells)} p={w.p}", flush=True)
    lib = imex.Imex(w)
    lib.assemble()
    dt = lib.info()["dt"]
    ft = inputs.ft_table(dt, 25, w.source_freq)
    u0 = np.zeros(w.n_grid)
    d = fcm.assemble(w)
    u0[d.active] = inputs.random_field(len(d.active), 3)
    lib.set_initial(u0, None, ft[0])
    lib.step(ft)
    umax = np.max(np.abs(lib.read(imex.FIELD_U)))
    for n_pts, seed in ((300, 1), (37, 2)):     # second call smaller than the first
        pts = _points(w, n_pts, seed)
        for which in (imex.FIELD_U, imex.FIELD_UPREV):
            want = lib.sample(pts, which)
            got = lib.sample_noalloc(pts, which)
            err = np.max(np.abs(got - want))
            print(f"[case] {name} n={n_pts} field={which}: max abs diff {err:.2e}", flush=True)
            assert err <= 1e-14 * umax, err
    big = imex.sample_noalloc_max_points(w.dim) + 1
    pts = np.tile(_points(w, 1, 4), (big, 1))
    with pytest.raises(imex.ImexError, match="too many sample points"):
        lib.sample_noalloc(pts)
    # a point in an empty cell is refused as by the allocating call
    flags = fcm.classify(w)
    empty = np.flatnonzero(flags == fcm.EMPTY)
    if len(empty):
        cidx = np.unravel_index(int(empty[0]), tuple(reversed(w.n_cells)))[::-1]
        centre = (np.array(cidx) + 0.5) * np.array(w.h)
        with pytest.raises(imex.ImexError, match="empty cell"):
            lib.sample_noalloc(centre[None, :])
    lib.close()
