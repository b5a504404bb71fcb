"""Failure detection of the time loop: with the finite-state check on, a step
call ends with a scan of the state and reports IMEX_EUNSTABLE on NaN or Inf.
Both failure cases are forced from the host (a NaN in the load table, a
step size above the explicit stability limit of Eq. CDMstep); every kernel
still runs to its normal end."""
import numpy as np
import pytest

from paper_2310_14712_amd import inputs

pytestmark = pytest.mark.gpu

UNSTABLE = -5


def _imex():
    from paper_2310_14712_amd import imex
    return imex


def _case():
    return inputs.small_2d(n=(7, 5), p=3, holes=((0.55, 0.45, 0.23),), depth=2, source=(0.05, 0.3))


def _run(w, n_steps, check, dt=0.0, ft=None):
    imex = _imex()
    lib = imex.Imex(w, dt=dt)
    lib.assemble()
    if check:
        lib.set_check_finite(True)
    if ft is None:
        ft = inputs.ft_table(lib.info()["dt"], n_steps, w.source_freq)
    lib.set_initial(None, None, ft[0])
    return lib, ft


def test_check_leaves_a_stable_run_unchanged():
    w = _case()
    print("\n[case] finite check on a stable run", flush=True)
    a, ft = _run(w, 40, check=True)
    a.step(ft[:41])
    b, _ = _run(w, 40, check=False, ft=ft)
    b.step(ft[:41])
    imex = _imex()
    assert np.array_equal(a.read(imex.FIELD_U), b.read(imex.FIELD_U))
    assert np.linalg.norm(a.read(imex.FIELD_U)) > 0


def test_nonfinite_load_is_reported():
    w = _case()
    print("\n[case] NaN in the load table", flush=True)
    lib, ft = _run(w, 20, check=True)
    lib.step(ft[:6])                       # finite so far
    bad = ft.copy()
    bad[8] = np.nan
    with pytest.raises(_imex().ImexError) as err:
        lib.step(bad[5:21])
    assert err.value.status == UNSTABLE
    assert "after step 20" in str(err.value)


def test_unstable_step_size_is_reported():
    """Twice the explicit critical step of an uncut cell: the highest uncut
    mode grows by a factor of about 14 per step and overflows within a few
    hundred steps."""
    w = _case()
    imex = _imex()
    probe = imex.Imex(w, device_mode=imex.HOST_ONLY)
    dt = 2.0 * probe.info()["dt_crit_uncut"]
    probe.close()
    print(f"\n[case] unstable dt = {dt:.3e}", flush=True)
    lib, ft = _run(w, 800, check=True, dt=dt)
    with pytest.raises(imex.ImexError) as err:
        lib.step(ft)
    assert err.value.status == UNSTABLE
    # the same run without the check completes and leaves a non-finite state
    quiet, _ = _run(w, 800, check=False, dt=dt, ft=ft)
    quiet.step(ft)
    assert not np.all(np.isfinite(quiet.read(imex.FIELD_U)))
