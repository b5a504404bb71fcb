"""The library's host-side setup (classification, space-tree integration,
assembly, the dissected factor (2D) and the nested-dissection factor with
its host solve (3D), the global critical step and receiver weights) built on its own with the address and undefined-behaviour
sanitizers and run on a ragged 2D and a 3D mesh with holes: it must finish
without a report, and its counts must equal those of a library context on
the same meshes."""
import shutil
import subprocess
from pathlib import Path

import pytest

from paper_2310_14712_amd import inputs

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2310_14712_amd" / "csrc"
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = tmp_path_factory.mktemp("san") / "imex_host_san"
    cmd = [gxx, "-std=c++17", "-O1", "-g", *SANITIZE, f"-I{CSRC}", str(ROOT / "tests/host_sanitize/driver.cpp"),
           str(CSRC / "setup.cpp"), str(CSRC / "nd_factor.cpp"), str(CSRC / "basis.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return exe


def _parse(line):
    tok = line.split()
    return {tok[i]: tok[i + 1] for i in range(0, len(tok), 2)}


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_host_setup_clean_under_sanitizers(driver, case):
    from paper_2310_14712_amd import imex
    run = subprocess.run([str(driver), case], capture_output=True, text=True, timeout=600,
                         env={"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr[-4000:]
    got = _parse(run.stdout.strip())
    if case == "2d":
        w = inputs.small_2d(n=(7, 5), p=2, holes=((0.55, 0.45, 0.23), (0.2, 0.8, 0.12)), depth=2,
                            source=(0.05, 0.3))
    else:
        w = inputs.small_3d(n=(5, 3, 4), p=3, holes=((0.5, 0.45, 0.55, 0.3), (0.1, 0.9, 0.1, 0.25)), depth=1)
    lib = imex.Imex(w, device_mode=imex.HOST_ONLY)
    lib.assemble()
    inf = lib.info()
    for key in ("n_grid", "n_d", "n_c", "nnz_kc", "nnz_factor"):
        assert int(got[key]) == inf[key], (key, got[key], inf[key])
    assert int(got["components"]) == inf["n_components"]
    assert int(got["nd"]) == inf["factor_form"] == (1 if case == "3d" else 0)
    if case == "3d":
        assert float(got["nd_relres"]) <= 1e-10
    dt = lib.global_critical_step(300, 1e-8)
    assert abs(float(got["dt_global"]) - dt) <= 1e-6 * dt
