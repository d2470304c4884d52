"""The C ABI library loads on a machine without a GPU and exports every
function declared in include/scvt.h; argument validation runs on the host.
No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scvt.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scvt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("scvt_create", "scvt_step", "scvt_solve", "scvt_energy", "scvt_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1709_06924_amd import scvt
    lib = ctypes.CDLL(scvt.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", scvt.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (scvt_[a-z_]+)", out))
    assert set(declared()) <= exported
    assert set(scvt.exported_symbols()) <= exported


def test_calibration_library_exports_its_header():
    from paper_1709_06924_amd import build
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "scvt_calib.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(scvt_[a-z_]+)\s*\(", text)))
    assert names == ["scvt_calib_count", "scvt_calib_math", "scvt_calib_valu"]
    lib = ctypes.CDLL(build.CALIB_LIB)
    for name in names:
        assert hasattr(lib, name), name
    assert lib.scvt_calib_count() == 14  # no device work


def test_config_defaults_and_validation_on_host():
    from paper_1709_06924_amd import scvt
    c = scvt.make_config(10)
    assert c.m_hist == 7 and c.quad_levels == 2 and c.ls_max_evals == 10
    assert abs(c.ls_c1 - 1e-4) < 1e-18 and c.precision == scvt.FP64
    # invalid configurations are rejected before any device work
    import numpy as np
    z = np.ones((3, 3))
    with pytest.raises(scvt.ScvtError) as e:
        scvt.Solver(z)  # n < 4
    assert e.value.code == -1
    z = np.ones((8, 3))
    with pytest.raises(scvt.ScvtError) as e:
        scvt.Solver(z, quad_levels=7)
    assert e.value.code == -1
    z[2] = np.nan
    with pytest.raises(scvt.ScvtError) as e:
        scvt.Solver(z)
    assert e.value.code == -1
    z[2] = 0.0
    with pytest.raises(scvt.ScvtError) as e:
        scvt.Solver(z)
    assert e.value.code == -3
    assert scvt._lib.scvt_strerror(-4).decode().startswith("a Voronoi cell")
