"""C ABI surface checks that need no GPU: the library loads, exports every
entry point the header declares, the binding wraps exactly those, and the
host-side geometry validation accepts/rejects what the header says."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1706_07075_amd import lmtof as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmtof.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*\**(lmtof_\w+)\(", txt, re.M)))


def test_header_declares_entry_points():
    names = declared()
    for must in ["lmtof_create", "lmtof_destroy", "lmtof_set_geometry", "lmtof_load_events",
                 "lmtof_compute_sensitivity", "lmtof_set_image", "lmtof_iterate", "lmtof_read_image",
                 "lmtof_forward_project", "lmtof_back_project", "lmtof_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(set(re.findall(r" T (lmtof_\w+)", out)))
    assert exported == declared()


def test_binding_wraps_exactly_the_header():
    assert L.exported_symbols() == declared()
    for n in declared():
        assert callable(getattr(L, n)), n


def _geom(**kw):
    g = dict(nx=64, ny=64, nz=64, vx=4.0, vy=4.0, vz=4.0, x0=-128.0, y0=-128.0, z0=-128.0,
             scanner_radius=400.0, scanner_half_length=128.0, max_axial_angle_deg=0.0, tof_fwhm_ps=300.0)
    g.update(kw)
    return g


def test_geometry_validation_host_only():
    assert L.lmtof_check_geometry(_geom()) == ""
    assert L.lmtof_check_geometry(_geom(nx=0)) != ""
    assert L.lmtof_check_geometry(_geom(vx=-1.0)) != ""
    assert L.lmtof_check_geometry(_geom(vz=float("nan"))) != ""
    assert "radius" in L.lmtof_check_geometry(_geom(scanner_radius=150.0))
    assert "z range" in L.lmtof_check_geometry(_geom(scanner_half_length=100.0))
    assert L.lmtof_check_geometry(_geom(max_axial_angle_deg=95.0)) != ""
    assert L.lmtof_check_geometry(_geom(tof_trunc_sigmas=-1.0)) != ""
    assert L.lmtof_check_geometry(_geom(tof_fwhm_ps=0.0)) == ""      # non-TOF is valid
    # whole-body geometry: grid corners at 424 mm inside R = 450, |z| = H
    wb = _geom(nx=150, ny=150, nz=600, x0=-300.0, y0=-300.0, z0=-1200.0, scanner_radius=450.0,
               scanner_half_length=1200.0, max_axial_angle_deg=45.0)
    assert L.lmtof_check_geometry(wb) == ""


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device error path")
def test_create_without_device_reports_error():
    with pytest.raises(L.LmtofError) as e:
        L.lmtof_create(0)
    assert e.value.code in (L.LMTOF_EHIP, L.LMTOF_EINVAL)
    assert e.value.msg
