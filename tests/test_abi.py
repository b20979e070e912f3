"""The C ABI library loads on a CPU-only host and exports every symbol include/sps*.h
declares; argument validation that happens before any device call returns error codes."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import paper_2609_30145_amd as pkg
from paper_2609_30145_amd import sps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(sps_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    names = declared_symbols()
    assert {"sps_library_load", "sps_forward", "sps_logl", "sps_logl_grad", "sps_obs_create"} <= names
    for n in sorted(names):
        assert hasattr(L, n), f"{n} declared but not exported"


def test_version_and_error_strings():
    L = pkg.lib()
    assert L.sps_version().startswith(b"sps-gfx950")


def test_library_load_rejects_bad_arguments_before_touching_a_device():
    L = pkg.lib()
    h = C.c_void_p()
    assert L.sps_library_load(None, C.byref(h)) == -1
    d = sps.LibraryDesc()
    d.n_age, d.n_z, d.n_afe, d.n_wave = 3, 1, 1, 4
    ages = np.array([1e6, 5e5, 1e8])            # not increasing
    logz = np.array([0.0])
    wave = np.array([1000.0, 2000.0, 3000.0, 4000.0])
    flux = np.ones((1, 1, 3, 4))
    d.ages, d.logz, d.wave, d.flux = (a.ctypes.data_as(C.POINTER(C.c_double)) for a in (ages, logz, wave, flux))
    d.t_young, d.n_sfh, d.T1, d.H0, d.Om = 1e7, 4, 1e7, 70.0, 0.3
    assert L.sps_library_load(C.byref(d), C.byref(h)) == -1
    assert b"ages" in L.sps_last_error()
    ages[:] = [1e6, 5e6, 1e8]
    flux[0, 0, 1, 2] = -1.0                      # negative flux
    assert L.sps_library_load(C.byref(d), C.byref(h)) == -1
    flux[0, 0, 1, 2] = 1.0
    d.n_sfh = 1                                  # too few SFH bins
    assert L.sps_library_load(C.byref(d), C.byref(h)) == -2
    d.n_sfh = 4
    d.Om = 1.5
    assert L.sps_library_load(C.byref(d), C.byref(h)) == -1
    assert not h.value


def _header_struct_fields(name):
    """Field names of ``typedef struct { ... } name;`` in include/sps.h, in order."""
    text = open(os.path.join(ROOT, "include", "sps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    out = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"^(const\s+)?\w+\s*", "", decl)       # drop the type
        for part in decl.split(","):
            out.append(part.strip().lstrip("*").strip())
    return out


@pytest.mark.parametrize("cname,pyname", [("sps_library_desc", "LibraryDesc"), ("sps_layout", "Layout"),
                                          ("sps_library_info", "LibraryInfo"), ("sps_obs_desc", "ObsDesc")])
def test_struct_layouts_match_header_field_order(cname, pyname):
    # the ctypes mirrors list the header's fields, in the header's order
    fields = [n for n, _ in getattr(sps, pyname)._fields_]
    assert fields == _header_struct_fields(cname)
    assert C.sizeof(sps.LibraryInfo) == 7 * 4 + 4 + 8


def test_binding_requires_built_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sps, "_lib", None)
    monkeypatch.setattr(sps, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        sps.lib()
