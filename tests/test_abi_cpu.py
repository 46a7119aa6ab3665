"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function include/rsc.h declares, reject bad
arguments before touching a device, and build the same FP64 basis as the
reference (the two constructions share no code).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import rsc


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rsc.LIB_PATH):
        from paper_1806_04374_amd import build_lib
        build_lib.build()
    return rsc.lib()


def test_exports_every_declared_function(L):
    names = rsc.header_functions()
    assert "rsc_project" in names and "rsc_omp_encode" in names and "rsc_reconstruct" in names
    out = subprocess.run(["nm", "-D", "--defined-only", rsc.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in names:
        assert n in exported, n
        assert getattr(L, n) is not None


# the calls of the boundary: handle and basis, dictionary upload, projection (patch arrays
# and images), the encoder with its workspace query, reconstruction, and the stream wait
# with the error text
BOUNDARY = ["rsc_create", "rsc_destroy", "rsc_basis_info", "rsc_get_basis", "rsc_set_dictionary",
            "rsc_project", "rsc_project_images", "rsc_encode_workspace_size", "rsc_omp_encode",
            "rsc_reconstruct", "rsc_sync", "rsc_last_error"]


def test_boundary_calls_are_declared_and_exported(L):
    names = set(rsc.header_functions())
    for n in BOUNDARY:
        assert n in names, n
        assert getattr(L, n) is not None


def test_boundary_state_without_device(L):
    """Argument errors come back synchronously and name the problem; the workspace query,
    the fault setter and the stream wait validate their handle before any device use."""
    n = ctypes.c_size_t(77)
    assert L.rsc_encode_workspace_size(None, 10, 2, ctypes.byref(n)) == rsc.RSC_E_INVALID
    assert b"handle" in L.rsc_last_error(None)
    assert n.value == 77                                   # untouched on error
    assert L.rsc_set_fault(None, b"x") == rsc.RSC_E_INVALID
    assert L.rsc_set_dictionary(None, None, 4, 8, None) == rsc.RSC_E_INVALID
    assert b"handle is NULL" in L.rsc_last_error(None)
    # a later successful call clears the thread's message
    assert L.rsc_destroy(None) == rsc.RSC_OK
    assert L.rsc_last_error(None) == b""


def test_header_documents_every_function():
    import re
    text = open(rsc.HEADER).read()
    for n in rsc.header_functions():
        m = re.search(r"(rsc_status|const char\*)\s+" + n + r"\(", text)
        assert m, n
        assert text[:m.start()].rstrip().endswith("*/"), n


@pytest.mark.parametrize("geom", [(11, 5, 5), (15, 7, 7), (13, 3, 4)])
def test_library_basis_matches_reference(L, geom):
    N, S, T = geom
    phi, pinv, cond = rsc.rsc_basis_host(N, S, T)
    ref = orc.build_basis(N, S, T)
    mask = ref.mask.ravel()
    assert np.abs(phi[mask] - ref.phi).max() < 1e-12
    assert np.abs(phi[~mask]).max() == 0.0
    assert np.abs(pinv[:, mask] - ref.pinv).max() < 1e-10 * np.abs(ref.pinv).max()
    assert np.abs(pinv[:, ~mask]).max() == 0.0
    assert abs(cond - np.linalg.cond(ref.phi.T @ ref.phi)) < 1e-6 * cond


def test_library_basis_custom_profiles(L):
    centres = [0.7, 1.9, 3.1, 4.0, 5.2]
    phi, pinv, _ = rsc.rsc_basis_host(11, 5, 5, centres, 1.3)
    ref = orc.build_basis(11, 5, 5, centres, 1.3)
    assert np.abs(phi[ref.mask.ravel()] - ref.phi).max() < 1e-12


def test_argument_errors_without_device(L):
    h = ctypes.c_void_p()
    assert L.rsc_create(10, 5, 5, None, 0.0, 0, ctypes.byref(h)) == rsc.RSC_E_INVALID
    assert b"odd" in L.rsc_last_error(None)
    assert L.rsc_create(15, 7, 9, None, 0.0, 0, ctypes.byref(h)) == rsc.RSC_E_UNSUPPORTED   # B = 133
    assert L.rsc_create(31, 1, 16, None, 0.0, 0, ctypes.byref(h)) == rsc.RSC_E_UNSUPPORTED   # T > 15
    assert L.rsc_create(11, 5, 2, None, 0.0, 1, ctypes.byref(h)) == rsc.RSC_E_UNSUPPORTED    # 16-bit
    assert L.rsc_create(11, 5, 5, None, 0.0, 0, None) == rsc.RSC_E_INVALID
    assert L.rsc_create(11, 5, 5, None, 0.0, 7, ctypes.byref(h)) == rsc.RSC_E_INVALID
    assert L.rsc_precision_stats(None, None, 0) == rsc.RSC_E_INVALID
    assert L.rsc_set_dictionary(None, None, 4, 8, None) == rsc.RSC_E_INVALID
    assert L.rsc_project(None, None, 10, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_omp_encode(None, None, 10, 2, None, 0, None, None, None, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_reconstruct(None, None, None, None, 10, 2, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_synthesize(None, None, None, None, 10, 2, None, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_destroy(None) == rsc.RSC_OK
    assert L.rsc_basis_host(4, 5, 5, None, 0.0, None, None, None, None, None) == rsc.RSC_E_INVALID
    # more basis columns than disk pixels
    assert L.rsc_basis_host(5, 5, 5, None, 0.0, None, None, None, None, None) == rsc.RSC_E_INVALID
    assert b"more columns" in L.rsc_last_error(None)


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(rsc, "_lib", None)
    monkeypatch.setattr(rsc, "LIB_PATH", "/nonexistent/librsc.so")
    with pytest.raises(RuntimeError, match="missing"):
        rsc.lib()
