"""The C-ABI library loads and exports every entry point declared in include/pdf.h
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1006_0532_amd import pdfgpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "pdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("pdf_grid_create", "pdf_particles_init", "pdf_step", "pdf_stats", "pdf_control"):
        assert n in names
    assert sorted(pdfgpu.EXPORTS) == names


@pytest.mark.skipif(not os.path.exists(pdfgpu.LIB_PATH), reason="libpdfgpu.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pdfgpu.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    L = pdfgpu.load()
    assert isinstance(L.pdf_last_error(), bytes)   # the last error message of this thread


@pytest.mark.skipif(not os.path.exists(pdfgpu.LIB_PATH), reason="libpdfgpu.so not built")
def test_host_side_argument_errors():
    """Argument checks run before any device call."""
    L = pdfgpu.load()
    h = ctypes.c_void_p()
    assert L.pdf_grid_create(None, None, None, None, ctypes.byref(h)) == -1
    assert b"null" in L.pdf_last_error()
    assert L.pdf_step(None, None, 1, None) == -1
    assert L.pdf_stats(None, 0, pdfgpu.PDF_STATS_ALL, None, 0, None) == -1
    assert L.pdf_control(None, 5, 1, None, None) == -1
    assert L.pdf_sync(None) == -1


@pytest.mark.skipif(not os.path.exists(pdfgpu.LIB_PATH), reason="libpdfgpu.so not built")
def test_option_and_tuning_argument_errors():
    L = pdfgpu.load()
    o = pdfgpu.Options(0, 256, 4)
    assert L.pdf_set_options(None, ctypes.byref(o)) == -1
    assert L.pdf_get_options(None, ctypes.byref(o)) == -1
    assert L.pdf_autotune(None, None, 1, None, None, None, None) == -1
    assert L.pdf_particles_init(None, None, 0, None, None) == -1
    moves = ctypes.c_int64(7)
    assert L.pdf_redistribute(None, -1, 3, ctypes.byref(moves), None) == -1
    assert moves.value == 0
    it = ctypes.c_int32(5)
    assert L.pdf_elliptic_relaxation(None, None, 1e-10, 100, 0, None, 0, ctypes.byref(it), None) == -1
    assert it.value == 0
    assert L.pdf_pressure_projection(None, 1e-3, 1e-3, 1e-10, 100, None, 0, None, None) == -1
