"""CPU-side checks of the C ABI: the built library loads and exports every
function that include/sem.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z_0-9]+)\s*\(", src)))


def _lib_path():
    from paper_1110_2316_amd.semlib import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1110_2316_amd.build import build
        build()
    return LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sem_setup", "sem_residual", "sem_precond", "sem_pcg_solve", "sem_error", "sem_rhs"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1110_2316_amd.semlib import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_setup_rejects_bad_mesh_without_gpu_work():
    """Argument validation happens on the host before any device call."""
    from paper_1110_2316_amd import semlib
    lib = semlib.lib()
    h = ctypes.c_void_p()
    st = lib.sem_setup(None, None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"NULL" in lib.sem_last_error() or b"null" in lib.sem_last_error()
