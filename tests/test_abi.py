"""The C-ABI library loads on a host without a GPU and exports what include/mot.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mot.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mot_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mot_create", "mot_set_lag", "mot_step", "mot_run", "mot_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2510_07989_amd import _lib
    lib = _lib.load()
    for name in _declared():
        getattr(lib, name)          # raises AttributeError when missing
    assert sorted(_lib.EXPORTS) == sorted(_declared())


def test_default_options_without_gpu():
    import paper_2510_07989_amd as p
    o = p.default_options()
    assert o.gmres_tol == 1e-13 and o.gmres_restart == 40 and o.keep_history == 1
