"""The C-ABI library loads and exports every function include/slosh.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slosh.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+((?:sph|mlp|lpv)_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("sph_init", "sph_step", "sph_slosh_wrench", "sph_rollout", "mlp_forward",
                 "mlp_train_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2604_12505_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libslosh.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layout_matches_header():
    """sph_params: 4 int32, 16 doubles, 2 int32, 2 doubles, 4 doubles."""
    from paper_2604_12505_amd._lib import SphParams
    assert ctypes.sizeof(SphParams) == 4 * 4 + 16 * 8 + 2 * 4 + 2 * 8 + 4 * 8


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2604_12505_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.LibraryMissing):
        _lib.load()
