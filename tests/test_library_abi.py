"""CPU checks of the C-ABI library: it loads, exports every function the
public header declares, and rejects bad arguments before touching a device.
No kernel is launched here."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bto.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bto_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2004_02003_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libbto.so not built")
    return _lib.load()


def test_header_declares_the_path_entry_points():
    names = _declared()
    for fn in ("bto_create", "bto_destroy", "bto_last_error", "bto_seed", "bto_seed_explicit",
               "bto_advect_interval", "bto_flowmap_out", "bto_stats", "bto_adjoint_interval", "bto_ftle",
               "bto_set_tuning", "bto_get_tuning"):
        assert fn in names, fn


def test_library_exports_every_declared_symbol(lib):
    from paper_2004_02003_amd import _lib

    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(bto_[a-z_]+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(lib, n)


def test_create_rejects_bad_blocks_before_touching_a_device(lib):
    from paper_2004_02003_amd import _lib

    h = ctypes.c_void_p()
    for n, sp, cap in [((1, 8, 8), 1.0, 10), ((8, 8, 2000), 1.0, 10), ((8, 8, 8), 0.0, 10),
                       ((8, 8, 8), float("nan"), 10), ((8, 8, 8), 1.0, 0)]:
        blk = _lib.Block()
        blk.n[:] = n
        blk.spacing[:] = [sp] * 3
        assert lib.bto_create(ctypes.byref(blk), cap, 0, ctypes.byref(h)) == _lib.BTO_EINVAL
    assert lib.bto_create(None, 10, 0, ctypes.byref(h)) == _lib.BTO_EINVAL
    assert lib.bto_destroy(None) == _lib.BTO_EINVAL
    assert lib.bto_last_error(None) == b"null context"
    for fn, args in [("bto_seed", (None, 2, None, None, None)),
                     ("bto_advect_interval", (None, None, None, 1, 0, 0, None)),
                     ("bto_flowmap_out", (None, None, None, None, None, None, None)),
                     ("bto_stats", (None, None, None)), ("bto_exit_points", (None, None, None)),
                     ("bto_set_tuning", (None, None)), ("bto_get_tuning", (None, None)),
                     ("bto_adjoint_interval", (None, None, None, 1, 0, 0, None, 1, None, None, None, 1, None)),
                     ("bto_ftle", (None, None, 0, 1.0, None, None))]:
        assert getattr(lib, fn)(*args) == _lib.BTO_EINVAL, fn


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2004_02003_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, flags=re.M), f
                assert "bto_oracle" not in txt and "liboracle" not in txt, f
