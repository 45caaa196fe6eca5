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
    for n, sp, cap in [((1, 8, 8), 1.0, 10), ((8, 8, 2000), 1.0, 10), ((8, 1025, 8), 1.0, 10), ((8, 8, 8), 0.0, 10),
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


def _header_constants():
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for body in re.findall(r"enum(?:\s+\w+)?\s*\{([^}]*)\}", txt):
        for name, expr in re.findall(r"(BTO_[A-Z0-9_]+)\s*=\s*([^,]+)", body):
            parts = [int(v) for v in expr.split("<<")]  # integer literals, optionally one shift
            vals[name] = parts[0] << parts[1] if len(parts) == 2 else parts[0]
    return vals


def _header_struct_fields(name):
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + r"\s*;", txt).group(1)
    return re.findall(r"\b(int32_t|int64_t|double)\s+([a-z_0-9]+)(?:\[(\d+)\])?\s*;", body)


def test_python_binding_mirrors_the_header():
    """Every constant and struct the binding marshals has the header's value
    and field layout (names, types, order)."""
    from paper_2004_02003_amd import _lib

    consts = _header_constants()
    for name in ("BTO_OK", "BTO_EINVAL", "BTO_ENOMEM", "BTO_EHIP", "BTO_ESTATE", "BTO_ERANGE", "BTO_F32",
                 "BTO_F16", "BTO_BF16", "BTO_TIME_LINEAR", "BTO_TIME_FROZEN", "BTO_RECORD_EXIT", "BTO_RECORD_CKPT",
                 "BTO_SAMPLE_FP64",
                 "BTO_VALID", "BTO_TERMINATED", "BTO_INVALID", "BTO_ADJ_DROPPED", "BTO_ADJ_DROPPED_PARTIAL"):
        assert getattr(_lib, name) == consts[name], name
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
    for cname, py in (("bto_tuning", _lib.Tuning), ("bto_block", _lib.Block), ("bto_stats_t", _lib.Stats)):
        want = [(f, ctype[t] * int(n) if n else ctype[t]) for t, f, n in _header_struct_fields(cname)]
        got = list(py._fields_)
        assert [f for f, _ in got] == [f for f, _ in want], cname
        for (f, a), (_, b) in zip(got, want):
            assert ctypes.sizeof(a) == ctypes.sizeof(b) and getattr(a, "_type_", a) == getattr(b, "_type_", b), (cname, f)
