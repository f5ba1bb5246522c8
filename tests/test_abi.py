"""The C-ABI library loads, exports every function include/gsc.h declares, and the Python
struct layouts match the C ones (CPU only; no device call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gsc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2507_19718_amd import _abi
    lib = ctypes.CDLL(_abi.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.exported_symbols())


def test_struct_layouts_match():
    from paper_2507_19718_amd import _abi
    lib = _abi.load()
    for i, st in enumerate(_abi.STRUCTS):
        assert lib.gsc_abi_struct_size(i) == ctypes.sizeof(st), st.__name__
    assert ctypes.sizeof(_abi.gsc_path_record) == 20


def test_public_entry_points_named_after_the_path():
    names = declared_functions()
    for n in ("gsc_trace_targets", "gsc_project_bin", "gsc_splat_forward", "gsc_splat_backward",
              "gsc_adam_step", "gsc_render_frame"):
        assert n in names


def test_package_import_has_no_cpu_fallback():
    import paper_2507_19718_amd as gsc
    src = open(gsc.__file__).read()
    assert "import oracle" not in src and "from oracle" not in src
