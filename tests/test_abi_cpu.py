"""CPU-side checks of the C ABI: the HIP library builds for gfx950, loads, and
exports every function declared in include/ccd.h; host-only entry points work
without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccd.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2009_13349_amd import ccd
    if not os.path.exists(ccd.LIB_PATH):
        from paper_2009_13349_amd import build
        build.build()
    return ccd.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+[\s\*]+(ccd_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ccd_vf", "ccd_ee", "ccd_batch", "ccd_context_create", "ccd_strerror"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2009_13349_amd import ccd
    out = subprocess.run(["nm", "-D", "--defined-only", ccd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in declared_functions():
        assert hasattr(lib, n)
    assert set(ccd.EXPORTED) <= set(declared_functions())


def test_gfx950_code_object_present():
    from paper_2009_13349_amd import ccd
    data = open(ccd.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_host_only_entry_points(lib):
    from paper_2009_13349_amd import ccd
    assert lib.ccd_strerror(0) == b"ok"
    assert lib.ccd_strerror(-1) == b"invalid argument"
    p = ccd.Params()
    lib.ccd_params_default(ctypes.byref(p))
    assert (p.delta, p.max_iter, p.min_sep, p.t_max, p.flags) == (1e-6, 1_000_000, 0.0, 1.0, 0)


def test_struct_layouts_match_header():
    from paper_2009_13349_amd import ccd
    assert ctypes.sizeof(ccd.Params) == 40
    assert ctypes.sizeof(ccd.Result) == 32
    assert ctypes.sizeof(ccd.Tuning) == 40
    assert ctypes.sizeof(ccd.BatchDesc) == 104
    assert ctypes.sizeof(ccd.ResultSoA) == 40
    assert ctypes.sizeof(ccd.Stats) == 104


def test_null_arguments_rejected_without_gpu(lib):
    from paper_2009_13349_amd import ccd
    assert lib.ccd_batch(None, None, None, None) == ccd.EINVAL
    assert lib.ccd_context_set_engine(None, 0) == ccd.EINVAL
    assert lib.ccd_vf(None, None, None, None) == ccd.EINVAL
