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


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the size and field offsets of the C structs: a C
    program compiled against include/ccd.h prints them."""
    from paper_2009_13349_amd import ccd
    mirrors = {"ccd_params": ccd.Params, "ccd_result": ccd.Result, "ccd_tuning": ccd.Tuning,
               "ccd_batch_desc": ccd.BatchDesc, "ccd_result_soa": ccd.ResultSoA,
               "ccd_stats": ccd.Stats, "ccd_indexed_desc": ccd.IndexedDesc,
               "ccd_serve_config": ccd.ServeConfig, "ccd_serve_info": ccd.ServeInfo,
               "ccd_serve_stats": ccd.ServeStats}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "ccd.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
    assert ctypes.sizeof(ccd.IndexedDesc) == 112 and ctypes.sizeof(ccd.BatchDesc) == 104


def test_null_arguments_rejected_without_gpu(lib):
    from paper_2009_13349_amd import ccd
    assert lib.ccd_batch(None, None, None, None) == ccd.EINVAL
    assert lib.ccd_context_set_engine(None, 0) == ccd.EINVAL
    assert lib.ccd_vf(None, None, None, None) == ccd.EINVAL
