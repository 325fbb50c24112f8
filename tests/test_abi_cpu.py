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
               "ccd_serve_stats": ccd.ServeStats, "ccd_scratch_plan": ccd.ScratchPlan}
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


def test_scratch_plan_sizes_are_overflow_safe(lib):
    """The scratch plan (host-only) stays inside the budget for any m_I: the
    block engine's arena is 2 m_I + 2 words per buffer clamped to a quarter of
    the budget, computed without wrapping at m_I = 1e18 or INT64_MAX."""
    from paper_2009_13349_amd import ccd
    budget = 32 << 30
    small = ccd.plan_scratch(1_000_000, 1_000_000, mem_budget_bytes=budget)
    assert small["block_capacity"] == 2 * 1_000_000 + 2
    assert small["bytes"] <= budget
    for mi in (10 ** 18, 2 ** 63 - 1, 2 ** 62, 190_000_000_000_000_000):
        p = ccd.plan_scratch(1_000_000, mi, mem_budget_bytes=budget)
        assert p["bytes"] <= budget, (mi, p)
        assert p["block_capacity"] * 48 <= budget // 4 + 48
        assert p["block_capacity"] >= p["group_capacity"] >= 256
        assert p["block_count"] >= 1 and p["group_count"] >= 1
    # the plan stays inside the budget at every batch size up to the largest
    # it admits (one arena of each engine first, then the pool and the rest)
    for b in (256 << 20, 1 << 30, 32 << 30):
        for n in (1, 1000, 100_000, 900_000, 963_000, 4_000_000, 100_000_000):
            try:
                p = ccd.plan_scratch(n, 10 ** 6, mem_budget_bytes=b)
            except ccd.CCDError as e:
                assert e.code == ccd.ENOMEM
                continue
            assert p["bytes"] <= b, (b, n, p)
    # the hand-off pool takes what the engines' arenas leave, up to handoff_words
    big = ccd.plan_scratch(1_000_000, 10 ** 6, mem_budget_bytes=160 << 30)
    assert big["handoff_words"] == 1 << 33 and big["group_count"] == 3072 and big["block_count"] == 512
    for b in (16 << 30, 32 << 30):
        p = ccd.plan_scratch(1_000_000, 10 ** 6, mem_budget_bytes=b)
        assert b - 8 * 48 * max(p["group_capacity"], p["block_capacity"]) < p["bytes"] <= b
        assert p["handoff_words"] * 8 >= b // 16
    capped = ccd.plan_scratch(1_000_000, 10 ** 6, mem_budget_bytes=160 << 30, handoff_words=1 << 20)
    assert capped["handoff_words"] == 1 << 20 and capped["bytes"] < big["bytes"]
    # a tuning can shrink the block arena (never below a group arena)
    p = ccd.plan_scratch(1000, 10 ** 6, mem_budget_bytes=budget, group_capacity=256,
                         block_capacity=300)
    assert p["block_capacity"] == 300 and p["group_capacity"] == 256
    p = ccd.plan_scratch(1000, 10 ** 6, mem_budget_bytes=budget, group_capacity=4096,
                         block_capacity=300)
    assert p["block_capacity"] == 4096
    # LDS frontier of the lane engine: two buffers of lane_capacity keys per thread
    p = ccd.plan_scratch(1000, 100, lane_capacity=16)
    assert p["lane_lds_bytes"] == 2 * 16 * 128 * 8
    assert ccd.plan_scratch(1000, 100, lane_capacity=1000)["lane_lds_bytes"] == 2 * 32 * 128 * 8
    # too small a budget, and bad arguments
    with pytest.raises(ccd.CCDError) as e:
        ccd.plan_scratch(10 ** 9, 100, mem_budget_bytes=1 << 20)
    assert e.value.code == ccd.ENOMEM
    for bad in ((-1, 10), (10, 0)):
        with pytest.raises(ccd.CCDError) as e:
            ccd.plan_scratch(*bad)
        assert e.value.code == ccd.EINVAL
