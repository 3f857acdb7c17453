"""The C-ABI library loads on any host and exports every entry point that
include/hyperflow.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperflow.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(
        r"^(?:fp_status|void|int32_t|const char\s*\*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_01556_amd import hyperflow
    return hyperflow.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("flow_problem_create", "maxflow_solve", "mincut_source_side",
                 "flow_batch_solve", "flow_problem_pierce", "flow_problem_destroy",
                 "fp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2201_01556_amd import hyperflow
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in hyperflow.EXPORTED, name
    out = subprocess.run(["nm", "-D", "--defined-only", hyperflow.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    # nothing but the C ABI leaves the library
    assert exported == set(_declared()), exported ^ set(_declared())


def test_last_error_is_empty_string_initially(lib):
    assert lib.fp_last_error() in (b"",)


def test_missing_library_fails_loudly(tmp_path):
    from paper_2201_01556_amd import hyperflow
    saved = hyperflow._lib
    hyperflow._lib = None
    try:
        with pytest.raises(RuntimeError, match="missing"):
            hyperflow.load_library(str(tmp_path / "nope.so"))
    finally:
        hyperflow._lib = saved


def test_options_struct_matches_header():
    from paper_2201_01556_amd import hyperflow
    assert ctypes.sizeof(hyperflow.Options) == 17 * 4
    assert ctypes.sizeof(hyperflow.Stats) == 16 * 8


def test_binding_struct_layouts_match_the_header(tmp_path):
    """Every field of every struct the binding mirrors sits at the offset and
    has the size the C compiler gives it from the header."""
    from paper_2201_01556_amd import hyperflow
    structs = {"fp_options": hyperflow.Options, "fp_stats": hyperflow.Stats,
               "fp_batch_config": hyperflow.BatchConfig,
               "fp_cutter_result": hyperflow.CutterResult,
               "fp_cutter_step": hyperflow.CutterStep,
               "fp_refine_config": hyperflow.RefineConfig,
               "fp_refine_result": hyperflow.RefineResult}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hyperflow.h"',
             "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu %zu\\n", offsetof({cname}, {fname}), '
                         f'sizeof((({cname}*)0)->{fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        parts = line.split()
        got[(parts[0], parts[1])] = tuple(int(x) for x in parts[2:])
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == (ctypes.sizeof(cls),), cname
        for fname, _ in cls._fields_:
            f = getattr(cls, fname)
            assert got[(cname, fname)] == (f.offset, f.size), (cname, fname)
