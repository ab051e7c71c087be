"""The C-ABI library: it loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aboria.h")
LIB = os.path.join(ROOT, "paper_1704_08907_amd", "libaboria_mi355x.so")
CSRC = os.path.join(ROOT, "paper_1704_08907_amd", "csrc")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:aboria_status|const char\*|int32_t)\s+(aboria_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("aboria_build_cells", "aboria_pair_sum", "aboria_pair_sum_backward", "aboria_dense_sum"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1704_08907_amd import _native
    assert sorted(_native.EXPORTS) == declared()


def test_static_queries_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_1704_08907_amd import _native as N
    assert N.op_ny("spring", 3) == 3 and N.op_ny("soft_sphere", 3) == 1 and N.op_na("dem_spring") == 1
    assert N.lib().aboria_op_ny(99, 3) == -1 and N.lib().aboria_op_ny(1, 4) == -1
    assert N.variant_count() >= 1 and N.variant_name(0)


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's ctypes structures against the header, compiled by the host C compiler
    import shutil
    import subprocess
    from paper_1704_08907_amd import _native as N
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"aboria_box": N.Box, "aboria_cells_view": N.CellsView}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "aboria.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_box_reach_per_dimension_marshalling():
    from paper_1704_08907_amd import _native as N
    b = N.BoxSpec(3, [0] * 3, [1] * 3, [1] * 3, 0.1, None, 2).to_c()
    assert list(b.reach) == [2, 2, 2]
    b = N.BoxSpec(3, [0] * 3, [1] * 3, [1] * 3, 0.1, None, [3, 1, 1]).to_c()
    assert list(b.reach) == [3, 1, 1]
    b = N.BoxSpec(2, [0] * 2, [1] * 2, [1] * 2, 0.1).to_c()
    assert list(b.reach) == [0, 0, 0]  # 0 = reach 1 in the library
    with pytest.raises(ValueError):
        N.BoxSpec(3, [0] * 3, [1] * 3, [1] * 3, 0.1, None, [2, 1]).to_c()


def test_build_generation_never_takes_a_reserved_value(tmp_path):
    # the device's build counter (csrc/generation.hpp) skips 0 (mask status "no
    # record") and 0xFFFFFFFF (list "never recorded") when it wraps, so neither
    # a missing record nor an unrecorded list can ever match a build
    src = tmp_path / "gen.cpp"
    src.write_text('#include "generation.hpp"\n#include <stdio.h>\nusing namespace aboria;\n'
                   'int main() {\n'
                   '  const uint32_t probe[] = {0u, 1u, 2u, 0x7FFFFFFFu, 0xFFFFFFFDu, 0xFFFFFFFEu, 0xFFFFFFFFu};\n'
                   '  for (uint32_t g : probe) printf("%u %u\\n", g, next_generation(g));\n'
                   '  uint32_t g = 0xFFFFFFF0u;\n'
                   '  for (int k = 0; k < 64; ++k) { g = next_generation(g); if (g == kGenNone || g == kGenNeverListed) return 1; }\n'
                   '  return 0;\n}\n')
    exe = tmp_path / "gen"
    subprocess.run(["g++", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0
    got = dict(tuple(int(v) for v in line.split()) for line in out.stdout.split("\n") if line)
    assert got == {0: 1, 1: 2, 2: 3, 0x7FFFFFFF: 0x80000000, 0xFFFFFFFD: 0xFFFFFFFE, 0xFFFFFFFE: 1, 0xFFFFFFFF: 1}
