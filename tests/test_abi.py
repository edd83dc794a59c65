"""CPU checks of the C interface: the library loads, exports every entry point
declared in include/mars.h, and the Python structures match the C layout.
No compute call is made (there is no GPU here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mars.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mars_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1907_05124_amd import build, mars

    if not os.path.exists(mars.LIB_PATH):
        build.build()
    return mars.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1907_05124_amd import mars

    declared = _declared()
    assert declared, "no declarations parsed"
    out = subprocess.run(["nm", "-D", "--defined-only", mars.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mars_\w+)", out))
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)
    assert sorted(mars.EXPORTS) == declared


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against the header with gcc and compare sizes/offsets with ctypes."""
    import ctypes

    from paper_1907_05124_amd import mars

    probe = tmp_path / "probe.c"
    fields_s = [f for f, _ in mars.Schedule._fields_]
    fields_r = [f for f, _ in mars.Result._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mars.h"', "int main(void){"]
    lines.append('printf("S %zu\\n", sizeof(mars_schedule));')
    lines.append('printf("R %zu\\n", sizeof(mars_result));')
    for f in fields_s:
        lines.append('printf("s.%s %%zu\\n", offsetof(mars_schedule, %s));' % (f, f))
    for f in fields_r:
        lines.append('printf("r.%s %%zu\\n", offsetof(mars_result, %s));' % (f, f))
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(got["S"]) == ctypes.sizeof(mars.Schedule)
    assert int(got["R"]) == ctypes.sizeof(mars.Result)
    for f in fields_s:
        assert int(got["s." + f]) == getattr(mars.Schedule, f).offset, f
    for f in fields_r:
        assert int(got["r." + f]) == getattr(mars.Result, f).offset, f


def test_status_strings(lib):
    from paper_1907_05124_amd import mars

    for code in range(9):
        assert mars.status_str(code) != "unknown status"
    assert mars.status_str(99) == "unknown status"
