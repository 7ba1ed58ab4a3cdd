"""No C++ exception crosses the C ABI (CPU only).

Every function include/cspd.h declares is either a one-line accessor that
cannot throw or runs its body inside `guarded` (status entry points) or a
try/catch (void and count entry points); and `guarded` itself, compiled into
a small host program, turns std::bad_alloc into CSPD_E_NOMEM, any other
exception into CSPD_E_DEVICE with the thread's error message set, and passes
a normal return through.
"""
import os
import re
import shutil
import subprocess

import pytest

from test_abi import declared_functions

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_05174_amd", "csrc")
ONE_LINERS = {"cspd_last_error", "cspd_version", "cspd_plan_device_bytes"}


def _definitions():
    """name -> body text of every top-level function definition in csrc."""
    defs = {}
    for fn in sorted(os.listdir(CSRC)):
        if not fn.endswith((".cpp", ".hip")):
            continue
        text = open(os.path.join(CSRC, fn)).read()
        for m in re.finditer(r"^(?:extern \"C\" )?[a-z_0-9 ]+\*?\s*\b(cspd_[a-z_]+)\(([^;{]*?)\)\s*\n?\{", text,
                             flags=re.M | re.S):
            start = m.end()
            depth, i = 1, start
            while depth:
                depth += {"{": 1, "}": -1}.get(text[i], 0)
                i += 1
            defs[m.group(1)] = (fn, text[start:i - 1])
    return defs


def test_every_entry_point_is_guarded():
    defs = _definitions()
    for name in declared_functions():
        if name in ONE_LINERS:
            continue
        assert name in defs, f"no definition of {name} found"
        fn, body = defs[name]
        first = body.strip().splitlines()[0].strip()
        if name == "cspd_patch_count":
            # pure arithmetic on a caller struct: no allocation, no library call
            assert "new" not in body and "std::" not in body and "hip" not in body, body
            continue
        assert first.startswith("return guarded(") or first.startswith("try {"), f"{fn}: {name} starts with {first!r}"


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_guard_turns_exceptions_into_statuses(tmp_path):
    src = tmp_path / "guard.cpp"
    src.write_text(r'''
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include "cspd_internal.h"
namespace cspd {
static char msg[256];
cspd_status set_error(cspd_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof(msg), fmt, ap);
    va_end(ap);
    return code;
}
}
int main()
{
    using namespace cspd;
    int bad = 0;
    if (guarded([] () -> cspd_status { throw std::bad_alloc(); }) != CSPD_E_NOMEM) bad |= 1;
    if (guarded([] () -> cspd_status { throw std::runtime_error("boom"); }) != CSPD_E_DEVICE) bad |= 2;
    if (!std::strstr(msg, "boom")) bad |= 4;
    if (guarded([] () -> cspd_status { throw 7; }) != CSPD_E_DEVICE) bad |= 8;
    if (guarded([] () -> cspd_status { return CSPD_E_SHAPE; }) != CSPD_E_SHAPE) bad |= 16;
    std::printf("%d\n", bad);
    return bad;
}
''')
    exe = tmp_path / "guard"
    inc = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    r = subprocess.run(["hipcc", "-std=c++17", "-O1", *inc, str(src), "-o", str(exe)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
