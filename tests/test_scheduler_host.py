"""Host checks of the serving layer: the continuous-batching scheduler runs
with a fake executor (sleeps in place of solves) in a small C++ driver built
with g++, and the ctypes records of the serving ABI match the C layout of
include/vie.h field by field."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1902_02196_amd", "csrc")
CASES = ("oversize", "slots", "budget", "backfill", "aging", "fifo", "status", "percentiles", "shutdown")


def _gxx():
    g = shutil.which("g++")
    if g is None:
        pytest.skip("g++ not available")
    return g


def test_scheduler_with_fake_executor(tmp_path):
    exe = str(tmp_path / "sched_driver")
    subprocess.run([_gxx(), "-std=c++17", "-O1", "-pthread", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "sched_driver.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    ok = {line.split()[1] for line in r.stdout.splitlines() if line.startswith("ok ")}
    assert ok == set(CASES), r.stdout


def _c_layout(tmp_path, struct, fields):
    src = tmp_path / ("%s.c" % struct)
    body = "".join('printf("%%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));\n' % (struct, f, struct, f)
                   for f in fields)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"vie.h\"\nint main(void){\n%s"
                   "printf(\"%%zu\\n\", sizeof(%s));return 0;}\n" % (body, struct))
    exe = str(tmp_path / struct)
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    rows = [tuple(int(v) for v in line.split()) for line in out[:len(fields)]]
    return rows, int(out[len(fields)])


@pytest.mark.parametrize("name,cname", [("SolveOpts", "vie_solve_opts"), ("SolveStats", "vie_solve_stats"),
                                        ("Request", "vie_request"), ("RequestInfo", "vie_request_info"),
                                        ("ServingStats", "vie_serving_stats"), ("TuckerInfo", "vie_tucker_info")])
def test_ctypes_records_match_header(tmp_path, name, cname):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    try:
        import paper_1902_02196_amd as vie
    except ImportError as e:
        pytest.skip(str(e))
    cls = getattr(vie, name)
    fields = [f for f, _ in cls._fields_]
    rows, size = _c_layout(tmp_path, cname, fields)
    for f, (off, sz) in zip(fields, rows):
        d = getattr(cls, f)
        assert (d.offset, d.size) == (off, sz), f
    assert ctypes.sizeof(cls) == size
