"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Every source is compiled with the host pass instrumented (the device code is
built as usual) into a separate library in a temporary directory, and
host_sanitizer_driver.cpp creates meshes from valid and invalid inputs
through the C ABI.  Without a GPU a valid mesh stops at the first device
allocation, after validation, geometry, the recursive bisection and the
whole tile plan have run on the host; invalid inputs take the error paths.
The run must end normally with no sanitizer report and the expected status
of every case.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = "-O1 -g -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined " \
      "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer".split()


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, (" ".join(cmd), res.stderr[-2000:])


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    from paper_2606_23458_amd import build as b
    out = tmp_path_factory.mktemp("san")
    cc = b.hipcc()
    objs = [str(out / (s + ".o")) for s in b.SOURCES]
    cmds = [[cc, *b.flags(), *SAN, "-c", os.path.join(b.CSRC, s), "-o", o] for s, o in zip(b.SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(_run, cmds))
    lib = out / "libpfrac_san.so"
    _run([cc, f"--offload-arch={b.ARCH}", "-shared", "-fPIC", *SAN, "-o", str(lib), *objs])
    exe = out / "driver"
    _run([cc, "-std=c++17", *SAN, "-I", os.path.join(b.ROOT, "include"), os.path.join(HERE, "host_sanitizer_driver.cpp"),
          "-o", str(exe), "-L", str(out), "-lpfrac_san", f"-Wl,-rpath,{out}"])
    return str(exe)


def test_mesh_creation_is_clean_under_host_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    report = res.stdout + res.stderr
    assert res.returncode == 0, report[-3000:]
    assert "AddressSanitizer" not in report and "LeakSanitizer" not in report, report[-3000:]
    assert "runtime error" not in report, report[-3000:]
    status = dict(line.split() for line in res.stdout.splitlines())
    status = {k: int(v) for k, v in status.items()}
    # valid meshes: created (a GPU is present) or stopped at the first device allocation
    for k in ("valid_f64_t64", "valid_f32_t256", "valid_f64_t2048", "valid_batched"):
        assert status[k] in (0, 3, 4), (k, status[k])
    assert status["zero_area"] == 2 and status["index_range"] == 2 and status["unused_node"] == 2, status
    assert status["no_instances"] == 1 and status["tile_too_large"] == 1, status
