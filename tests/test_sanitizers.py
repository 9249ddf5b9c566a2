"""The oracle's pins and the host-side ABI tests, rerun in child processes
against copies of the oracle and of the library's host units built with
AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal). CPU
only: the host tests return before any launch."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

RUNNER = """
import sys
sys.path.insert(0, {root!r})
import {module} as m
m.LIB_PATH = {lib!r}
import pytest
rc = pytest.main(["-q", "-x", "-p", "no:cacheprovider", {tests!r}])
maps = open("/proc/self/maps").read()
if {lib!r} not in maps:
    print("the sanitized library was not loaded")
    rc = 3
sys.exit(rc)
"""


def _run(module, lib, tests, preload, tmp_path):
    script = tmp_path / ("run_%s.py" % module.replace(".", "_"))
    script.write_text(RUNNER.format(root=ROOT, module=module, lib=lib, tests=tests))
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])


def test_oracle_pins_under_asan_ubsan(tmp_path):
    from oracle import build as ob
    lib = ob.build(out=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    _run("oracle", lib, os.path.join(ROOT, "tests", "test_oracle_pins.py"), libasan, tmp_path)


def test_host_abi_under_asan_ubsan(tmp_path):
    from paper_0907_0792_amd import build as hb
    if not os.path.exists(hb.LIB):
        pytest.skip("the library is not built")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's ASan runtime is not installed")
    lib = hb.build_host_sanitized(str(tmp_path / "libmoa_asan.so"))
    _run("paper_0907_0792_amd", lib, os.path.join(ROOT, "tests", "test_abi_host.py"), rt[-1], tmp_path)
