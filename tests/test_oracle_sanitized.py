"""CPU test: the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs every pin
cleanly (no out-of-bounds access, use after free, signed overflow, misaligned access, ... in the
C code the GPU path is compared with).

The instrumented library is loaded into a child Python process with the ASan runtime preloaded
(a sanitized shared object cannot be loaded into an uninstrumented interpreter otherwise);
leak detection is off because the interpreter itself keeps allocations until exit. Any sanitizer
report aborts the child, so the test passes only on a clean run of all pins.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

CHILD = r"""
import sys
sys.path[:0] = [{tests!r}, {root!r}]
import oracle, oracle_pins
O = oracle.Oracle(oracle.load({lib!r}))
for pin in oracle_pins.PINS + oracle_pins.EXTRA_PINS:
    pin(O)
    print("ok", pin.__name__, flush=True)
print("all pins clean under the sanitizers", flush=True)
"""


def runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.timeout(900)
def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libblink_ref_san.so")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", oracle.HERE, "-o", lib, oracle.SRC, "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    code = CHILD.format(tests=HERE, root=os.path.dirname(HERE), lib=lib)
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=850)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "all pins clean under the sanitizers" in res.stdout, tail
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, tail
