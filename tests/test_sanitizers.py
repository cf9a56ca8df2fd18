"""The oracle and the seeded generators built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code, g++/gcc) and run by a driver on tiny
random inputs with empty inputs, duplicate and extreme keys; any report
aborts the driver."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1",
         "-fno-omit-frame-pointer"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="needs gcc/g++")
def test_oracle_and_generators_under_sanitizers(tmp_path):
    objs = []
    for src, comp, std in [("oracle/oracle.cpp", "g++", "-std=c++17"),
                           ("paper_2508_04701_amd/datagen/gen.c", "gcc", "-std=c11"),
                           ("tests/sanitize/driver.cpp", "g++", "-std=c++17")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([comp, std, *FLAGS, "-c", os.path.join(ROOT, src), "-o", obj], check=True)
        objs.append(obj)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", *FLAGS, *objs, "-o", exe, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized ok" in r.stdout
