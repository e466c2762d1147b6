"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle and the seeded graph generators, built with -fsanitize=address,undefined
(no recovery: any report aborts) and exercised by tests/sanitize_driver.cpp
on generated graphs and closed forms.  CPU only."""
from __future__ import annotations

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    objs = []
    for src in ("bc_oracle.c", "sssp_oracle.c", "tc_oracle.c"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call(["gcc", "-std=c99", "-ffp-contract=off", *SAN, "-c",
                               os.path.join(ROOT, "oracle", src), "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(["g++", "-std=c++17", "-pthread", *SAN,
                           os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
                           os.path.join(ROOT, "paper_2305_03317_amd", "csrc", "graphgen.cpp"),
                           *objs, "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "sanitizer driver ok" in r.stdout
