"""The CPU-side code under AddressSanitizer and UndefinedBehaviorSanitizer: the FP64
oracle (every entry point on small frames) and the server's scheduling core (a seeded
random scenario with failures, cancellations and a device loss), each built with g++
into a program of its own and run as a child process."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_14827_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def build_and_run(tmp_path, name, sources, extra):
    exe = str(tmp_path / name)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *SAN, *extra, *sources, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    report = r.stdout + r.stderr
    if "LeakSanitizer does not work under ptrace" in report:
        env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "runtime error" not in report and "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert r.stdout.startswith("ok"), report[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "oracle_san",
                        [os.path.join(ROOT, "oracle", "dqj_oracle.cpp"),
                         os.path.join(ROOT, "tests", "sanitize_oracle_main.cpp")],
                        ["-fopenmp", "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle")])
    assert int(out.split()[1]) > 0


def test_serve_core_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "core_san",
                        [os.path.join(CSRC, "serve_core.cpp"),
                         os.path.join(ROOT, "tests", "sanitize_serve_core_main.cpp")],
                        ["-I", CSRC])
    assert "completed" in out
