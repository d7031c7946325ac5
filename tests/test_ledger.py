"""The residency ledger's rule (which in-flight persistent launches a new
launch must follow so that no two launches whose workers do not fit the
device together overlap), compiled from the library's own header with the
host compiler and checked on the CPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ledger_rule(tmp_path):
    exe = tmp_path / "ledger_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror",
                           "-I", os.path.join(ROOT, "paper_2508_16522_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "ledger_check.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all cases pass" in r.stdout
