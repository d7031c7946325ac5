"""The C ABI used from plain C99: a client built with the host C compiler
against include/taskgraph.h and linked with the library builds, compiles and
models a graph and computes last-user dependences (host calls only)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2508_16522_amd")


def test_c_client(tglib, tmp_path):
    exe = tmp_path / "abi_client"
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "native", "abi_client.c"), "-o", str(exe), "-L", LIBDIR,
                           "-ltaskgraph", "-Wl,-rpath," + LIBDIR, "-Wl,--allow-shlib-undefined"])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi client ok" in r.stdout
