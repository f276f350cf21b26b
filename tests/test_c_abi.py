"""The library called from plain C (tests/c_abi/embed_file.c: include/lne.h
and the HIP runtime only): argument errors are returned on the host before
any GPU call."""
import os
import subprocess

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "embed_file")


def test_c_caller_argument_checks(lne):
    lne.load()                                   # liblne.so is built
    if not os.path.exists(EXE):
        from tests.c_abi import build
        build.build()
    r = subprocess.run([EXE, "--check"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "checks ok" in r.stdout
