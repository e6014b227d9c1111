"""Memory admission of the query server, on the CPU with a fake executor.

The server admits queued queries in submission order while a slot is free
and its hash tables get a contiguous range of the fixed pool of table
entries (server_admission.h, the code the server runs).  A C++ fake executor
drives thousands of queries with random table sizes and run lengths through
it and checks that admission never over-commits the pool, never hands out
overlapping ranges, keeps submission order, rejects only queries larger than
the whole pool, and returns the pool whole."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fake(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("admission") / "fake")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", os.path.join(ROOT, "tests", "server_admission_fake.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_admission_never_over_commits(fake, seed):
    r = subprocess.run([fake, str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
