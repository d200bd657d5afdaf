"""The library used from C alone (tests/c_api/halo_world.c, built by
build()): a GPU-built locality plan of a 5-point grid, one request per rank
batched, each stage's messages moved by the program, halos and the backward
checked with plain loops, under block and cyclic placement."""
import os
import subprocess

import pytest

from tests.c_api.build import EXE
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def test_c_program_through_the_abi():
    need_gpu()
    assert os.path.exists(EXE), f"{EXE} is missing: build() compiles it"
    say("C ABI program")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok") and "node map 1: 0 mismatch" in r.stdout, r.stdout
