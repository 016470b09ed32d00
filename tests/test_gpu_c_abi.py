"""The C ABI from a plain C program (tests/c_abi_droplet.c, built with the
library): context, caller-owned workspace from the HIP runtime, a 32^3
droplet stepped 200 times, mass and momentum invariants on the reductions.
No Python or PyTorch sits between the program and liblbfe.so."""
import os
import subprocess

import pytest

from gpu_util import say
from paper_2504_03819_amd import build

pytestmark = pytest.mark.gpu


def test_plain_c_program_steps_a_droplet():
    exe = build.C_EXAMPLE
    assert os.path.exists(exe), f"{exe} missing: build the package first (python __graft_entry__.py)"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    say(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    assert "200 steps" in r.stdout
