"""The C ABI driven from a plain C program on the GPU (no Python or PyTorch in
the process): parameter rejection, FP64 mass conservation over 200 steps of a
ragged two-component gray domain with solid voxels and adhesion, a
bit-for-bit checkpoint restart, and a shortest-first server whose results
equal contexts stepped alone (tests/c_driver/abi_driver.c)."""
import subprocess

import pytest

from _common import build_c_driver

pytestmark = pytest.mark.gpu


def test_c_program_runs_on_the_device(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = build_c_driver(tmp_path / "abi_driver")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "C ABI OK" in r.stdout, r.stdout + r.stderr
