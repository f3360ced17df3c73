"""The library used from C through its ABI alone (tests/c_abi_client.c): device buffers
from the HIP runtime, sal_saliency on a small volume compared with the FP64 oracle at
cube 8, the paper's cube 5 and split-BF16 at cube 16, the batched tile check against
sal_raw_box and the whole-volume maps (bit for bit), and the refusal paths."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi_client")


def test_c_abi_client():
    if not os.path.exists(BIN):
        pytest.skip("tests/c_abi_client is built by __graft_entry__.build()")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c abi client: ok" in r.stdout
