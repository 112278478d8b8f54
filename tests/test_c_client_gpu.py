"""GPU: the library used from C with no Python (tests/c_abi_client.c): a
key + payload merge, device and host co-ranks and two argument errors,
checked against the oracle's C merge inside the program."""
import subprocess

import pytest

from tests import c_client

pytestmark = pytest.mark.gpu


def test_c_client_runs(tmp_path):
    exe = c_client.build(str(tmp_path))
    print("\n[c client] running", exe, flush=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr + res.stdout
    assert "c client ok" in res.stdout
