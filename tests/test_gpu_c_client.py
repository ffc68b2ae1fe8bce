"""The C ABI from plain C: runs tests/c_client/eigupd_client (built by
__graft_entry__.build() or tests/c_client/build.py), which creates a state,
uploads A = diag(lambda), applies the rank-2 update e_j a^T + a e_j^T of
Sec. 2.2 through eig_update_rankk and checks on the host the trace identity,
the ordering, orthogonality and the residual of the result."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "c_client", "eigupd_client")


def test_c_client_update():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(CLIENT), "build the C client first (tests/c_client/build.py)"
    print("case plain C client n=96 k=2", flush=True)
    r = subprocess.run([CLIENT], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "c client ok" in r.stdout
