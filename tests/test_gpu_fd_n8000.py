"""N=8000 cluster (Q of order 24000): one position component of the adjoint
gradient (through the torch.autograd.Function) against a central difference
of FP64 GPU energies.  The 20-component check is tests/fd_check_n8000.py."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def test_fd_n8000_one_component():
    import fd_check_n8000
    res = fd_check_n8000.run(n_coords=1, n_alpha=0, log=lambda s: print(s, flush=True))
    assert res["max_err_grad_R"] <= 1e-6, res["components"]
