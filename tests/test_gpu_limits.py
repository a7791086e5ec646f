"""Batched launches put the matrices of a call on one grid dimension, which
holds at most 65535: larger requests are refused up front with
MBD_ERR_UNSUPPORTED (6) instead of failing a launch."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

UNSUPPORTED = 6


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_03140_amd import torch_api as T
    c = T.Context(0, "fp64")
    yield c
    c.close()


def test_eigh_batch_limit(ctx):
    from paper_2308_03140_amd import _abi as A
    _note("limits: eigh batch of 65536")
    nb = 65536
    M = torch.ones(nb, dtype=torch.float64, device="cuda")
    w = torch.empty(nb, dtype=torch.float64, device="cuda")
    code = A.mbd_eigh(ctx.handle, 0, 1, nb, M.data_ptr(), 1, 1, w.data_ptr(), None, 1, 1)
    assert code == UNSUPPORTED
    # the largest accepted batch still solves (order 1: w = A)
    code = A.mbd_eigh(ctx.handle, 0, 1, nb - 1, M.data_ptr(), 1, 1, w.data_ptr(), None, 1, 1)
    assert code == 0
    assert torch.all(w[:nb - 1] == 1.0)


def test_q_point_limit(ctx):
    from paper_2308_03140_amd import torch_api as T
    _note("limits: 65536 q points")
    c = gen.small_crystal(66, 2, kgrid=(1, 1, 1))
    q = np.zeros((65536, 3))
    with pytest.raises(T.MBDError) as e:
        T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                   beta=c["beta"], a=c["a"], lattice=c["lattice"], q_frac=q)
    assert e.value.code == UNSUPPORTED


def test_freq_matrix_limit(ctx):
    from paper_2308_03140_amd import torch_api as T
    _note("limits: frequency route, 16 frequencies x 4097 q points")
    c = gen.small_crystal(67, 2, kgrid=(1, 1, 1))
    q = np.zeros((4097, 3))
    with pytest.raises(T.MBDError) as e:
        T.freq_evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                        beta=c["beta"], a=c["a"], lattice=c["lattice"], q_frac=q, n_freq=16)
    assert e.value.code == UNSUPPORTED
