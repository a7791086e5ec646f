"""torch.autograd.Function over the C ABI: gradients vs the oracle and vs
central finite differences of the GPU energy."""
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_03140_amd import torch_api as T
    c = T.Context(0, "fp64")
    yield c
    c.close()


def _t(x, grad=False):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda", requires_grad=grad)


def test_finite_autograd_matches_oracle(ctx):
    from paper_2308_03140_amd.autograd import mbd_energy
    _note("autograd finite N=40")
    c = gen.finite_cluster(31, 40, 12.0 * (40 / 32.0) ** (1 / 3))
    R, a0, om, rv = _t(c["coords"], True), _t(c["alpha0"], True), _t(c["omega"], True), _t(c["rvdw"], True)
    E = mbd_energy(R, a0, om, rv, ctx, beta=c["beta"], a=c["a"])
    (2.5 * E).backward()
    ref = oracle.mbd_finite(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"])
    assert abs(E.item() - ref["energy"]) / 40 < 1e-10
    np.testing.assert_allclose(R.grad.cpu().numpy(), 2.5 * ref["grad_R"], atol=1e-9)
    np.testing.assert_allclose(a0.grad.cpu().numpy(), 2.5 * ref["grad_alpha0"], atol=1e-9)
    np.testing.assert_allclose(om.grad.cpu().numpy(), 2.5 * ref["grad_omega"], atol=1e-9)
    np.testing.assert_allclose(rv.grad.cpu().numpy(), 2.5 * ref["grad_rvdw"], atol=1e-9)


def test_periodic_autograd_lattice(ctx):
    from paper_2308_03140_amd.autograd import mbd_energy
    _note("autograd periodic N=3")
    c = gen.small_crystal(61, 3, kgrid=(2, 2, 2))
    R, a0 = _t(c["coords"], True), _t(c["alpha0"], True)
    L = torch.tensor(c["lattice"], dtype=torch.float64, requires_grad=True)  # host tensor
    E = mbd_energy(R, a0, _t(c["omega"]), _t(c["rvdw"]), ctx, lattice=L, q_frac=c["q_frac"])
    E.backward()
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c["omega"], c["rvdw"])
    np.testing.assert_allclose(L.grad.numpy(), ref["grad_lattice"], atol=1e-9)
    np.testing.assert_allclose(R.grad.cpu().numpy(), ref["grad_R"], atol=1e-9)
    np.testing.assert_allclose(a0.grad.cpu().numpy(), ref["grad_alpha0"], atol=1e-9)


def test_fd_of_gpu_energy(ctx):
    """Central differences (h = 1e-4 bohr) of the GPU FP64 energy at random
    coordinates of a 400-atom dense cluster vs the autograd gradient."""
    from paper_2308_03140_amd.autograd import mbd_energy
    from paper_2308_03140_amd import torch_api as T
    _note("autograd FD N=400")
    c = gen.cluster_dense(41, 400)
    s = 0.4  # well inside the positive-definite region at this density
    a0 = c["alpha0"] * s
    R = _t(c["coords"], True)
    E = mbd_energy(R, _t(a0), _t(c["omega"]), _t(c["rvdw"]), ctx)
    E.backward()
    g = R.grad.cpu().numpy()
    rng = np.random.default_rng(55)
    h = 1e-4
    for _ in range(6):
        i, k = int(rng.integers(400)), int(rng.integers(3))
        vals = []
        for sg in (1, -1):
            X = c["coords"].copy()
            X[i, k] += sg * h
            vals.append(T.evaluate(ctx, _t(X), a0, c["omega"], c["rvdw"], gradients=False)["energy"].item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i, k]) < 1e-6, (i, k, fd, g[i, k])
