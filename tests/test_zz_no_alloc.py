"""mbd_evaluate_noalloc (workspaces from the library's static device scratch,
no allocation) against mbd_evaluate on the same inputs, through the C ABI:
two calls in a row, the second on a smaller system, both precisions; the
FP64 fallback of an unconverged refinement runs inside the scratch too."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_E = {"fp64": 1e-10, "fp32_refined": 1e-7}
TOL_G = 1e-6


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _system(seed, N):
    return gen.finite_cluster(seed, N, 12.0 * (N / 32.0) ** (1.0 / 3.0))


def _eval(ctx, c, noalloc):
    from paper_2308_03140_amd import torch_api as T
    return T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                      beta=c["beta"], a=c["a"], eigvals=True, noalloc=noalloc)


def _same(prec, c, a, b):
    N = len(c["omega"])
    assert abs(a["energy"].item() - b["energy"].item()) / N <= TOL_E[prec]
    for k in ("grad_coords", "grad_alpha0", "grad_omega", "grad_rvdw"):
        assert (a[k] - b[k]).abs().max().item() <= TOL_G, k
    tol = 1e-12 if prec == "fp64" else 1e-9
    assert (a["eigvals"] - b["eigvals"]).abs().max().item() <= tol
    np.testing.assert_array_equal(a["errors"][2].item(), b["errors"][2].item())


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_noalloc_matches_evaluate(prec, monkeypatch):
    from paper_2308_03140_amd import torch_api as T
    monkeypatch.delenv("MBD_REFINE_TOL", raising=False)
    monkeypatch.delenv("MBD_REFINE_FALLBACK", raising=False)
    ctx = T.Context(0, prec)
    try:
        for seed, N in ((901, 256), (902, 40)):
            _note("noalloc %s N=%d" % (prec, N))
            c = _system(seed, N)
            ref = _eval(ctx, c, False)
            out = _eval(ctx, c, True)
            torch.cuda.synchronize()
            _same(prec, c, out, ref)
    finally:
        ctx.close()


def test_noalloc_fallback_fits_scratch(monkeypatch):
    """A refinement forced to miss its target: the FP32 attempt and the FP64
    re-evaluation of the largest accepted system share the scratch."""
    from paper_2308_03140_amd import torch_api as T
    monkeypatch.setenv("MBD_REFINE_TOL", "1e-300")
    monkeypatch.delenv("MBD_REFINE_FALLBACK", raising=False)
    ctx = T.Context(0, "fp32_refined")
    try:
        for seed, N in ((903, 256), (904, 17)):
            _note("noalloc fallback N=%d" % N)
            c = _system(seed, N)
            ref = _eval(ctx, c, False)
            out = _eval(ctx, c, True)
            assert out["errors"][2].item() == 0.0
            _same("fp64", c, out, ref)
    finally:
        ctx.close()


def test_noalloc_limits():
    from paper_2308_03140_amd import torch_api as T
    from paper_2308_03140_amd import _abi as A
    ctx = T.Context(0, "fp64")
    try:
        c = _system(905, A.MBD_NOALLOC_MAX_ATOMS + 1)
        with pytest.raises(T.MBDError) as e:
            _eval(ctx, c, True)
        assert e.value.code == A.MBD_ERR_INVALID_ARGUMENT
        p = gen.small_crystal(61, 2, kgrid=(1, 1, 1))
        with pytest.raises(T.MBDError) as e:
            T.evaluate(ctx, torch.tensor(p["coords"], device="cuda"), p["alpha0"], p["omega"], p["rvdw"],
                       lattice=p["lattice"], q_frac=p["q_frac"], noalloc=True)
        assert e.value.code == A.MBD_ERR_UNSUPPORTED
    finally:
        ctx.close()
