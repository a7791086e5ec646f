"""Periodic MBD parity (Ewald-summed T^lr(q), all q of the mesh batched):
HIP path through the C ABI vs the CPU oracle on seeded triclinic cells."""
import json
import os
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL_E = {"fp64": 1e-10, "fp32_refined": 1e-7}
TOL_G = 1e-6


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["fp64", "fp32_refined"])
def ctx(request):
    from paper_2308_03140_amd import torch_api as T
    c = T.Context(0, request.param)
    yield c
    c.close()


def _run(ctx, c, **kw):
    from paper_2308_03140_amd import torch_api as T
    return T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                      beta=c["beta"], a=c["a"], lattice=c["lattice"], q_frac=c["q_frac"], **kw)


def _compare(ctx, N, out, ref):
    dE = abs(out["energy"].item() - ref["energy"]) / N
    assert dE <= TOL_E[ctx.precision], ("energy per atom", dE)
    gR = out["grad_coords"].cpu().numpy()
    assert np.abs(gR - ref["grad_R"]).max() <= TOL_G, ("grad_R", np.abs(gR - ref["grad_R"]).max())
    ga = out["grad_alpha0"].cpu().numpy()
    assert np.abs(ga - ref["grad_alpha0"]).max() <= TOL_G, ("grad_alpha0", np.abs(ga - ref["grad_alpha0"]).max())
    gl = out["grad_lattice"].cpu().numpy()
    assert np.abs(gl - ref["grad_lattice"]).max() <= TOL_G, ("grad_lattice", np.abs(gl - ref["grad_lattice"]).max())


@pytest.mark.parametrize("N,kgrid", [(1, (2, 1, 1)), (3, (2, 2, 2)), (8, (2, 2, 1))])
def test_small_cells(ctx, N, kgrid):
    _note("periodic %s N=%d k=%s" % (ctx.precision, N, kgrid))
    c = gen.small_crystal(50 + N, N, kgrid=kgrid)
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c["omega"], c["rvdw"],
                              c["beta"], c["a"])
    out = _run(ctx, c, eigvals=True)
    torch.cuda.synchronize()
    _compare(ctx, N, out, ref)
    tol = 1e-12 if ctx.precision == "fp64" else 1e-9
    assert np.abs(out["eigvals"].cpu().numpy() - ref["eigs"]).max() <= tol


def test_gamma_containing_grid_and_undamped(ctx):
    _note("periodic gamma grid %s" % ctx.precision)
    c = gen.small_crystal(77, 4, kgrid=(2, 2, 2))
    qf = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.5, 0.5]])
    c = dict(c, q_frac=qf, beta=0.0)
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], qf, c["alpha0"], c["omega"], c["rvdw"], 0.0, c["a"])
    out = _run(ctx, c)
    _compare(ctx, 4, out, ref)


def test_crystal_n64_golden(ctx):
    path = os.path.join(GOLDEN, "crystal_n64.json")
    if not os.path.exists(path):
        pytest.skip("golden values not generated")
    _note("periodic crystal N=64 4x4x4 %s" % ctx.precision)
    g = json.load(open(path))
    c = gen.crystal_n64()
    assert abs(c["alpha_scale"] - g["alpha_scale"]) == 0.0
    ref = {"energy": g["energy"], "grad_R": np.array(g["grad_R"]), "grad_alpha0": np.array(g["grad_alpha0"]),
           "grad_lattice": np.array(g["grad_lattice"])}
    out = _run(ctx, c)
    _compare(ctx, 64, out, ref)
