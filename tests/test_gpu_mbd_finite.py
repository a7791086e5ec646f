"""Finite-system MBD parity: HIP path through the C ABI vs the CPU oracle,
element by element on seeded inputs.  Tolerances: |dE|/N <= 1e-10 Ha/atom
(FP64 path), <= 1e-7 Ha/atom (FP32 + refinement path), gradients <= 1e-6
Ha/bohr (both paths)."""
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

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


def _cluster(seed, N, side_ang=None):
    side = side_ang if side_ang else 12.0 * (N / 32.0) ** (1.0 / 3.0)
    return gen.finite_cluster(seed, N, side)


def _run(ctx, c, **kw):
    from paper_2308_03140_amd import torch_api as T
    return T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                      beta=c["beta"], a=c["a"], **kw)


def _compare(ctx, c, out, ref):
    N = len(c["omega"])
    dE = abs(out["energy"].item() - ref["energy"]) / N
    assert dE <= TOL_E[ctx.precision], ("energy per atom", dE)
    for k in ("grad_R", "grad_alpha0", "grad_omega", "grad_rvdw"):
        g = out[{"grad_R": "grad_coords"}.get(k, k)].cpu().numpy().reshape(ref[k].shape)
        err = np.abs(g - ref[k]).max()
        assert err <= TOL_G, (k, err)


@pytest.mark.parametrize("N", [1, 2, 5, 22, 32, 75, 150])
def test_cluster_parity(ctx, N):
    _note("finite parity %s N=%d" % (ctx.precision, N))
    c = _cluster(100 + N, N)
    ref = oracle.mbd_finite(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"])
    out = _run(ctx, c)
    torch.cuda.synchronize()
    _compare(ctx, c, out, ref)


def test_config_n32(ctx):
    _note("config N=32 seed 1 %s" % ctx.precision)
    c = gen.cluster_n32()
    ref = oracle.mbd_finite(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"])
    out = _run(ctx, c, eigvals=True)
    _compare(ctx, c, out, ref)
    w = out["eigvals"].cpu().numpy()[0]
    tol = 1e-12 if ctx.precision == "fp64" else 1e-9
    assert np.abs(w - ref["eigs"]).max() <= tol


def test_dimer_closed_form_gpu(ctx):
    _note("dimer %s" % ctx.precision)
    coords = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 7.5]])
    c = {"coords": coords, "alpha0": np.array([11.0, 17.0]), "omega": np.array([0.6, 0.4]),
         "rvdw": np.array([3.5, 3.9]), "beta": 0.83, "a": 6.0}
    ref = oracle.mbd_finite(coords, c["alpha0"], c["omega"], c["rvdw"], 0.83, 6.0)
    out = _run(ctx, c)
    _compare(ctx, c, out, ref)


def test_c6_input(ctx):
    _note("c6 input %s" % ctx.precision)
    from paper_2308_03140_amd import torch_api as T
    c = _cluster(7, 12)
    c6 = 0.75 * c["omega"] * c["alpha0"] ** 2
    ref = oracle.mbd_finite_c6(c["coords"], c["alpha0"], c6, c["rvdw"])
    out = T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c6, c["rvdw"],
                     param="c6")
    assert abs(out["energy"].item() - ref["energy"]) / 12 <= TOL_E[ctx.precision]
    assert np.abs(out["grad_alpha0"].cpu().numpy() - ref["grad_alpha0_c6"]).max() <= TOL_G
    assert np.abs(out["grad_omega"].cpu().numpy() - ref["grad_c6"]).max() <= TOL_G


def test_collapse_reported(ctx):
    _note("collapse %s" % ctx.precision)
    from paper_2308_03140_amd import torch_api as T
    coords = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]])
    with pytest.raises(T.CollapseError):
        T.evaluate(ctx, torch.tensor(coords, device="cuda"), [200.0, 200.0], [0.5, 0.5], [1.0, 1.0], beta=0.0)


def test_invalid_inputs(ctx):
    _note("invalid inputs %s" % ctx.precision)
    from paper_2308_03140_amd import torch_api as T
    coords = torch.tensor([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], dtype=torch.float64, device="cuda")
    with pytest.raises(T.MBDError) as e:
        T.evaluate(ctx, coords, [10.0, 10.0], [0.5, 0.5], [3.0, 3.0])
    assert e.value.code == 1
    coords = torch.tensor([[0.0, 0.0, 0.0], [0.0, 0.0, 5.0]], dtype=torch.float64, device="cuda")
    with pytest.raises(T.MBDError) as e:
        T.evaluate(ctx, coords, [-10.0, 10.0], [0.5, 0.5], [3.0, 3.0])
    assert e.value.code == 1
    with pytest.raises(T.MBDError) as e:
        T.evaluate(ctx, coords, [float("nan"), 10.0], [0.5, 0.5], [3.0, 3.0])
    assert e.value.code == 1


def test_config_n2000_golden(ctx):
    """Full-size N=2000 cluster in the benchmark's launch configuration against
    stored oracle values (frequency route, 48-point grid): energy per atom and
    dE/dR of 8 sampled atoms.  The quadrature converges to ~1e-12 relative on
    small clusters; the bound here is the path's own tolerance."""
    import json
    import os
    _note("config N=2000 golden %s" % ctx.precision)
    with open(os.path.join(os.path.dirname(__file__), "golden", "cluster_n2000.json")) as f:
        ref = json.load(f)
    c = gen.cluster_n2000()
    assert abs(c["alpha_scale"] - ref["alpha_scale"]) < 1e-15
    out = _run(ctx, c)
    N = len(c["omega"])
    dE = abs(out["energy"].item() - ref["energy"]) / N
    _note("  dE/N = %.3e" % dE)
    assert dE <= TOL_E[ctx.precision], dE
    g = out["grad_coords"].cpu().numpy()[ref["atoms"]]
    err = np.abs(g - np.array(ref["grad_R_sample"])).max()
    _note("  max |dE/dR - ref| = %.3e" % err)
    assert err <= TOL_G, err
    for k, o in (("grad_alpha0_sample", "grad_alpha0"), ("grad_omega_sample", "grad_omega")):
        e = np.abs(out[o].cpu().numpy()[ref["atoms"]] - np.array(ref[k])).max()
        _note("  max |%s - ref| = %.3e" % (o, e))
        assert e <= TOL_G, (k, e)


@pytest.mark.parametrize("N", [5, 150])
def test_energy_only(ctx, N):
    """Energy alone: on the FP64 path the eigenvalues come from Sturm-count
    multisection (no eigenvectors are formed)."""
    _note("energy only %s N=%d" % (ctx.precision, N))
    c = _cluster(400 + N, N)
    ref = oracle.mbd_finite(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"], gradients=False)
    out = _run(ctx, c, gradients=False, eigvals=True)
    assert abs(out["energy"].item() - ref["energy"]) / N <= TOL_E[ctx.precision]
    tol = 1e-12 if ctx.precision == "fp64" else 1e-9
    assert np.abs(out["eigvals"].cpu().numpy()[0] - ref["eigs"]).max() <= tol


def test_energy_only_n2000_golden(ctx):
    import json
    import os
    _note("energy only N=2000 golden %s" % ctx.precision)
    with open(os.path.join(os.path.dirname(__file__), "golden", "cluster_n2000.json")) as f:
        ref = json.load(f)
    c = gen.cluster_n2000()
    out = _run(ctx, c, gradients=False)
    dE = abs(out["energy"].item() - ref["energy"]) / 2000
    _note("  dE/N = %.3e" % dE)
    assert dE <= TOL_E[ctx.precision], dE
