"""Uneven batches of finite molecules in one launch sequence
(mbd_evaluate_batch): per-molecule energy and force errors vs the oracle."""
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_E = {"fp64": 1e-10, "fp32_refined": 1e-7}


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["fp64", "fp32_refined"])
def ctx(request):
    from paper_2308_03140_amd import torch_api as T
    c = T.Context(0, request.param)
    yield c
    c.close()


def _mols(seed, count, nmin, nmax):
    rng = np.random.default_rng(seed)
    out = []
    for m in range(count):
        N = int(rng.integers(nmin, nmax + 1))
        out.append(gen.finite_cluster(seed * 1000 + m, N, 12.0 * (N / 32.0) ** (1 / 3)))
    return out


@pytest.mark.parametrize("count,nmin,nmax", [(1, 5, 5), (7, 1, 30), (24, 10, 70)])
def test_uneven_batch(ctx, count, nmin, nmax):
    from paper_2308_03140_amd import torch_api as T
    _note("batch %s count=%d N in [%d,%d]" % (ctx.precision, count, nmin, nmax))
    mols = _mols(count + nmin, count, nmin, nmax)
    outs = T.evaluate_batch(ctx, [dict(m, coords=torch.tensor(m["coords"], device="cuda")) for m in mols])
    for m, o in zip(mols, outs):
        assert o["status"] == 0
        ref = oracle.mbd_finite(m["coords"], m["alpha0"], m["omega"], m["rvdw"], m["beta"], m["a"])
        N = len(m["omega"])
        assert abs(o["energy"].item() - ref["energy"]) / N <= TOL_E[ctx.precision]
        assert np.abs(o["grad_coords"].cpu().numpy() - ref["grad_R"]).max() <= 1e-6
        assert np.abs(o["grad_alpha0"].cpu().numpy() - ref["grad_alpha0"]).max() <= 1e-6
        assert np.abs(o["grad_omega"].cpu().numpy() - ref["grad_omega"]).max() <= 1e-6


def test_batch_repeat_and_status(ctx):
    """Same signature twice (the second call replays the captured launch
    sequence) with different inputs; a collapsed member reports its own status."""
    from paper_2308_03140_amd import torch_api as T
    _note("batch repeat %s" % ctx.precision)
    mols = _mols(5, 6, 8, 40)
    for rep in range(3):
        ms = [dict(m, alpha0=m["alpha0"] * (1.0 + 0.1 * rep)) for m in mols]
        outs = T.evaluate_batch(ctx, [dict(m, coords=torch.tensor(m["coords"], device="cuda")) for m in ms])
        for m, o in zip(ms, outs):
            ref = oracle.mbd_finite(m["coords"], m["alpha0"], m["omega"], m["rvdw"], m["beta"], m["a"])
            assert abs(o["energy"].item() - ref["energy"]) / len(m["omega"]) <= TOL_E[ctx.precision]
    bad = dict(mols[2], coords=np.array([[0.0, 0, 0], [0, 0, 3.0]]), alpha0=np.array([200.0, 200.0]),
               omega=np.array([0.5, 0.5]), rvdw=np.array([1.0, 1.0]), beta=0.0)
    ms = [mols[0], bad, mols[1]]
    outs = T.evaluate_batch(ctx, [dict(m, coords=torch.tensor(m["coords"], device="cuda")) for m in ms])
    assert [o["status"] for o in outs] == [0, 2, 0]
    ref = oracle.mbd_finite(mols[1]["coords"], mols[1]["alpha0"], mols[1]["omega"], mols[1]["rvdw"])
    assert abs(outs[2]["energy"].item() - ref["energy"]) / len(mols[1]["omega"]) <= TOL_E[ctx.precision]


def test_tuning_change_retires_captured_batches(ctx, tmp_path):
    """A batch is captured on its first call and replayed after; loading a
    tuning table (here with each GEMM output tile in turn) retires the
    captured sequences, and the replays after it still match the oracle."""
    import json
    from paper_2308_03140_amd import torch_api as T
    _note("batch tuning change %s" % ctx.precision)
    mols = _mols(9, 5, 20, 60)
    systems = [dict(m, coords=torch.tensor(m["coords"], device="cuda")) for m in mols]
    refs = [oracle.mbd_finite(m["coords"], m["alpha0"], m["omega"], m["rvdw"], m["beta"], m["a"]) for m in mols]
    nmax = max(3 * len(m["omega"]) for m in mols)
    key = "fp32" if ctx.precision == "fp32_refined" else "fp64"
    try:
        for ts in (64, 128, 64):
            path = tmp_path / ("tune_%d.json" % ts)
            path.write_text(json.dumps({"fp64": {}, "fp32": {}, key: {str(nmax): [1536, 1536, ts]}}))
            ctx.load_tuning(str(path))
            for rep in range(2):   # capture, then replay
                outs = T.evaluate_batch(ctx, systems)
                for m, o, ref in zip(mols, outs, refs):
                    assert o["status"] == 0
                    N = len(m["omega"])
                    assert abs(o["energy"].item() - ref["energy"]) / N <= TOL_E[ctx.precision], (ts, rep)
                    assert np.abs(o["grad_coords"].cpu().numpy() - ref["grad_R"]).max() <= 1e-6, (ts, rep)
    finally:
        # back to the untuned defaults for the module's later tests
        empty = tmp_path / "tune_empty.json"
        empty.write_text(json.dumps({"fp64": {}, "fp32": {}}))
        ctx.load_tuning(str(empty))


def test_molecule_batch_512():
    """The 512-molecule workload (N ~ U{10..300}) in one batched call with
    FP32 + refinement: every molecule against the FP64 GPU path (which
    reduces this batch with one workgroup per matrix, largest first), and a
    seeded sample (plus the largest molecule) against the oracle in both."""
    from paper_2308_03140_amd import torch_api as T
    _note("molecule batch 512")
    mols = gen.molecule_batch()
    systems = [dict(m, coords=torch.tensor(m["coords"], device="cuda")) for m in mols]
    c32 = T.Context(0, "fp32_refined")
    c64 = T.Context(0, "fp64")
    o32 = T.evaluate_batch(c32, systems)
    o64 = T.evaluate_batch(c64, systems)
    worst = {"E": 0.0, "R": 0.0, "a": 0.0, "w": 0.0}
    for m, a, b in zip(mols, o32, o64):
        assert a["status"] == 0 and b["status"] == 0
        N = len(m["omega"])
        worst["E"] = max(worst["E"], abs(a["energy"].item() - b["energy"].item()) / N)
        for k, key in (("R", "grad_coords"), ("a", "grad_alpha0"), ("w", "grad_omega")):
            worst[k] = max(worst[k], (a[key] - b[key]).abs().max().item())
    _note("  worst vs FP64: %s" % worst)
    assert worst["E"] <= 1e-7 and max(worst["R"], worst["a"], worst["w"]) <= 1e-6, worst
    rng = np.random.default_rng(41)
    sample = sorted(set(rng.choice(len(mols), 6, replace=False).tolist())
                    | {int(np.argmax([len(m["omega"]) for m in mols]))})
    for i in sample:
        m = mols[i]
        ref = oracle.mbd_finite(m["coords"], m["alpha0"], m["omega"], m["rvdw"], m["beta"], m["a"])
        N = len(m["omega"])
        for o, tolE in ((o32[i], 1e-7), (o64[i], 1e-10)):
            assert abs(o["energy"].item() - ref["energy"]) / N <= tolE, (i, N)
            assert np.abs(o["grad_coords"].cpu().numpy() - ref["grad_R"]).max() <= 1e-6, (i, N)
            assert np.abs(o["grad_alpha0"].cpu().numpy() - ref["grad_alpha0"]).max() <= 1e-6, (i, N)
            assert np.abs(o["grad_omega"].cpu().numpy() - ref["grad_omega"]).max() <= 1e-6, (i, N)
    c32.close()
    c64.close()


@pytest.mark.parametrize("tol", ["1e-30", "1e30"])
def test_refinement_second_step_forced_and_suppressed(monkeypatch, tol):
    """FP32 + refinement with the second refinement step taken by every
    molecule (threshold 1e-30) and by none (1e30): the second step's products
    and the pass-through of molecules that skip it both reach the oracle."""
    from paper_2308_03140_amd import torch_api as T
    _note("refinement second step, MBD_REFINE_TOL=%s" % tol)
    monkeypatch.setenv("MBD_REFINE_TOL", tol)
    c = T.Context(0, "fp32_refined")
    try:
        mols = _mols(77, 6, 8, 60)
        outs = T.evaluate_batch(c, [dict(m, coords=torch.tensor(m["coords"], device="cuda")) for m in mols])
        for m, o in zip(mols, outs):
            assert o["status"] == 0
            ref = oracle.mbd_finite(m["coords"], m["alpha0"], m["omega"], m["rvdw"], m["beta"], m["a"])
            N = len(m["omega"])
            assert abs(o["energy"].item() - ref["energy"]) / N <= 1e-7
            assert np.abs(o["grad_coords"].cpu().numpy() - ref["grad_R"]).max() <= 1e-6
            assert np.abs(o["grad_omega"].cpu().numpy() - ref["grad_omega"]).max() <= 1e-6
    finally:
        c.close()
