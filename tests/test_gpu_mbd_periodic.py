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
    for k, o in (("grad_R", "grad_coords"), ("grad_alpha0", "grad_alpha0"), ("grad_omega", "grad_omega"),
                 ("grad_rvdw", "grad_rvdw"), ("grad_lattice", "grad_lattice")):
        if k not in ref:
            continue
        g = out[o].cpu().numpy().reshape(np.shape(ref[k]))
        err = np.abs(g - ref[k]).max()
        assert err <= TOL_G, (k, err)


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
           "grad_omega": np.array(g["grad_omega"]), "grad_rvdw": np.array(g["grad_rvdw"]),
           "grad_lattice": np.array(g["grad_lattice"])}
    out = _run(ctx, c)
    _compare(ctx, 64, out, ref)


@pytest.mark.parametrize("kgrid,kshift", [((4, 4, 4), (0.0, 0.0, 0.0)), ((2, 3, 1), (0.1, -0.05, 0.2))])
def test_library_monkhorst_pack_mesh(ctx, kgrid, kshift):
    """n_q = 0: the library builds the mesh (2r - n - 1)/(2n) + kshift per axis
    itself; the oracle gets the same fractions explicitly."""
    from paper_2308_03140_amd import torch_api as T
    _note("periodic library mesh %s k=%s shift=%s" % (ctx.precision, kgrid, kshift))
    c = gen.small_crystal(61, 3, kgrid=kgrid)
    qf = oracle.monkhorst_pack(*kgrid) + np.array(kshift)
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], qf, c["alpha0"], c["omega"], c["rvdw"],
                              c["beta"], c["a"])
    out = T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                     beta=c["beta"], a=c["a"], lattice=c["lattice"], kgrid=kgrid, kshift=kshift,
                     eigvals=True)
    _compare(ctx, 3, out, ref)
    tol = 1e-12 if ctx.precision == "fp64" else 1e-9
    assert np.abs(out["eigvals"].cpu().numpy() - ref["eigs"]).max() <= tol


def test_explicit_ewald_parameters(ctx):
    """gamma = 0.7 and 1.4 times the default, with R_c = 6/gamma and k_c =
    10 gamma: the Ewald split changes, the lattice sum does not (energy within
    1e-10 Ha/cell of the default split on the FP64 path); each run also
    matches the oracle given the same explicit parameters."""
    _note("periodic explicit ewald %s" % ctx.precision)
    c = gen.small_crystal(62, 4, kgrid=(2, 2, 2))
    g0, _, _ = oracle.ewald_defaults(c["lattice"])
    base = _run(ctx, c)["energy"].item()
    for s in (0.7, 1.4):
        g = s * g0
        ref = oracle.mbd_periodic(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c["omega"], c["rvdw"],
                                  c["beta"], c["a"], gamma=g, rc=6.0 / g, kc=10.0 * g)
        out = _run(ctx, c, ewald=(g, 6.0 / g, 10.0 * g))
        _compare(ctx, 4, out, ref)
        if ctx.precision == "fp64":
            assert abs(out["energy"].item() - base) <= 1e-10


@pytest.mark.parametrize("kgrid", [(2, 2, 1), (3, 1, 1)])
def test_energy_only_eigenvalues(ctx, kgrid):
    """Energy without gradients: on the FP64 path the eigenvalues come from
    the Sturm-count solver, which finds each pair of the real embedding once
    and writes it to both slots.  Energy and every eigenvalue of every q
    against the oracle."""
    _note("periodic energy only %s k=%s" % (ctx.precision, kgrid))
    c = gen.small_crystal(65, 5, kgrid=kgrid)
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c["omega"], c["rvdw"],
                              c["beta"], c["a"], gradients=False)
    out = _run(ctx, c, gradients=False, eigvals=True)
    torch.cuda.synchronize()
    assert abs(out["energy"].item() - ref["energy"]) / 5 <= TOL_E[ctx.precision]
    tol = 1e-12 if ctx.precision == "fp64" else 1e-9
    assert np.abs(out["eigvals"].cpu().numpy() - ref["eigs"]).max() <= tol


def _recip_counts(lattice, q_frac, kc):
    """Reciprocal vectors G with 0 < |G + q| < kc, per q point (geometry only)."""
    B = 2.0 * np.pi * np.linalg.inv(np.asarray(lattice)).T
    m = np.array([[x, y, z] for x in range(-8, 9) for y in range(-8, 9) for z in range(-8, 9)], float)
    G = m @ B
    out = []
    for qf in np.asarray(q_frac):
        k2 = np.sum((G + qf @ B) ** 2, axis=1)
        out.append(int(np.sum((k2 > 0.0) & (k2 < kc * kc))))
    return out


@pytest.mark.parametrize("kc_scale", [1e-4, 0.4])
def test_reciprocal_sphere_empty_and_ragged(ctx, kc_scale):
    """The reciprocal-space term runs as a product over one column per
    reciprocal vector of each q point's sphere.  k_c far below the shortest
    G + q leaves no column at any q (the embedding's product has no depth,
    the adjoint's reciprocal kernels are skipped); 0.4 times the default
    leaves the q points of a shifted mesh with different counts (padded
    columns).  Both against the oracle with the same explicit parameters
    (alpha0 scaled by 0.3, so that Q stays positive definite without most of
    the reciprocal sum)."""
    _note("periodic reciprocal sphere kc x %g %s" % (kc_scale, ctx.precision))
    c = gen.small_crystal(64, 4, kgrid=(2, 2, 2))
    c["q_frac"] = c["q_frac"] + np.array([0.1, 0.05, 0.0])
    c["alpha0"] = 0.3 * c["alpha0"]
    g0, rc0, kc0 = oracle.ewald_defaults(c["lattice"])
    kc = kc_scale * kc0
    counts = _recip_counts(c["lattice"], c["q_frac"], kc)
    if kc_scale < 1e-2:
        assert max(counts) == 0, counts
    else:
        assert 0 < min(counts) < max(counts), counts
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c["omega"], c["rvdw"],
                              c["beta"], c["a"], gamma=g0, rc=rc0, kc=kc)
    out = _run(ctx, c, ewald=(g0, rc0, kc))
    torch.cuda.synchronize()
    _compare(ctx, 4, out, ref)


def test_periodic_c6_input(ctx):
    from paper_2308_03140_amd import torch_api as T
    _note("periodic c6 input %s" % ctx.precision)
    c = gen.small_crystal(63, 3, kgrid=(2, 2, 1))
    c6 = 0.75 * c["omega"] * c["alpha0"] ** 2
    ref = oracle.mbd_periodic_c6(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c6, c["rvdw"],
                                 c["beta"], c["a"])
    out = T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c6, c["rvdw"],
                     beta=c["beta"], a=c["a"], lattice=c["lattice"], q_frac=c["q_frac"], param="c6")
    assert abs(out["energy"].item() - ref["energy"]) / 3 <= TOL_E[ctx.precision]
    assert np.abs(out["grad_alpha0"].cpu().numpy() - ref["grad_alpha0_c6"]).max() <= TOL_G
    assert np.abs(out["grad_omega"].cpu().numpy() - ref["grad_c6"]).max() <= TOL_G
    assert np.abs(out["grad_rvdw"].cpu().numpy() - ref["grad_rvdw"]).max() <= TOL_G


@pytest.mark.parametrize("kgrid,kshift", [((3, 3, 2), (0.0, 0.0, 0.0)), ((4, 2, 2), (0.125, 0.0, 0.0))])
def test_time_reversal_pairs_match_full_mesh(ctx, kgrid, kshift, monkeypatch):
    """With MBD_Q_PAIRS=1 the library evaluates one q point of each
    time-reversed pair (q, -q modulo the reciprocal lattice) with weight 2;
    by default, every mesh point.  Energy and every gradient agree between
    the two (FP64 to rounding), and with the oracle on the full mesh.  The
    shifted mesh pairs only some of its points."""
    from paper_2308_03140_amd import torch_api as T
    _note("periodic time reversal %s k=%s shift=%s" % (ctx.precision, kgrid, kshift))
    c = gen.small_crystal(64, 5, kgrid=kgrid)
    qf = oracle.monkhorst_pack(*kgrid) + np.array(kshift)
    ref = oracle.mbd_periodic(c["coords"], c["lattice"], qf, c["alpha0"], c["omega"], c["rvdw"],
                              c["beta"], c["a"])
    runs = []
    for pairs in ("1", "0"):
        monkeypatch.setenv("MBD_Q_PAIRS", pairs)
        runs.append(T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                               beta=c["beta"], a=c["a"], lattice=c["lattice"], q_frac=qf))
    torch.cuda.synchronize()
    for out in runs:
        _compare(ctx, 5, out, ref)
    if ctx.precision == "fp64":
        a, b = runs
        assert abs(a["energy"].item() - b["energy"].item()) <= 1e-12
        for k in ("grad_coords", "grad_alpha0", "grad_omega", "grad_rvdw", "grad_lattice"):
            assert (a[k] - b[k]).abs().max().item() <= 1e-11, k
