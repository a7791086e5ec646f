"""Frequency route (mbd_freq_evaluate): log-formula energy, renormalised
energy and many-body orders from the eigenvalues of
alpha(iu)^{1/2} T^lr alpha(iu)^{1/2} on the GPU, against the oracle on the
same frequency grid (so the quadrature is identical and the comparison is at
rounding level), plus the N=2000 cluster against its stored frequency-route
energy (48 points, the oracle's Cholesky route)."""
import json
import os
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10  # Ha per atom, every term


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2308_03140_amd import torch_api as T
    c = T.Context(0, "fp64")
    yield c
    c.close()


def _run(ctx, c, **kw):
    from paper_2308_03140_amd import torch_api as T
    return T.freq_evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                           beta=c["beta"], a=c["a"], **kw)


def _compare(N, out, ref, norder):
    for k in ("energy", "energy_gould"):
        assert abs(out[k].item() - ref[k]) / N <= TOL, (k, out[k].item(), ref[k])
    assert abs(out["min_one_plus_x"].item() - ref["min_one_plus_x"]) <= 1e-12
    o = out["orders"].cpu().numpy()
    assert np.abs(o - ref["orders"][:norder]).max() / N <= TOL, (o, ref["orders"])


@pytest.mark.parametrize("N", [2, 7, 32, 75])
def test_freq_finite(ctx, N):
    _note("freq finite N=%d" % N)
    c = gen.finite_cluster(500 + N, N, 12.0 * (N / 32.0) ** (1 / 3))
    ref = oracle.freq_terms(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"], nfreq=15,
                            norder=6)
    _compare(N, _run(ctx, c, n_freq=15, n_order=6), ref, 6)


@pytest.mark.parametrize("N,kgrid", [(1, (1, 1, 1)), (3, (2, 2, 2))])
def test_freq_periodic(ctx, N, kgrid):
    _note("freq periodic N=%d k=%s" % (N, kgrid))
    c = gen.small_crystal(90 + N, N, kgrid=kgrid)
    qf = c["q_frac"] if kgrid != (1, 1, 1) else np.zeros((1, 3))   # a Gamma-only mesh: E^(1) != 0
    ref = oracle.freq_terms(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"], nfreq=12,
                            norder=4, lattice=c["lattice"], q_frac=qf)
    out = _run(ctx, c, lattice=c["lattice"], q_frac=qf, n_freq=12, n_order=4)
    _compare(N, out, ref, 4)


def test_freq_crystal_n64(ctx):
    """The 64-atom cell at its real size (two q points, 15 frequencies: 30
    embedded matrices of order 384 in one batch)."""
    _note("freq crystal N=64")
    c = gen.crystal_n64()
    qf = np.array([[0.125, 0.125, 0.125], [0.375, -0.125, 0.125]])
    ref = oracle.freq_terms(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"], nfreq=15,
                            norder=4, lattice=c["lattice"], q_frac=qf)
    out = _run(ctx, c, lattice=c["lattice"], q_frac=qf, n_freq=15, n_order=4)
    _compare(64, out, ref, 4)


def test_freq_collapse(ctx):
    _note("freq collapse")
    c = {"coords": np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]]), "alpha0": np.array([20.0, 20.0]),
         "omega": np.array([0.5, 0.5]), "rvdw": np.array([1.0, 1.0]), "beta": 0.0, "a": 6.0}
    ref = oracle.freq_terms(c["coords"], c["alpha0"], c["omega"], c["rvdw"], 0.0, 6.0, nfreq=15, norder=3)
    out = _run(ctx, c, n_freq=15, n_order=3)
    assert np.isnan(out["energy"].item()) and np.isnan(ref["energy"])
    assert out["min_one_plus_x"].item() <= 0.0
    assert abs(out["energy_gould"].item() - ref["energy_gould"]) <= 1e-10 * abs(ref["energy_gould"])
    assert np.abs(out["orders"].cpu().numpy() - ref["orders"]).max() <= 1e-10 * np.abs(ref["orders"]).max()


def test_freq_log_formula_equals_eigen_route_gpu(ctx):
    """On the GPU alone: the log-formula energy (40 points) equals the
    eigenvalue-route energy of mbd_evaluate."""
    from paper_2308_03140_amd import torch_api as T
    _note("freq vs eigen route")
    c = gen.cluster_n32()
    e = T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                   beta=c["beta"], a=c["a"], gradients=False)["energy"].item()
    f = _run(ctx, c, n_freq=40, n_order=2)["energy"].item()
    assert abs(f - e) <= 1e-11 * abs(e)


def test_freq_n2000_golden(ctx):
    """N=2000 at the 48-point grid of the stored oracle value (same quadrature)."""
    _note("freq N=2000 golden (48 points)")
    with open(os.path.join(os.path.dirname(__file__), "golden", "cluster_n2000.json")) as f:
        ref = json.load(f)
    c = gen.cluster_n2000()
    out = _run(ctx, c, n_freq=48, n_order=2)
    dE = abs(out["energy"].item() - ref["energy"]) / 2000
    _note("  dE/N = %.3e" % dE)
    assert dE <= TOL
