"""GPU eigensolver of the MBD path (Householder reduction + divide and conquer +
back-transform) against the oracle's Jacobi solver, through the C ABI."""
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


def _check(A, w, Z, tol):
    nrm = max(1.0, np.abs(A).sum(axis=1).max())
    ref = oracle.jacobi(A, vectors=False)
    assert np.abs(w - ref).max() <= tol * nrm, ("eigenvalues", np.abs(w - ref).max())
    if Z is not None:
        res = np.abs(A @ Z - Z * w).max()
        orth = np.abs(Z.T @ Z - np.eye(A.shape[0])).max()
        assert res <= tol * nrm, ("residual", res)
        assert orth <= tol * max(1, A.shape[0] / 100), ("orthogonality", orth)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 63, 64, 65, 97, 130, 300])
def test_eigh_fp64_random(ctx, n):
    from paper_2308_03140_amd import torch_api as T
    _note("eigh fp64 n=%d" % n)
    A = gen.random_symmetric(1000 + n, n)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda"))
    torch.cuda.synchronize()
    _check(A, w.cpu().numpy(), Z.cpu().numpy(), 1e-12)


@pytest.mark.parametrize("n", [2, 40, 129])
def test_eigh_fp32_random(ctx, n):
    from paper_2308_03140_amd import torch_api as T
    _note("eigh fp32 n=%d" % n)
    A = gen.random_symmetric(2000 + n, n)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda", dtype=torch.float32))
    torch.cuda.synchronize()
    _check(A, w.double().cpu().numpy(), Z.double().cpu().numpy(), 2e-5)


# orders around the hand-over from the panel path to the LDS tail kernel (the
# last <= 256 columns in FP32, <= 192 in FP64, from a 32-column panel boundary):
# whole matrix in the tail, one panel then the tail, two panels then the tail
@pytest.mark.parametrize("n", [256, 257, 289, 320])
def test_eigh_fp32_tail_boundary(ctx, n):
    from paper_2308_03140_amd import torch_api as T
    _note("eigh fp32 tail boundary n=%d" % n)
    A = gen.random_symmetric(3000 + n, n)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda", dtype=torch.float32))
    torch.cuda.synchronize()
    _check(A, w.double().cpu().numpy(), Z.double().cpu().numpy(), 2e-5)


@pytest.mark.parametrize("n", [192, 193, 225])
def test_eigh_fp64_tail_boundary(ctx, n):
    from paper_2308_03140_amd import torch_api as T
    _note("eigh fp64 tail boundary n=%d" % n)
    A = gen.random_symmetric(4000 + n, n)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda"))
    torch.cuda.synchronize()
    _check(A, w.cpu().numpy(), Z.cpu().numpy(), 1e-12)


def test_eigh_degenerate_cases(ctx):
    from paper_2308_03140_amd import torch_api as T
    _note("eigh degenerate")
    # exact multiplicities, zero off-diagonals (splitting)
    A = np.diag([1.0, 1.0, 2.0, 2.0, 2.0, 3.0, 0.5, 0.5])
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda"))
    _check(A, w.cpu().numpy(), Z.cpu().numpy(), 1e-13)
    # real embedding of a Hermitian matrix: every eigenvalue twice
    rng = np.random.default_rng(3)
    n = 48
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = 0.5 * (X + X.conj().T)
    E = np.block([[H.real, -H.imag], [H.imag, H.real]])
    w, Z = T.eigh(ctx, torch.tensor(E, device="cuda"))
    _check(E, w.cpu().numpy(), Z.cpu().numpy(), 1e-12)
    # known spectrum with clusters
    lam = np.repeat(np.linspace(-1, 1, 20), 5)
    Qm, _ = np.linalg.qr(rng.standard_normal((100, 100)))
    A = (Qm * lam) @ Qm.T
    A = 0.5 * (A + A.T)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda"))
    _check(A, w.cpu().numpy(), Z.cpu().numpy(), 1e-12)


def test_eigh_batched(ctx):
    from paper_2308_03140_amd import torch_api as T
    _note("eigh batched 3 x 70")
    As = np.stack([gen.random_symmetric(77 + b, 70) for b in range(3)])
    w, Z = T.eigh(ctx, torch.tensor(As, device="cuda"))
    for b in range(3):
        _check(As[b], w[b].cpu().numpy(), Z[b].cpu().numpy(), 1e-12)


def test_autotune_table_roundtrip(tmp_path):
    from paper_2308_03140_amd import torch_api as T
    _note("autotune")
    path = str(tmp_path / "tune.json")
    for prec, dt, tol in (("fp64", torch.float64, 1e-12), ("fp32_refined", torch.float32, 2e-5)):
        c = T.Context(0, prec)
        c.autotune([150, 400], path)
        c.close()
        c2 = T.Context(0, prec)
        c2.load_tuning(path)
        A = gen.random_symmetric(99, 400)
        w, Z = T.eigh(c2, torch.tensor(A, device="cuda", dtype=dt))
        _check(A, w.double().cpu().numpy(), Z.double().cpu().numpy(), tol)
        c2.close()
    import json
    tab = json.load(open(path))
    assert set(tab) == {"fp64", "fp32"} and "400" in tab["fp32"]
    # each order maps to [upper-range target, lower-range target, GEMM tile]
    assert all(len(v) == 3 and min(v[:2]) > 0 and v[2] in (64, 128) for p in tab.values() for v in p.values())
    # a table may also give one target for both ranges, or two targets with
    # the GEMM tile left to the order; both tiles are usable at any order
    for tab in ({"fp64": {"400": 768}, "fp32": {"400": [1536, 512]}},
                {"fp64": {"400": [768, 512, 128]}, "fp32": {"400": [1536, 512, 64]}},
                {"fp64": {"400": [768, 512, 64]}, "fp32": {"400": [1536, 512, 128]}}):
        with open(path, "w") as f:
            json.dump(tab, f)
        for prec, dt, tol in (("fp64", torch.float64, 1e-12), ("fp32_refined", torch.float32, 2e-5)):
            c3 = T.Context(0, prec)
            c3.load_tuning(path)
            A = gen.random_symmetric(98, 400)
            w, Z = T.eigh(c3, torch.tensor(A, device="cuda", dtype=dt))
            _check(A, w.double().cpu().numpy(), Z.double().cpu().numpy(), tol)
            c3.close()
    # a tile that is neither 64 nor 128 is refused
    with open(path, "w") as f:
        json.dump({"fp64": {"400": [768, 512, 96]}, "fp32": {}}, f)
    c4 = T.Context(0, "fp64")
    with pytest.raises(Exception):
        c4.load_tuning(path)
    c4.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_gemm_tile_choice_same_results(tmp_path, prec):
    """An evaluation (energy and every gradient) at order 3N = 600 through a
    tuning table that sets the general GEMM's tile to 64, then to 128: the
    two must agree to rounding (the products differ only in blocking)."""
    import json
    from paper_2308_03140_amd import torch_api as T
    _note("gemm tile choice %s" % prec)
    c = gen.finite_cluster(611, 200, 12.0 * (200 / 32.0) ** (1.0 / 3.0))
    key = "fp64" if prec == "fp64" else "fp32"
    out = []
    for ts in (64, 128):
        path = str(tmp_path / ("tile%d.json" % ts))
        with open(path, "w") as f:
            json.dump({key: {"600": [1536, 1536, ts]}}, f)
        ctx = T.Context(0, prec)
        try:
            ctx.load_tuning(path)
            out.append(T.evaluate(ctx, torch.tensor(c["coords"], device="cuda"), c["alpha0"], c["omega"], c["rvdw"],
                                  beta=c["beta"], a=c["a"]))
            torch.cuda.synchronize()
        finally:
            ctx.close()
    a, b = out
    # FP32+refine: the tile also changes the FP32 products, so the two runs
    # agree to the refined path's own bounds, not to FP64 rounding
    tol_e, tol_g = (1e-12, 1e-9) if prec == "fp64" else (1e-7, 1e-6)
    assert abs(a["energy"].item() - b["energy"].item()) <= tol_e * 200
    for k in ("grad_coords", "grad_alpha0", "grad_omega", "grad_rvdw"):
        assert (a[k] - b[k]).abs().max().item() <= tol_g, k


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 3e-5)])
def test_eigh_clustered_n1100(ctx, dtype, tol):
    """Order 1100: merges of 1024 and 2048 entries deflate in the LDS kernel
    (several entries per thread, rotation chains from 8-fold clusters and
    negligible z components), and the back-transform splits V^T X over three
    512-row chunks.  Residual and orthogonality are checked directly, the
    eigenvalues against LAPACK's (numpy) solver."""
    from paper_2308_03140_amd import torch_api as T
    _note("eigh clustered n=1100 %s" % dtype)
    rng = np.random.default_rng(1100)
    n = 1100
    lam = np.concatenate([np.repeat(np.linspace(-2.0, 2.0, 100), 8), rng.uniform(-2.0, 2.0, n - 800)])
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Qm * lam) @ Qm.T
    A = 0.5 * (A + A.T)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda", dtype=getattr(torch, dtype)))
    torch.cuda.synchronize()
    w = w.double().cpu().numpy()
    Z = Z.double().cpu().numpy()
    nrm = np.abs(A).sum(axis=1).max()
    assert np.abs(w - np.linalg.eigvalsh(A)).max() <= tol * nrm
    assert np.abs(A @ Z - Z * w).max() <= tol * nrm
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= tol * n / 100


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("n", [1, 2, 7, 64, 150, 257, 700])
def test_eigh_values_only(ctx, dtype, n):
    """No eigenvectors asked for: the Householder reduction followed by the
    Sturm-count multisection (no divide and conquer, no back-transform)."""
    from paper_2308_03140_amd import torch_api as T
    _note("eigh values only %s n=%d" % (dtype, n))
    A = gen.random_symmetric(5000 + n, n)
    w, Z = T.eigh(ctx, torch.tensor(A, device="cuda", dtype=getattr(torch, dtype)), vectors=False)
    assert Z is None
    tol = 1e-12 if dtype == "float64" else 2e-5
    _check(A, w.double().cpu().numpy(), None, tol)


def test_eigh_values_only_structured(ctx):
    """Exact multiplicities and zero couplings (a split tridiagonal), the real
    embedding of a Hermitian matrix (every value twice), and a batch."""
    from paper_2308_03140_amd import torch_api as T
    _note("eigh values only structured")
    A = np.diag([1.0, 1.0, 2.0, 2.0, 2.0, 3.0, 0.5, 0.5])
    w, _ = T.eigh(ctx, torch.tensor(A, device="cuda"), vectors=False)
    _check(A, w.cpu().numpy(), None, 1e-14)
    rng = np.random.default_rng(4)
    n = 48
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = 0.5 * (X + X.conj().T)
    E = np.block([[H.real, -H.imag], [H.imag, H.real]])
    w, _ = T.eigh(ctx, torch.tensor(E, device="cuda"), vectors=False)
    _check(E, w.cpu().numpy(), None, 1e-12)
    As = np.stack([gen.random_symmetric(88 + b, 90) for b in range(3)])
    w, _ = T.eigh(ctx, torch.tensor(As, device="cuda"), vectors=False)
    for b in range(3):
        _check(As[b], w[b].cpu().numpy(), None, 1e-12)


_PATH_CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import gen
import oracle
from paper_2308_03140_amd import torch_api as T
out = []
for dtype, tol in (("float64", 1e-12), ("float32", 3e-5)):
    ctx = T.Context(0, "fp64")
    for n in (300, 700):
        A = gen.random_symmetric(7000 + n, n)
        w, Z = T.eigh(ctx, torch.tensor(A, device="cuda", dtype=getattr(torch, dtype)))
        torch.cuda.synchronize()
        w = w.double().cpu().numpy(); Z = Z.double().cpu().numpy()
        nrm = max(1.0, np.abs(A).sum(axis=1).max())
        ev = np.abs(w - oracle.jacobi(A, vectors=False)).max() / nrm
        res = np.abs(A @ Z - Z * w).max() / nrm
        orth = np.abs(Z.T @ Z - np.eye(n)).max()
        ok = ev <= tol and res <= tol and orth <= tol * max(1, n / 100)
        print("%s n=%d ev=%.2e res=%.2e orth=%.2e %s" % (dtype, n, ev, res, orth, "ok" if ok else "FAIL"), flush=True)
        out.append(ok)
    ctx.close()
sys.exit(0 if all(out) else 1)
"""


_WG_CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import gen
from paper_2308_03140_amd import torch_api as T
out = []
for dtype, tol in (("float64", 1e-12), ("float32", 3e-5)):
    ctx = T.Context(0, "fp64")
    for n, nb in ((1024, 8), (450, 9), (257, 9), (193, 9)):
        As = np.stack([gen.random_symmetric(6000 + 31 * n + b, n) for b in range(nb)])
        w, Z = T.eigh(ctx, torch.tensor(As, device="cuda", dtype=getattr(torch, dtype)))
        torch.cuda.synchronize()
        w = w.double().cpu().numpy(); Z = Z.double().cpu().numpy()
        for b in range(nb):
            A = As[b].astype(np.float32).astype(np.float64) if dtype == "float32" else As[b]
            nrm = max(1.0, np.abs(A).sum(axis=1).max())
            ev = np.abs(w[b] - np.linalg.eigvalsh(A)).max() / nrm
            res = np.abs(A @ Z[b] - Z[b] * w[b]).max() / nrm
            orth = np.abs(Z[b].T @ Z[b] - np.eye(n)).max()
            ok = ev <= tol and res <= tol and orth <= tol * max(1, n / 100)
            out.append(ok)
        print("%s n=%d nb=%d %s" % (dtype, n, nb, "ok" if all(out) else "FAIL"), flush=True)
    ctx.close()
sys.exit(0 if all(out) else 1)
"""


@pytest.mark.parametrize("min_batch", [0, 8])
def test_eigh_one_workgroup_path_choice(min_batch):
    """The batch-size threshold of the one-workgroup-per-matrix reduction
    set through MBD_SYTRD_WG_MIN_BATCH (read once per process, hence the
    child process): 8 sends these batches of 8 and 9 matrices through it in
    both precisions (by default only FP64 batches of 256 or more take it),
    0 sends every batch through the per-column launches."""
    import os
    import subprocess
    _note("one-workgroup path, min batch %d" % min_batch)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MBD_SYTRD_WG_MIN_BATCH=str(min_batch))
    r = subprocess.run([sys.executable, "-c", _WG_CHILD, root], env=env, capture_output=True, text=True,
                       timeout=110)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 3e-5)])
@pytest.mark.parametrize("n,nb", [(1024, 8), (450, 10), (257, 9), (193, 12)])
def test_eigh_one_workgroup_batches(dtype, tol, n, nb):
    """Batches of 8 to 12 matrices of order <= 1024 through the default
    (per-column) reduction: the largest order the one-workgroup path would
    take, orders whose last panel ends just past the LDS tail's start (257 in
    FP32, 193 in FP64: one panel) and one in between, each matrix checked by
    residual, orthogonality and its eigenvalues against LAPACK's (numpy)."""
    from paper_2308_03140_amd import torch_api as T
    _note("eigh one-workgroup batch n=%d nb=%d %s" % (n, nb, dtype))
    c = T.Context(0, "fp64" if dtype == "float64" else "fp32_refined")
    try:
        As = np.stack([gen.random_symmetric(5000 + 37 * n + b, n) for b in range(nb)])
        dt = torch.float64 if dtype == "float64" else torch.float32
        w, Z = T.eigh(c, torch.tensor(As, device="cuda", dtype=dt))
        w = w.double().cpu().numpy()
        Z = Z.double().cpu().numpy()
    finally:
        c.close()
    for b in range(nb):
        A = As[b].astype(np.float32).astype(np.float64) if dtype == "float32" else As[b]
        nrm = max(1.0, np.abs(A).sum(axis=1).max())
        assert np.abs(w[b] - np.linalg.eigvalsh(A)).max() <= tol * nrm, b
        assert np.abs(A @ Z[b] - Z[b] * w[b]).max() <= tol * nrm, b
        assert np.abs(Z[b].T @ Z[b] - np.eye(n)).max() <= tol * max(1, n / 100), b


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("nb", [3, 9])
def test_eigh_nonfinite_input_reported(dtype, nb):
    """A NaN in one matrix of a batch (per-column path: 3 matrices; one
    workgroup per matrix: 9) is reported as an invalid argument, the
    tridiagonal solvers having seen zeros instead of it; the same context
    then solves a clean batch correctly."""
    from paper_2308_03140_amd import torch_api as T
    _note("eigh non-finite input nb=%d %s" % (nb, dtype))
    n = 300
    dt = torch.float64 if dtype == "float64" else torch.float32
    tol = 1e-12 if dtype == "float64" else 3e-5
    c = T.Context(0, "fp64" if dtype == "float64" else "fp32_refined")
    try:
        As = np.stack([gen.random_symmetric(7100 + b, n) for b in range(nb)])
        bad = As.copy()
        bad[1, 17, 5] = bad[1, 5, 17] = np.nan
        with pytest.raises(Exception):
            T.eigh(c, torch.tensor(bad, device="cuda", dtype=dt))
        w, Z = T.eigh(c, torch.tensor(As, device="cuda", dtype=dt))
        w = w.double().cpu().numpy()
        Z = Z.double().cpu().numpy()
    finally:
        c.close()
    for b in range(nb):
        A = As[b].astype(np.float32).astype(np.float64) if dtype == "float32" else As[b]
        nrm = max(1.0, np.abs(A).sum(axis=1).max())
        assert np.abs(w[b] - np.linalg.eigvalsh(A)).max() <= tol * nrm, b
        assert np.abs(A @ Z[b] - Z[b] * w[b]).max() <= tol * nrm, b


@pytest.mark.parametrize("max_order", [0, 1000000])
def test_eigh_reduction_paths(max_order):
    """Both per-column paths of the reduction in both precisions: the fused
    launch everywhere (FP64 included, which the default never fuses) and the
    SYMV + finish launches everywhere (FP32 included), chosen through the
    library's MBD_SYTRD_FUSED_MAXN override, which is read once per process,
    hence the child process."""
    import os
    import subprocess
    _note("reduction paths, fused max order %d" % max_order)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MBD_SYTRD_FUSED_MAXN=str(max_order))
    r = subprocess.run([sys.executable, "-c", _PATH_CHILD, root], env=env, capture_output=True, text=True,
                       timeout=110)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
