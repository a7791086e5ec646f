"""Writes gen/alpha_scale.json: the collapse-rule alpha0 factor per dense config.

Rule (applied before any timing): with mu_min the smallest eigenvalue of
alpha0^{1/2} T^lr alpha0^{1/2}, if 1 + mu_min <= 0.05 all alpha0 are scaled by
s = 0.9/|mu_min| (so 1 + s mu_min = 0.1); else s = 1.  mu_min is bracketed by
the oracle's Cholesky test (S - t I is positive definite iff t < mu_min), so
only the oracle is called.  For the N=8000 cluster (order 24000, where one
oracle factorisation takes a quarter of an hour) mu_min is first located by a
Lanczos iteration with full reorthogonalisation on the oracle's coupling
matrix (matrix-vector products only), then confirmed by one oracle Cholesky
test just below it.

    python gen/make_alpha_scale.py [names...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import gen  # noqa: E402
import oracle  # noqa: E402


def mu_min_bisect(S, lo=-4.0, hi=0.0, tol=2e-3):
    n = S.shape[0]
    eye = np.eye(n)
    assert oracle.is_positive_definite(S - lo * eye), "mu_min below the bracket"
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if oracle.is_positive_definite(S - mid * eye):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def mu_min_lanczos(S, iters=400, seed=0):
    """Smallest eigenvalue of symmetric S by Lanczos with full
    reorthogonalisation; returns the smallest Ritz value."""
    n = S.shape[0]
    rng = np.random.default_rng(seed)
    V = np.zeros((iters + 1, n))
    v = rng.standard_normal(n)
    V[0] = v / np.linalg.norm(v)
    alpha, beta = [], []
    for k in range(iters):
        w = S @ V[k]
        a = float(V[k] @ w)
        w -= a * V[k] + (beta[-1] * V[k - 1] if k > 0 else 0.0)
        w -= V[:k + 1].T @ (V[:k + 1] @ w)  # full reorthogonalisation
        b = float(np.linalg.norm(w))
        alpha.append(a)
        if b < 1e-12:
            break
        beta.append(b)
        V[k + 1] = w / b
    m = len(alpha)
    Tm = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    return float(np.linalg.eigvalsh(Tm)[0])


def scale_lanczos(c):
    S = oracle.coupling_matrix(c["coords"], c["alpha0"], c["rvdw"], c["beta"], c["a"])
    mu = mu_min_lanczos(S)
    # a Ritz value lies above mu_min; confirm with one oracle Cholesky that
    # mu_min > mu - 2e-3 (S - (mu - 2e-3) I positive definite)
    assert oracle.is_positive_definite(S - (mu - 2e-3) * np.eye(S.shape[0])), "Lanczos missed mu_min"
    return (0.9 / abs(mu) if 1.0 + mu <= 0.05 else 1.0), mu


def scale_for(c):
    S = oracle.coupling_matrix(c["coords"], c["alpha0"], c["rvdw"], c["beta"], c["a"])
    # quick test: no rescale needed if S + 0.95 I is positive definite
    if oracle.is_positive_definite(S + 0.95 * np.eye(S.shape[0])):
        return 1.0, None
    mu = mu_min_bisect(S)
    return 0.9 / abs(mu), mu


def main(names):
    path = os.path.join(HERE, "alpha_scale.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        t = time.time()
        if name == "cluster_n2000":
            s, mu = scale_for(gen.finite_cluster(2, 2000, gen.cube_side_for_density(2000)))
            table[name] = s
        elif name == "cluster_n8000":
            s, mu = scale_lanczos(gen.finite_cluster(5, 8000, gen.cube_side_for_density(8000)))
            table[name] = s
        elif name == "crystal_n64":
            c = gen.crystal_n64()
            mu = 1e300
            for qf in c["q_frac"]:
                q = qf @ (2 * np.pi * np.linalg.inv(c["lattice"]).T)
                S = oracle.assemble_periodic(c["coords"], c["lattice"], q, c["alpha0"],
                                             np.ones(len(c["omega"])), c["rvdw"], c["beta"], c["a"])
                S = S - np.eye(S.shape[0])
                mu = min(mu, float(oracle.jacobi_hermitian(S)[0]))
            table[name] = 0.9 / abs(mu) if 1.0 + mu <= 0.05 else 1.0
        elif name == "molecule_batch":
            mols = gen.molecule_batch()
            out = {}
            for m, c in enumerate(mols):
                s, mu = scale_for(c)
                if s != 1.0:
                    out[str(m)] = s
            table[name] = out
            mu = None
        else:
            raise SystemExit("unknown config " + name)
        print(name, "scale", table[name] if name != "molecule_batch" else len(table[name]),
              "mu_min", mu, "%.1fs" % (time.time() - t), flush=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cluster_n2000", "molecule_batch"])
