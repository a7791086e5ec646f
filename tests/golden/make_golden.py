"""Writes the stored expected values of the large parity cases.  Calls only
the oracle (and the seeded input generators); run from the repository root:

    python tests/golden/make_golden.py crystal_n64 cluster_n2000

crystal_n64.json   64-atom triclinic cell, 4x4x4 Monkhorst-Pack mesh: energy
                   per cell, dE/dR, dE/dalpha0, dE/domega, dE/dRv, dE/dA from
                   the oracle's Jacobi route (Hermitian matrices by real
                   embedding).
cluster_n2000.json N=2000 cluster: energy by the frequency route (48-point
                   Gauss-Legendre grid, oracle Cholesky) and dE/dR, dE/dalpha0,
                   dE/domega of 8 seeded atoms from the rows of
                   Q^{-1/2} = (2/pi) int (Q + u^2)^{-1} du.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402


def crystal_n64():
    c = gen.crystal_n64()
    out = oracle.mbd_periodic(c["coords"], c["lattice"], c["q_frac"], c["alpha0"], c["omega"], c["rvdw"],
                              c["beta"], c["a"])
    return {"alpha_scale": c["alpha_scale"], "energy": out["energy"], "grad_R": out["grad_R"].tolist(),
            "grad_alpha0": out["grad_alpha0"].tolist(), "grad_omega": out["grad_omega"].tolist(),
            "grad_rvdw": out["grad_rvdw"].tolist(), "grad_lattice": out["grad_lattice"].tolist(),
            "eig_min": float(out["eigs"].min())}


def cluster_n2000():
    c = gen.cluster_n2000()
    atoms = sorted(np.random.default_rng(22).choice(2000, 8, replace=False).tolist())
    out = oracle.mbd_finite_freq(c["coords"], c["alpha0"], c["omega"], c["rvdw"], c["beta"], c["a"],
                                 npts=48, sample_atoms=atoms)
    return {"alpha_scale": c["alpha_scale"], "energy": out["energy"], "atoms": atoms,
            "grad_R_sample": out["grad_R_sample"].tolist(),
            "grad_alpha0_sample": out["grad_alpha0_sample"].tolist(),
            "grad_omega_sample": out["grad_omega_sample"].tolist(), "route": "frequency, 48 points"}


if __name__ == "__main__":
    for name in sys.argv[1:] or ["crystal_n64", "cluster_n2000"]:
        t = time.time()
        res = globals()[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(res, f, indent=1)
        print(name, "done in %.1fs" % (time.time() - t), flush=True)
