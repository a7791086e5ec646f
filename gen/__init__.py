"""Seeded synthetic MBD inputs shared by the oracle tests and the HIP path.

This module only draws random geometry and oscillator parameters; it holds
none of the method's arithmetic.  Positions are drawn in Angstrom and returned
in bohr (1 bohr = 0.529177210903 A, CODATA 2018).  Oscillator parameters are
drawn in atomic units:

  alpha0 ~ U[5, 50] bohr^3, omega ~ U[0.3, 0.9] Ha, R_vdW ~ U[3, 4.5] bohr,
  beta = 0.83, a = 6 (Fermi damping of the long-range MBD tensor)

drawn as N values each, in that order, after the geometry.

The dense configurations lie inside the dipole collapse region of the paper
(Sec. 2.1: negative eigenvalues of Q).  Their alpha0 are multiplied by one
factor per configuration, ``alpha_scale``, read from ``alpha_scale.json`` in
this directory; that file is written by ``make_alpha_scale.py`` (which calls
the oracle) and leaves positions, omega, R_vdW and matrix sizes unchanged.
"""
import json
import os

import numpy as np

BOHR_IN_ANGSTROM = 0.529177210903
BETA = 0.83
DAMP_A = 6.0
_HERE = os.path.dirname(os.path.abspath(__file__))


def _scale_table():
    path = os.path.join(_HERE, "alpha_scale.json")
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def alpha_scale(name):
    return float(_scale_table().get(name, 1.0))


def rsa_cube(rng, n_atoms, side_ang, dmin_ang=1.5, max_tries=10_000_000):
    """Random sequential addition in [0, side]^3 (Angstrom), min distance dmin."""
    pts = np.empty((n_atoms, 3))
    # cell list for O(1) neighbour checks
    ncell = max(1, int(side_ang // dmin_ang))
    csize = side_ang / ncell
    cells = {}
    k = 0
    tries = 0
    d2 = dmin_ang * dmin_ang
    while k < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA did not place all atoms")
        p = rng.uniform(0.0, side_ang, size=3)
        ci = tuple(np.minimum((p // csize).astype(int), ncell - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in cells.get((ci[0] + dx, ci[1] + dy, ci[2] + dz), ()):
                        if np.sum((pts[j] - p) ** 2) < d2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[k] = p
            cells.setdefault(ci, []).append(k)
            k += 1
    return pts


def draw_params(rng, n_atoms):
    alpha0 = rng.uniform(5.0, 50.0, size=n_atoms)
    omega = rng.uniform(0.3, 0.9, size=n_atoms)
    rvdw = rng.uniform(3.0, 4.5, size=n_atoms)
    return alpha0, omega, rvdw


def finite_cluster(seed, n_atoms, side_ang, name=None, rng=None):
    rng = rng if rng is not None else np.random.default_rng(seed)
    pos = rsa_cube(rng, n_atoms, side_ang) / BOHR_IN_ANGSTROM
    alpha0, omega, rvdw = draw_params(rng, n_atoms)
    s = alpha_scale(name) if name else 1.0
    return {"coords": pos, "alpha0": alpha0 * s, "omega": omega, "rvdw": rvdw,
            "beta": BETA, "a": DAMP_A, "alpha_scale": s, "lattice": None}


def cluster_n32(seed=1):
    """N=32 atoms in a 12 A cube, min pair distance 1.5 A."""
    return finite_cluster(seed, 32, 12.0, name="cluster_n32")


def cube_side_for_density(n_atoms, density_per_ang3=0.1):
    return (n_atoms / density_per_ang3) ** (1.0 / 3.0)


def cluster_n2000(seed=2):
    """N=2000 atoms at liquid-like density 0.1 atoms/A^3 (cube side 27.144 A)."""
    return finite_cluster(seed, 2000, cube_side_for_density(2000), name="cluster_n2000")


def cluster_n8000(seed=5):
    """N=8000 atoms at 0.1 atoms/A^3 (cube side 43.09 A)."""
    return finite_cluster(seed, 8000, cube_side_for_density(8000), name="cluster_n8000")


def cluster_dense(seed, n_atoms, name=None):
    """Generic cluster at 0.1 atoms/A^3 (used for parity cases between the sizes)."""
    return finite_cluster(seed, n_atoms, cube_side_for_density(n_atoms), name=name)


def random_lattice(rng):
    """Triclinic cell: lengths U[8,12] A, angles U[60,120] deg, a along x, b in xy;
    rejected while the volume is below half of a*b*c.  Returns rows = vectors (A)."""
    while True:
        la, lb, lc = rng.uniform(8.0, 12.0, size=3)
        al, be, ga = np.radians(rng.uniform(60.0, 120.0, size=3))
        cx = np.cos(be)
        cy = (np.cos(al) - np.cos(be) * np.cos(ga)) / np.sin(ga)
        cz2 = 1.0 - cx * cx - cy * cy
        if cz2 <= 0.0:
            continue
        A = np.array([[la, 0.0, 0.0],
                      [lb * np.cos(ga), lb * np.sin(ga), 0.0],
                      [lc * cx, lc * cy, lc * np.sqrt(cz2)]])
        if abs(np.linalg.det(A)) >= 0.5 * la * lb * lc:
            return A


def rsa_cell(rng, n_atoms, lattice_ang, dmin_ang=1.5, max_tries=1_000_000):
    """RSA in fractional coordinates with a minimum-image distance test."""
    frac = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    shifts = np.array([[x, y, z] for x in (-1, 0, 1) for y in (-1, 0, 1) for z in (-1, 0, 1)],
                      dtype=float)
    while k < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA in cell did not place all atoms")
        f = rng.uniform(0.0, 1.0, size=3)
        if k:
            df = frac[:k] - f
            df -= np.round(df)
            # check the nearest images explicitly (triclinic cells)
            cart = (df[:, None, :] + shifts[None, :, :]) @ lattice_ang
            if np.min(np.sum(cart ** 2, axis=-1)) < dmin_ang ** 2:
                continue
        frac[k] = f
        k += 1
    return frac


def monkhorst_pack(k1, k2, k3):
    """Uniform q grid offset from Gamma: f = (2r - n - 1)/(2n), r = 1..n per axis."""
    axes = [(2.0 * np.arange(1, k + 1) - k - 1) / (2.0 * k) for k in (k1, k2, k3)]
    return np.array([[x, y, z] for x in axes[0] for y in axes[1] for z in axes[2]])


def crystal_n64(seed=3, kgrid=(4, 4, 4)):
    """Periodic 64-atom triclinic cell with a Monkhorst-Pack q grid."""
    rng = np.random.default_rng(seed)
    lat_ang = random_lattice(rng)
    frac = rsa_cell(rng, 64, lat_ang)
    alpha0, omega, rvdw = draw_params(rng, 64)
    s = alpha_scale("crystal_n64")
    lat = lat_ang / BOHR_IN_ANGSTROM
    return {"coords": frac @ lat, "lattice": lat, "q_frac": monkhorst_pack(*kgrid),
            "alpha0": alpha0 * s, "omega": omega, "rvdw": rvdw, "beta": BETA, "a": DAMP_A,
            "alpha_scale": s, "kgrid": tuple(kgrid)}


def small_crystal(seed, n_atoms, kgrid=(2, 2, 2), side_scale=1.0):
    """Smaller periodic cell for fast parity cases (same recipe as crystal_n64)."""
    rng = np.random.default_rng(seed)
    lat_ang = random_lattice(rng) * side_scale
    frac = rsa_cell(rng, n_atoms, lat_ang)
    alpha0, omega, rvdw = draw_params(rng, n_atoms)
    lat = lat_ang / BOHR_IN_ANGSTROM
    return {"coords": frac @ lat, "lattice": lat, "q_frac": monkhorst_pack(*kgrid),
            "alpha0": alpha0, "omega": omega, "rvdw": rvdw, "beta": BETA, "a": DAMP_A,
            "alpha_scale": 1.0, "kgrid": tuple(kgrid)}


def molecule_batch(seed=4, n_mol=512, nmin=10, nmax=300):
    """Uneven batch: N_m ~ U{nmin..nmax}, cube side 12 (N_m/32)^(1/3) A (the
    density of the N=32 cluster); molecule m uses SeedSequence(seed).spawn."""
    ss = np.random.SeedSequence(seed)
    rng0 = np.random.default_rng(ss)
    sizes = rng0.integers(nmin, nmax + 1, size=n_mol)
    children = ss.spawn(n_mol)
    scales = _scale_table().get("molecule_batch", {})
    mols = []
    for m, (N, child) in enumerate(zip(sizes, children)):
        rng = np.random.default_rng(child)
        side = 12.0 * (N / 32.0) ** (1.0 / 3.0)
        pos = rsa_cube(rng, int(N), side) / BOHR_IN_ANGSTROM
        alpha0, omega, rvdw = draw_params(rng, int(N))
        s = float(scales.get(str(m), 1.0)) if isinstance(scales, dict) else 1.0
        mols.append({"coords": pos, "alpha0": alpha0 * s, "omega": omega, "rvdw": rvdw,
                     "beta": BETA, "a": DAMP_A, "alpha_scale": s, "lattice": None})
    return mols


def random_symmetric(seed, n, spread=1.0):
    """Dense random symmetric test matrix (eigen-solver unit tests)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) * spread
    return (X + X.T) * 0.5
