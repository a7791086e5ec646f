"""Plain FP64 CPU oracle for the MBD hot path (ctypes wrapper of mbd_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP path in ``paper_2308_03140_amd`` and never imports it.

Every function follows the paper (Hermann et al., arXiv:2308.03140); see the
header of ``mbd_oracle.c`` for the equations and the readings taken where the
paper is ambiguous.  Units: bohr, Hartree.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbd_oracle.c")
_LIB = os.path.join(_HERE, "libmbd_oracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def build(force=True):
    """Compile the oracle with gcc (OpenMP, -O2, strict IEEE: no -ffast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_jacobi.restype = ctypes.c_int
        lib.orc_jacobi_hermitian.restype = ctypes.c_int
        lib.orc_mbd_finite.restype = ctypes.c_int
        lib.orc_assemble_periodic.restype = ctypes.c_int
        lib.orc_mbd_periodic.restype = ctypes.c_int
        lib.orc_mbd_finite_freq.restype = ctypes.c_int
        lib.orc_min_coupling_eig.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _arr(x, shape=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class CollapseError(RuntimeError):
    """Q has a non-positive eigenvalue (dipole collapse, paper Sec. 2.1)."""


def _check(rc, what):
    if rc == 2:
        raise CollapseError(what + ": Q is not positive definite (dipole collapse)")
    if rc == 3:
        raise RuntimeError(what + ": Jacobi did not converge")
    if rc != 0:
        raise ValueError(what + ": invalid argument (code %d)" % rc)


def assemble_finite(R, alpha0, omega, rvdw, beta=0.83, a=6.0):
    """Q of eq:q-matrix, finite system, n x n with n = 3N."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    Q = np.empty((3 * N, 3 * N))
    _load().orc_assemble_finite(N, _p(R), _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)),
                                ctypes.c_double(beta), ctypes.c_double(a), _p(Q))
    return Q


def jacobi(A, vectors=True):
    """Eigen-decomposition of a real symmetric matrix by cyclic Jacobi."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n)) if vectors else None
    sw = _load().orc_jacobi(n, _p(A), _p(w), _p(V))
    if sw < 0:
        raise RuntimeError("Jacobi did not converge")
    return (w, V) if vectors else w


def jacobi_hermitian(A, vectors=False):
    """Eigenvalues of a Hermitian matrix via the 2n real embedding (each value twice)."""
    A = np.asarray(A)
    n = A.shape[0]
    re = _arr(A.real); im = _arr(A.imag)
    w = np.empty(2 * n)
    V = np.empty((2 * n, 2 * n)) if vectors else None
    sw = _load().orc_jacobi_hermitian(n, _p(re), _p(im), _p(w), _p(V))
    if sw < 0:
        raise RuntimeError("Jacobi did not converge")
    return (w, V) if vectors else w


def mbd_finite(R, alpha0, omega, rvdw, beta=0.83, a=6.0, gradients=True):
    """Finite MBD energy (eq:mbd-energy) and gradients.

    Returns dict with energy, eigs and (if gradients) grad_R [N,3], grad_alpha0,
    grad_omega, grad_rvdw [N].
    """
    R = _arr(R, (-1, 3)); N = R.shape[0]
    E = np.zeros(1); eigs = np.empty(3 * N)
    g = {k: (np.empty(s) if gradients else None) for k, s in
         (("grad_R", (N, 3)), ("grad_alpha0", N), ("grad_omega", N), ("grad_rvdw", N))}
    rc = _load().orc_mbd_finite(N, _p(R), _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)),
                                ctypes.c_double(beta), ctypes.c_double(a), _p(E),
                                _p(g["grad_R"]), _p(g["grad_alpha0"]), _p(g["grad_omega"]),
                                _p(g["grad_rvdw"]), _p(eigs))
    _check(rc, "mbd_finite")
    out = {"energy": float(E[0]), "eigs": eigs}
    if gradients:
        out.update(g)
    return out


def mbd_finite_c6(R, alpha0, c6, rvdw, beta=0.83, a=6.0):
    """Finite MBD with C6 input: omega = 4 C6 / (3 alpha0^2) (eq:osc-param)."""
    alpha0 = _arr(alpha0); c6 = _arr(c6)
    omega = 4.0 * c6 / (3.0 * alpha0 ** 2)
    out = mbd_finite(R, alpha0, omega, rvdw, beta, a, gradients=True)
    dEdw = out["grad_omega"]
    out["grad_alpha0_c6"] = out["grad_alpha0"] - 2.0 * omega / alpha0 * dEdw
    out["grad_c6"] = dEdw * omega / c6
    return out


def ewald_defaults(lattice):
    """gamma = 2.5/Omega^(1/3), Rc = 6/gamma, kc = 10 gamma (paper Sec. 3.3)."""
    L = _arr(lattice, (3, 3))
    g = ctypes.c_double(); rc = ctypes.c_double(); kc = ctypes.c_double()
    _load().orc_ewald_defaults(_p(L), ctypes.byref(g), ctypes.byref(rc), ctypes.byref(kc))
    return g.value, rc.value, kc.value


def assemble_periodic(R, lattice, q_cart, alpha0, omega, rvdw, beta=0.83, a=6.0,
                      gamma=None, rc=None, kc=None):
    """Complex Hermitian Q(q) of eq:q-matrix with the Ewald-summed T^lr(q)."""
    R = _arr(R, (-1, 3)); N = R.shape[0]; L = _arr(lattice, (3, 3))
    g0, rc0, kc0 = ewald_defaults(L)
    gamma = g0 if gamma is None else gamma
    rc = rc0 if rc is None else rc
    kc = kc0 if kc is None else kc
    Qr = np.empty((3 * N, 3 * N)); Qi = np.empty((3 * N, 3 * N))
    rcode = _load().orc_assemble_periodic(N, _p(R), _p(L), _p(_arr(q_cart)), ctypes.c_double(gamma),
                                          ctypes.c_double(rc), ctypes.c_double(kc),
                                          _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)),
                                          ctypes.c_double(beta), ctypes.c_double(a), _p(Qr), _p(Qi))
    _check(rcode, "assemble_periodic")
    return Qr + 1j * Qi


def mbd_periodic(R, lattice, q_frac, alpha0, omega, rvdw, beta=0.83, a=6.0,
                 gamma=None, rc=None, kc=None, gradients=True):
    """Periodic MBD energy per cell (eq:brillouin-int, mean over q) and gradients."""
    R = _arr(R, (-1, 3)); N = R.shape[0]; L = _arr(lattice, (3, 3))
    qf = _arr(q_frac, (-1, 3)); nq = qf.shape[0]
    g0, rc0, kc0 = ewald_defaults(L)
    gamma = g0 if gamma is None else gamma
    rc = rc0 if rc is None else rc
    kc = kc0 if kc is None else kc
    E = np.zeros(1); eigs = np.empty((nq, 3 * N))
    gR = np.empty((N, 3)) if gradients else None
    ga = np.empty(N) if gradients else None
    gw = np.empty(N) if gradients else None
    gv = np.empty(N) if gradients else None
    gl = np.empty((3, 3)) if gradients else None
    rcode = _load().orc_mbd_periodic(N, _p(R), _p(L), nq, _p(qf), ctypes.c_double(gamma),
                                     ctypes.c_double(rc), ctypes.c_double(kc),
                                     _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)),
                                     ctypes.c_double(beta), ctypes.c_double(a), _p(E),
                                     _p(gR), _p(ga), _p(gw), _p(gv), _p(gl), _p(eigs))
    _check(rcode, "mbd_periodic")
    out = {"energy": float(E[0]), "eigs": eigs}
    if gradients:
        out.update(grad_R=gR, grad_alpha0=ga, grad_omega=gw, grad_rvdw=gv, grad_lattice=gl)
    return out


def mbd_periodic_c6(R, lattice, q_frac, alpha0, c6, rvdw, beta=0.83, a=6.0, **kw):
    """Periodic MBD with C6 input: omega = 4 C6 / (3 alpha0^2) (eq:osc-param);
    the alpha0 gradient at fixed C6 and the C6 gradient by the chain rule."""
    alpha0 = _arr(alpha0); c6 = _arr(c6)
    omega = 4.0 * c6 / (3.0 * alpha0 ** 2)
    out = mbd_periodic(R, lattice, q_frac, alpha0, omega, rvdw, beta, a, gradients=True, **kw)
    dEdw = out["grad_omega"]
    out["grad_alpha0_c6"] = out["grad_alpha0"] - 2.0 * omega / alpha0 * dEdw
    out["grad_c6"] = dEdw * omega / c6
    return out


def gauss_legendre(n):
    x = np.empty(n); w = np.empty(n)
    _load().orc_gauss_legendre(n, _p(x), _p(w))
    return x, w


def mbd_finite_freq(R, alpha0, omega, rvdw, beta=0.83, a=6.0, npts=30, sample_atoms=()):
    """Finite MBD energy by the frequency route (eq:log-formula), optionally with
    dE/dR, dE/dalpha0 and dE/domega of the listed atoms from
    Q^{-1/2} = (2/pi) int (Q + u^2)^{-1} du."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    atoms = np.ascontiguousarray(np.asarray(sample_atoms, dtype=np.int32))
    ns = atoms.size
    E = np.zeros(1)
    g = np.zeros((max(ns, 1), 3))
    ga = np.zeros(max(ns, 1))
    gw = np.zeros(max(ns, 1))
    rc = _load().orc_mbd_finite_freq(N, _p(R), _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)),
                                     ctypes.c_double(beta), ctypes.c_double(a), npts, _p(E), ns,
                                     atoms.ctypes.data_as(_I) if ns else None, _p(g), _p(ga), _p(gw))
    _check(rc, "mbd_finite_freq")
    return {"energy": float(E[0]), "grad_R_sample": g[:ns], "grad_alpha0_sample": ga[:ns],
            "grad_omega_sample": gw[:ns]}


def ts(R, alpha0, omega, rvdw, sR, a=20.0, lattice=None, gamma=None, rc=None, kc=None):
    """Pairwise (TS) dispersion energy (eq:pairwise, Fermi damping a = 20) and
    its gradients; periodic (energy per cell) when a lattice is given, by the
    Ewald split of eq:ts-ewald plus the real-space damping correction."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    L = None
    if lattice is not None:
        L = _arr(lattice, (3, 3))
        g0, rc0, kc0 = ewald_defaults(L)
        gamma = g0 if gamma is None else gamma
        rc = rc0 if rc is None else rc
        kc = kc0 if kc is None else kc
    E = np.zeros(1); gR = np.empty((N, 3)); ga = np.empty(N); gw = np.empty(N); gv = np.empty(N)
    lib = _load()
    lib.orc_ts.restype = ctypes.c_int
    rcode = lib.orc_ts(N, _p(R), _p(L), ctypes.c_double(gamma or 0.0), ctypes.c_double(rc or 0.0),
                       ctypes.c_double(kc or 0.0), _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)),
                       ctypes.c_double(sR), ctypes.c_double(a), _p(E), _p(gR), _p(ga), _p(gw), _p(gv))
    _check(rcode, "ts")
    return {"energy": float(E[0]), "grad_R": gR, "grad_alpha0": ga, "grad_omega": gw, "grad_rvdw": gv}


def freq_terms(R, alpha0, omega, rvdw, beta=0.83, a=6.0, nfreq=15, norder=6, lattice=None, q_frac=None,
               gamma=None, rc=None, kc=None):
    """Frequency-route energies (Sec. 2.5): E by eq:log-formula, the
    renormalised energy of eq:gould-norm, min(1 + x_k), and the many-body
    orders E^(1..norder) of eq:rpa, from the eigenvalues x_k of
    alpha(iu)^{1/2} T^lr alpha(iu)^{1/2} on an nfreq-point frequency grid."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    L = None; qf = None; nq = 1
    if lattice is not None:
        L = _arr(lattice, (3, 3))
        qf = _arr(q_frac, (-1, 3)); nq = qf.shape[0]
        g0, rc0, kc0 = ewald_defaults(L)
        gamma = g0 if gamma is None else gamma
        rc = rc0 if rc is None else rc
        kc = kc0 if kc is None else kc
    t = np.empty(3 + norder)
    lib = _load()
    lib.orc_mbd_freq_terms.restype = ctypes.c_int
    rcode = lib.orc_mbd_freq_terms(N, _p(R), _p(L), nq, _p(qf), ctypes.c_double(gamma or 0.0),
                                   ctypes.c_double(rc or 0.0), ctypes.c_double(kc or 0.0), _p(_arr(alpha0)),
                                   _p(_arr(omega)), _p(_arr(rvdw)), ctypes.c_double(beta), ctypes.c_double(a),
                                   nfreq, norder, _p(t))
    _check(rcode, "freq_terms")
    return {"energy": t[0], "energy_gould": t[1], "min_one_plus_x": t[2], "orders": t[3:]}


def dipole_gg(r, s):
    """T^GG of eq:tgg and its r-derivative for s = sqrt(sigma_i^2 + sigma_j^2)."""
    T = np.empty(9); dT = np.empty(27)
    _load().orc_dipole_gg(_p(_arr(r)), ctypes.c_double(s), _p(T), _p(dT))
    return T.reshape(3, 3), dT.reshape(3, 3, 3)


def scs(R, alpha0, omega, rvdw, beta=0.83, a=6.0, nfreq=15):
    """Self-consistent screening (eq:scs, eq:contraction, eq:casimir-polder,
    eq:scale-rvdw-scs): screened alpha0, C6, omega, R_vdW and alpha_bar(iu) at
    u = 0 and the nfreq grid points."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    out = {k: np.empty(N) for k in ("alpha", "c6", "omega", "rvdw")}
    dyn = np.empty((nfreq + 1, N))
    lib = _load()
    lib.orc_scs.restype = ctypes.c_int
    rc = lib.orc_scs(N, _p(R), _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)), ctypes.c_double(beta),
                     ctypes.c_double(a), nfreq, _p(out["alpha"]), _p(out["c6"]), _p(out["omega"]),
                     _p(out["rvdw"]), _p(dyn))
    _check(rc, "scs")
    out["alpha_dyn"] = dyn
    return out


def mbd_rsscs(R, alpha0, omega, rvdw, beta=0.83, a=6.0, nfreq=15, gradients=True):
    """MBD@rsSCS energy (SCS stage, then MBD with the screened parameters) and
    dE/dR through the screened parameters."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    E = np.zeros(1)
    g = np.empty((N, 3)) if gradients else None
    sa, sw, sv = np.empty(N), np.empty(N), np.empty(N)
    lib = _load()
    lib.orc_mbd_rsscs.restype = ctypes.c_int
    rc = lib.orc_mbd_rsscs(N, _p(R), _p(_arr(alpha0)), _p(_arr(omega)), _p(_arr(rvdw)), ctypes.c_double(beta),
                           ctypes.c_double(a), nfreq, _p(E), _p(g), _p(sa), _p(sw), _p(sv))
    _check(rc, "mbd_rsscs")
    out = {"energy": float(E[0]), "alpha_scs": sa, "omega_scs": sw, "rvdw_scs": sv}
    if gradients:
        out["grad_R"] = g
    return out


def min_coupling_eig(R, alpha0, rvdw, beta=0.83, a=6.0):
    """Smallest eigenvalue of alpha0^{1/2} T^lr alpha0^{1/2} (collapse indicator)."""
    R = _arr(R, (-1, 3)); N = R.shape[0]
    mu = ctypes.c_double()
    rc = _load().orc_min_coupling_eig(N, _p(R), _p(_arr(alpha0)), _p(_arr(rvdw)),
                                      ctypes.c_double(beta), ctypes.c_double(a), ctypes.byref(mu))
    _check(rc, "min_coupling_eig")
    return mu.value


def is_positive_definite(A):
    """Cholesky test of a symmetric matrix (oracle's own factorisation)."""
    A = _arr(A)
    _load().orc_is_positive_definite.restype = ctypes.c_int
    return bool(_load().orc_is_positive_definite(A.shape[0], _p(A)))


def coupling_matrix(R, alpha0, rvdw, beta=0.83, a=6.0):
    """alpha0^{1/2} T^lr alpha0^{1/2} (finite): Q of eq:q-matrix with omega = 1, minus I."""
    R = _arr(R, (-1, 3))
    N = R.shape[0]
    S = assemble_finite(R, alpha0, np.ones(N), rvdw, beta, a)
    S[np.diag_indices(3 * N)] -= 1.0
    return S


def dipole(r):
    T = np.empty(9); dT = np.empty(27)
    _load().orc_dipole(_p(_arr(r)), _p(T), _p(dT))
    return T.reshape(3, 3), dT.reshape(3, 3, 3)


def dipole_erfc(r, gamma):
    T = np.empty(9); dT = np.empty(27)
    _load().orc_dipole_erfc(_p(_arr(r)), ctypes.c_double(gamma), _p(T), _p(dT))
    return T.reshape(3, 3), dT.reshape(3, 3, 3)


def monkhorst_pack(k1, k2, k3):
    """Uniform q grid offset from Gamma: f = (2r - n - 1)/(2n), r = 1..n per axis."""
    axes = [(2.0 * np.arange(1, k + 1) - k - 1) / (2.0 * k) for k in (k1, k2, k3)]
    return np.array([[x, y, z] for x in axes[0] for y in axes[1] for z in axes[2]])
