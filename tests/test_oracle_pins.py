"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed forms
(dimer), limits (large R, weak coupling -> eq:pairwise), textbook signs
(Axilrod-Teller-Muto), exact identities (frequency route eq:log-formula,
supercell/q-grid equivalence, Lorentz field of a cubic lattice), invariants
(traces, translation/rotation invariance, Euler homogeneity) and central
finite differences of the oracle's own energy.
"""
import numpy as np
import pytest

import gen
import oracle


def _dimer(R=7.5, a0=(11.0, 17.0), om=(0.6, 0.4), rv=(3.5, 3.9), beta=0.83):
    coords = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    return coords, np.array(a0), np.array(om), np.array(rv), beta


def _fermi(d, R0, a=6.0):
    return 1.0 / (1.0 + np.exp(-a * (d / R0 - 1.0)))


def _dimer_closed_form_energy(R, a0, om, rv, beta):
    """Heterodimer: Q splits into three 2x2 blocks with t = g/R^3, g/R^3, -2g/R^3."""
    g = _fermi(R, beta * (rv[0] + rv[1])) if beta > 0 else 1.0
    lam = []
    for t in (g / R ** 3, g / R ** 3, -2.0 * g / R ** 3):
        m = 0.5 * (om[0] ** 2 + om[1] ** 2)
        r = np.sqrt((0.5 * (om[0] ** 2 - om[1] ** 2)) ** 2
                    + om[0] ** 2 * om[1] ** 2 * a0[0] * a0[1] * t * t)
        lam += [m - r, m + r]
    lam = np.sort(lam)
    return 0.5 * np.sum(np.sqrt(lam)) - 1.5 * (om[0] + om[1]), lam


def _cluster(seed, n, side_bohr=14.0):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, side_bohr, 3)
        if all(np.linalg.norm(p - q) > 3.0 for q in pts):
            pts.append(p)
    a0, om, rv = gen.draw_params(rng, n)
    return np.array(pts), a0, om, rv


# --------------------------------------------------------------------------
# pair tensors
# --------------------------------------------------------------------------

def _num_hessian(f, r, h=1e-4):
    H = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            ea = np.eye(3)[a] * h
            eb = np.eye(3)[b] * h
            H[a, b] = (f(r + ea + eb) - f(r + ea - eb) - f(r - ea + eb) + f(r - ea - eb)) / (4 * h * h)
    return H


def test_dipole_is_minus_hessian_of_inverse_distance():
    r = np.array([1.3, -2.1, 2.7])
    T, _ = oracle.dipole(r)
    H = _num_hessian(lambda x: 1.0 / np.linalg.norm(x), r)
    np.testing.assert_allclose(T, -H, atol=1e-7)


def test_erfc_tensor_is_minus_hessian_and_reduces_to_bare():
    from math import erfc
    r = np.array([2.2, 0.7, -1.9])
    gamma = 0.37
    Te, _ = oracle.dipole_erfc(r, gamma)
    H = _num_hessian(lambda x: erfc(gamma * np.linalg.norm(x)) / np.linalg.norm(x), r)
    np.testing.assert_allclose(Te, -H, atol=1e-7)
    T, _ = oracle.dipole(r)
    T0, _ = oracle.dipole_erfc(r, 1e-9)
    np.testing.assert_allclose(T0, T, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("which", ["bare", "erfc"])
def test_tensor_derivatives_fd(which):
    r = np.array([1.1, 2.3, -0.8])
    f = (lambda x: oracle.dipole(x)) if which == "bare" else (lambda x: oracle.dipole_erfc(x, 0.45))
    _, dT = f(r)
    h = 1e-6
    for c in range(3):
        e = np.eye(3)[c] * h
        fd = (f(r + e)[0] - f(r - e)[0]) / (2 * h)
        np.testing.assert_allclose(dT[c], fd, atol=1e-8)


# --------------------------------------------------------------------------
# eigensolver pins
# --------------------------------------------------------------------------

def test_jacobi_known_spectrum_and_vectors():
    rng = np.random.default_rng(11)
    n = 40
    lam = np.sort(rng.uniform(-3, 5, n))
    lam[5] = lam[6]  # exact degeneracy
    X, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = X @ np.diag(lam) @ X.T
    A = 0.5 * (A + A.T)
    w, V = oracle.jacobi(A)
    np.testing.assert_allclose(w, np.sort(lam), atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(A @ V, V * w, atol=1e-12)


def test_jacobi_matches_lapack_and_trace_invariants():
    A = gen.random_symmetric(3, 73)
    w = oracle.jacobi(A, vectors=False)
    np.testing.assert_allclose(w, np.linalg.eigvalsh(A), atol=1e-12)
    np.testing.assert_allclose(w.sum(), np.trace(A), atol=1e-11)
    np.testing.assert_allclose((w ** 2).sum(), (A * A).sum(), rtol=1e-13)


def test_jacobi_2x2_closed_form():
    a, b, c = 0.7, -0.3, 1.9
    w = oracle.jacobi(np.array([[a, b], [b, c]]), vectors=False)
    m, r = 0.5 * (a + c), np.hypot(0.5 * (a - c), b)
    np.testing.assert_allclose(w, [m - r, m + r], atol=1e-15)


def test_hermitian_embedding_doubles_eigenvalues():
    rng = np.random.default_rng(5)
    n = 12
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = 0.5 * (Z + Z.conj().T)
    w = oracle.jacobi_hermitian(H)
    ref = np.linalg.eigvalsh(H)
    np.testing.assert_allclose(w[0::2], ref, atol=1e-12)
    np.testing.assert_allclose(w[1::2], ref, atol=1e-12)


# --------------------------------------------------------------------------
# finite MBD energy pins
# --------------------------------------------------------------------------

@pytest.mark.parametrize("R", [4.0, 7.5, 12.0])
def test_dimer_closed_form(R):
    coords, a0, om, rv, beta = _dimer(R=R)
    out = oracle.mbd_finite(coords, a0, om, rv, beta=beta, gradients=False)
    E_ref, lam = _dimer_closed_form_energy(R, a0, om, rv, beta)
    np.testing.assert_allclose(out["eigs"], lam, atol=1e-15)
    assert abs(out["energy"] - E_ref) < 1e-15


def test_dimer_force_closed_form():
    coords, a0, om, rv, beta = _dimer(R=6.3)
    out = oracle.mbd_finite(coords, a0, om, rv, beta=beta)
    h = 1e-3
    f = lambda R: _dimer_closed_form_energy(R, a0, om, rv, beta)[0]
    # five-point stencil of the closed form (truncation O(h^4))
    dEdR = (-f(6.3 + 2 * h) + 8 * f(6.3 + h) - 8 * f(6.3 - h) + f(6.3 - 2 * h)) / (12 * h)
    np.testing.assert_allclose(out["grad_R"][1, 2], dEdR, atol=1e-13)
    np.testing.assert_allclose(out["grad_R"][0, 2], -dEdR, atol=1e-13)
    assert abs(out["grad_R"][:, :2]).max() < 1e-18


@pytest.mark.parametrize("R", [15.0, 25.0, 40.0])
def test_large_R_limit_c6(R):
    coords, a0, om, rv, beta = _dimer(R=R)
    E = oracle.mbd_finite(coords, a0, om, rv, beta=beta, gradients=False)["energy"]
    c6 = 1.5 * a0[0] * a0[1] * om[0] * om[1] / (om[0] + om[1])
    g = _fermi(R, beta * (rv[0] + rv[1]))
    ratio = E * R ** 6 / (-c6 * g * g)
    # next order in the R^-1 expansion is O(alpha^2 / R^6); ~1e-3 at R = 15
    assert abs(ratio - 1.0) < 3.0 * a0[0] * a0[1] / R ** 6 * 10


def test_weak_coupling_limit_is_pairwise():
    coords, a0, om, rv = _cluster(2, 7)
    beta = 0.83

    def e2(alpha):
        tot = 0.0
        for i in range(len(om)):
            for j in range(len(om)):
                if i == j:
                    continue
                d = np.linalg.norm(coords[j] - coords[i])
                c6 = 1.5 * alpha[i] * alpha[j] / (1 / om[i] + 1 / om[j])
                g = _fermi(d, beta * (rv[i] + rv[j]))
                tot += -0.5 * c6 * g * g / d ** 6
        return tot

    s1, s2 = 1e-3, 5e-4
    E1 = oracle.mbd_finite(coords, a0 * s1, om, rv, beta=beta, gradients=False)["energy"] / s1 ** 2
    E2 = oracle.mbd_finite(coords, a0 * s2, om, rv, beta=beta, gradients=False)["energy"] / s2 ** 2
    rich = (s1 * E2 - s2 * E1) / (s1 - s2)  # remove the O(s) term
    np.testing.assert_allclose(rich, e2(a0), rtol=1e-4)


def test_atm_three_body_sign():
    a0 = np.full(3, 10.0); om = np.full(3, 0.5); rv = np.full(3, 3.0)
    side = 15.0

    def energy(c):
        return oracle.mbd_finite(c, a0[:len(c)], om[:len(c)], rv[:len(c)], beta=0.0,
                                 gradients=False)["energy"]

    tri = np.array([[0, 0, 0], [side, 0, 0], [side / 2, side * np.sqrt(3) / 2, 0]])
    lin = np.array([[0, 0, 0], [side, 0, 0], [2 * side, 0, 0]])
    for geo, sign in ((tri, 1.0), (lin, -1.0)):
        e3 = energy(geo) - sum(energy(geo[[i, j]]) for i, j in ((0, 1), (0, 2), (1, 2)))
        assert sign * e3 > 0


def test_single_atom_and_far_apart():
    c = np.zeros((1, 3))
    out = oracle.mbd_finite(c, [10.0], [0.5], [3.0])
    assert out["energy"] == 0.0
    far = np.array([[0, 0, 0], [0, 0, 1e5]])
    assert abs(oracle.mbd_finite(far, [10.0, 20.0], [0.5, 0.7], [3.0, 3.3],
                                 gradients=False)["energy"]) < 1e-20


def test_trace_identities_on_q():
    coords, a0, om, rv = _cluster(4, 10)
    Q = oracle.assemble_finite(coords, a0, om, rv)
    np.testing.assert_allclose(Q, Q.T, atol=0)
    w = oracle.jacobi(Q, vectors=False)
    np.testing.assert_allclose(w.sum(), np.trace(Q), rtol=1e-14)
    np.testing.assert_allclose((w ** 2).sum(), (Q * Q).sum(), rtol=1e-13)


def test_frequency_route_equals_eigen_route():
    coords, a0, om, rv = _cluster(6, 12)
    Ee = oracle.mbd_finite(coords, a0, om, rv, gradients=True)
    Ef = oracle.mbd_finite_freq(coords, a0, om, rv, npts=40, sample_atoms=[0, 5])
    assert abs(Ef["energy"] - Ee["energy"]) < 1e-11 * abs(Ee["energy"]) + 1e-15
    np.testing.assert_allclose(Ef["grad_R_sample"], Ee["grad_R"][[0, 5]], atol=1e-10)
    np.testing.assert_allclose(Ef["grad_alpha0_sample"], Ee["grad_alpha0"][[0, 5]], atol=1e-11)
    np.testing.assert_allclose(Ef["grad_omega_sample"], Ee["grad_omega"][[0, 5]], atol=1e-10)
    # and against central differences of the frequency-route energy itself
    h = 1e-4 * a0[5]
    ap, am = a0.copy(), a0.copy()
    ap[5] += h
    am[5] -= h
    fd = (oracle.mbd_finite_freq(coords, ap, om, rv, npts=40)["energy"]
          - oracle.mbd_finite_freq(coords, am, om, rv, npts=40)["energy"]) / (2 * h)
    np.testing.assert_allclose(Ef["grad_alpha0_sample"][1], fd, rtol=1e-6)


def test_gauss_legendre_integrates_polynomials():
    x, w = oracle.gauss_legendre(9)
    for p in range(18):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        np.testing.assert_allclose(np.sum(w * x ** p), exact, atol=1e-14)


# --------------------------------------------------------------------------
# finite gradients
# --------------------------------------------------------------------------

def _fd(fun, x, idx, h):
    xp = x.copy(); xp[idx] += h
    xm = x.copy(); xm[idx] -= h
    return (fun(xp) - fun(xm)) / (2 * h)


def test_finite_gradients_fd_and_invariants():
    coords, a0, om, rv = _cluster(9, 8)
    beta = 0.83
    out = oracle.mbd_finite(coords, a0, om, rv, beta=beta)

    def E(c=coords, a=a0, w=om, r=rv):
        return oracle.mbd_finite(c, a, w, r, beta=beta, gradients=False)["energy"]

    for idx in [(0, 0), (3, 1), (7, 2)]:
        fd = _fd(lambda c: E(c=c), coords, idx, 1e-4)
        np.testing.assert_allclose(out["grad_R"][idx], fd, atol=1e-10)
    for i in (1, 6):
        np.testing.assert_allclose(out["grad_alpha0"][i], _fd(lambda a: E(a=a), a0, i, 1e-4 * a0[i]),
                                   rtol=1e-6, atol=1e-12)
        np.testing.assert_allclose(out["grad_omega"][i], _fd(lambda w: E(w=w), om, i, 1e-5),
                                   rtol=1e-6, atol=1e-12)
        np.testing.assert_allclose(out["grad_rvdw"][i], _fd(lambda r: E(r=r), rv, i, 1e-5),
                                   rtol=1e-5, atol=1e-12)
    g = out["grad_R"]
    assert abs(g.sum(axis=0)).max() < 1e-16
    torque = np.cross(coords, g).sum(axis=0)
    assert abs(torque).max() < 1e-14
    # E is homogeneous of degree one in omega
    np.testing.assert_allclose(np.dot(om, out["grad_omega"]), out["energy"], rtol=1e-11)


def test_c6_input_chain_rule():
    coords, a0, om, rv = _cluster(10, 6)
    c6 = 0.75 * om * a0 ** 2
    out = oracle.mbd_finite_c6(coords, a0, c6, rv)
    ref = oracle.mbd_finite(coords, a0, om, rv, gradients=False)["energy"]
    assert abs(out["energy"] - ref) < 1e-15

    def Ec6(a, c):
        return oracle.mbd_finite_c6(coords, a, c, rv)["energy"]

    i = 2
    fd_a = _fd(lambda a: Ec6(a, c6), a0, i, 1e-4 * a0[i])
    fd_c = _fd(lambda c: Ec6(a0, c), c6, i, 1e-4 * c6[i])
    np.testing.assert_allclose(out["grad_alpha0_c6"][i], fd_a, rtol=1e-6)
    np.testing.assert_allclose(out["grad_c6"][i], fd_c, rtol=1e-6)


# --------------------------------------------------------------------------
# periodic pins
# --------------------------------------------------------------------------

def _cell(seed=7, N=3):
    rng = np.random.default_rng(seed)
    lat = np.array([[9.0, 0.3, 0.1], [0.5, 10.0, -0.2], [0.7, 0.4, 11.0]])
    R = rng.uniform(0, 1, (N, 3)) @ lat
    a0 = rng.uniform(5, 20, N); om = rng.uniform(0.4, 0.8, N); rv = rng.uniform(3, 4, N)
    return R, lat, a0, om, rv


def test_lorentz_field_simple_cubic():
    L = 9.0
    lat = np.eye(3) * L
    Q = oracle.assemble_periodic(np.zeros((1, 3)), lat, np.zeros(3), [1.0], [1.0], [3.0], beta=0.0)
    T = Q - np.eye(3)
    np.testing.assert_allclose(T.real, -4 * np.pi / (3 * L ** 3) * np.eye(3), atol=1e-12)
    assert abs(T.imag).max() < 1e-14


def test_periodic_hermitian_and_time_reversal():
    R, lat, a0, om, rv = _cell()
    B = 2 * np.pi * np.linalg.inv(lat).T
    q = np.array([0.25, -0.25, 0.125]) @ B
    Q = oracle.assemble_periodic(R, lat, q, a0, om, rv)
    np.testing.assert_allclose(Q, Q.conj().T, atol=1e-14)
    w1 = oracle.jacobi_hermitian(Q)
    w2 = oracle.jacobi_hermitian(oracle.assemble_periodic(R, lat, -q, a0, om, rv))
    np.testing.assert_allclose(w1, w2, atol=1e-13)


def test_periodic_gamma_independence_and_cutoffs():
    R, lat, a0, om, rv = _cell()
    qf = oracle.monkhorst_pack(2, 2, 2)
    g, rc, kc = oracle.ewald_defaults(lat)
    E0 = oracle.mbd_periodic(R, lat, qf, a0, om, rv, gradients=False)["energy"]
    for s in (0.7, 1.4):
        Es = oracle.mbd_periodic(R, lat, qf, a0, om, rv, gamma=g * s, rc=6 / (g * s),
                                 kc=10 * g * s, gradients=False)["energy"]
        assert abs(Es - E0) < 1e-10
    Et = oracle.mbd_periodic(R, lat, qf, a0, om, rv, gamma=g, rc=7 / g, kc=12 * g,
                             gradients=False)["energy"]
    assert abs(Et - E0) < 1e-10


def test_supercell_equivalence():
    R, lat, a0, om, rv = _cell(seed=8, N=2)
    g, rc, kc = oracle.ewald_defaults(lat)
    qf = oracle.monkhorst_pack(2, 2, 2)
    cell = oracle.mbd_periodic(R, lat, qf, a0, om, rv, gamma=g, rc=rc, kc=kc)
    shifts = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], float)
    Rs = np.concatenate([R + s @ lat for s in shifts])
    rep = lambda v: np.concatenate([v] * 8)
    sup = oracle.mbd_periodic(Rs, 2 * lat, [[0.5, 0.5, 0.5]], rep(a0), rep(om), rep(rv),
                              gamma=g, rc=rc, kc=kc)
    assert abs(sup["energy"] / 8 - cell["energy"]) < 1e-13
    gsum = sup["grad_R"].reshape(8, 2, 3).sum(axis=0)
    np.testing.assert_allclose(gsum, 8 * cell["grad_R"], atol=1e-13)


def test_periodic_gradients_fd():
    R, lat, a0, om, rv = _cell()
    qf = oracle.monkhorst_pack(2, 2, 2)
    g, rc, kc = oracle.ewald_defaults(lat)
    kw = dict(gamma=g, rc=rc, kc=kc)
    out = oracle.mbd_periodic(R, lat, qf, a0, om, rv, **kw)

    def E(Rx=R, L=lat, a=a0):
        return oracle.mbd_periodic(Rx, L, qf, a, om, rv, gradients=False, **kw)["energy"]

    for idx in [(0, 0), (1, 2), (2, 1)]:
        np.testing.assert_allclose(out["grad_R"][idx], _fd(lambda x: E(Rx=x), R, idx, 1e-4),
                                   atol=2e-10)
    for idx in [(0, 0), (1, 0), (2, 2), (0, 2)]:
        np.testing.assert_allclose(out["grad_lattice"][idx], _fd(lambda x: E(L=x), lat, idx, 1e-4),
                                   atol=2e-10)
    np.testing.assert_allclose(out["grad_alpha0"][1], _fd(lambda x: E(a=x), a0, 1, 1e-4),
                               rtol=1e-6)
    assert abs(out["grad_R"].sum(axis=0)).max() < 1e-15


def test_periodic_omega_rvdw_gradients_fd():
    R, lat, a0, om, rv = _cell()
    qf = oracle.monkhorst_pack(2, 2, 1)
    g, rc, kc = oracle.ewald_defaults(lat)
    kw = dict(gamma=g, rc=rc, kc=kc)
    out = oracle.mbd_periodic(R, lat, qf, a0, om, rv, **kw)

    def E(w=om, v=rv):
        return oracle.mbd_periodic(R, lat, qf, a0, w, v, gradients=False, **kw)["energy"]

    for i in range(3):
        np.testing.assert_allclose(out["grad_omega"][i], _fd(lambda x: E(w=x), om, i, 1e-5),
                                   rtol=1e-7, atol=1e-10)
        np.testing.assert_allclose(out["grad_rvdw"][i], _fd(lambda x: E(v=x), rv, i, 1e-5),
                                   rtol=1e-6, atol=1e-11)
    # the damping radius matters here: a non-trivial R_vdW derivative
    assert abs(out["grad_rvdw"]).max() > 1e-5
    # Euler: Q(s omega) = s^2 Q(omega), so E is homogeneous of degree one in omega
    assert abs(np.dot(om, out["grad_omega"]) - out["energy"]) < 1e-13


def test_periodic_c6_chain_rule():
    R, lat, a0, om, rv = _cell(seed=9, N=2)
    qf = oracle.monkhorst_pack(2, 1, 1)
    c6 = 0.75 * om * a0 ** 2
    out = oracle.mbd_periodic_c6(R, lat, qf, a0, c6, rv)

    def Ec6(a, c):
        return oracle.mbd_periodic(R, lat, qf, a, 4.0 * c / (3.0 * a ** 2), rv, gradients=False)["energy"]

    fd_a = _fd(lambda a: Ec6(a, c6), a0, 1, 1e-4 * a0[1])
    fd_c = _fd(lambda c: Ec6(a0, c), c6, 1, 1e-4 * c6[1])
    np.testing.assert_allclose(out["grad_alpha0_c6"][1], fd_a, rtol=1e-6)
    np.testing.assert_allclose(out["grad_c6"][1], fd_c, rtol=1e-6)


def test_periodic_single_atom_lorentz_energy():
    """One atom per simple cubic cell at q = 0: the lattice sum of T is the
    Lorentz field -4 pi/(3 L^3) I (tin-foil, no k = 0 term), so Q(0) =
    omega^2 (1 - 4 pi alpha0/(3 L^3)) I and the energy per cell has the closed
    form (3/2) omega (sqrt(1 - 4 pi alpha0/(3 L^3)) - 1).  This fixes the
    normalisation of the periodic energy: one half of sum sqrt(lambda) per
    q-matrix (each Hermitian eigenvalue counted once), minus (3/2) sum omega,
    averaged over q (eq:brillouin-int); it tends to 0 like L^-3."""
    a0, om, rv = 11.0, 0.6, 3.5
    prev = None
    for L in (40.0, 80.0, 160.0):
        E = oracle.mbd_periodic(np.zeros((1, 3)), np.eye(3) * L, [[0.0, 0.0, 0.0]], [a0], [om], [rv],
                                gradients=False)["energy"]
        cf = 1.5 * om * (np.sqrt(1.0 - 4.0 * np.pi * a0 / (3.0 * L ** 3)) - 1.0)
        assert abs(E - cf) < 1e-12, (L, E, cf)
        if prev is not None:
            assert abs(prev / E - 8.0) < 0.01
        prev = E


def test_periodic_large_box_limit_dimer():
    """A heterodimer in a growing simple cubic cell at q = 0 approaches the
    finite dimer (closed form) with a leading L^-3 error (the images' dipole
    field) and an L^-5 correction: the ratio of successive errors at L, 2L is
    close to 8, and two Richardson steps (L^-3, then L^-5) reach the finite
    energy to about 1e-9 Ha."""
    Rd = 7.5
    coords, a0, om, rv, beta = _dimer(R=Rd)
    Efin, _ = _dimer_closed_form_energy(Rd, a0, om, rv, beta)
    d = {}
    for L in (40.0, 80.0, 160.0):
        E = oracle.mbd_periodic(coords + L / 2, np.eye(3) * L, [[0.0, 0.0, 0.0]], a0, om, rv, beta,
                                gradients=False)["energy"]
        d[L] = E - Efin
    assert abs(d[40.0] / d[80.0] - 8.0) < 0.2
    assert abs(d[80.0] / d[160.0] - 8.0) < 0.05
    r1 = (8.0 * d[80.0] - d[40.0]) / 7.0
    r2 = (8.0 * d[160.0] - d[80.0]) / 7.0
    assert abs(r2) < 2e-8
    assert abs((32.0 * r2 - r1) / 31.0) < 2e-9


# --------------------------------------------------------------------------
# pairwise (TS) dispersion, eq:pairwise and eq:ts-ewald
# --------------------------------------------------------------------------

def test_ts_equals_second_order_mbd_undamped():
    """eq:rpa: the second order of the many-body expansion is the pairwise
    energy.  Undamped (f = g = 1), E_MBD(s alpha0)/s^2 = E^(2) + s E^(3) +
    s^2 E^(4) + ..., so the pairwise energy is its limit s -> 0 (two
    Richardson steps over s, 2s, 4s)."""
    coords, a0, om, rv = _cluster(12, 7)
    Ets = oracle.ts(coords, a0, om, rv, sR=0.0)["energy"]
    e = {s: oracle.mbd_finite(coords, s * a0, om, rv, beta=0.0, gradients=False)["energy"] / s ** 2
         for s in (1e-3, 2e-3, 4e-3)}
    r1, r2 = 2 * e[1e-3] - e[2e-3], 2 * e[2e-3] - e[4e-3]
    lim = (4 * r1 - r2) / 3
    assert abs(lim - Ets) < 1e-7 * abs(Ets)


def _ts_direct(R, lat, a0, om, rv, sR, a, Rmax):
    """Plain lattice sum of f/R^6 over images within Rmax plus the continuum
    tail 4 pi/(3 Omega Rmax^3) per ordered pair (f = 1 there)."""
    R = np.asarray(R); N = len(R)
    vol = abs(np.linalg.det(lat))
    B = 2 * np.pi * np.linalg.inv(lat).T
    nmax = [int(np.ceil(Rmax * np.linalg.norm(B[v]) / (2 * np.pi))) + 2 for v in range(3)]
    n = np.array([[x, y, z] for x in range(-nmax[0], nmax[0] + 1) for y in range(-nmax[1], nmax[1] + 1)
                  for z in range(-nmax[2], nmax[2] + 1)], float) @ lat
    E = 0.0
    for i in range(N):
        for j in range(N):
            x = R[j] - R[i] + n
            d = np.linalg.norm(x, axis=1)
            d = d[(d > 0) & (d <= Rmax)]
            f = 1.0 / (1.0 + np.exp(-a * (d / (sR * (rv[i] + rv[j])) - 1.0))) if sR > 0 else 1.0
            c6 = 1.5 * a0[i] * a0[j] / (1 / om[i] + 1 / om[j])
            E += -0.5 * c6 * (np.sum(f / d ** 6) + 4 * np.pi / (3 * vol * Rmax ** 3))
    return E


@pytest.mark.parametrize("sR", [0.0, 0.94])
def test_ts_ewald_equals_direct_lattice_sum(sR):
    """The R^-6 lattice sum converges absolutely, so the Ewald split must agree
    with the plain sum over images (this pins the readings of eq:ts-ewald:
    G = 0 term included, self term -gamma^6/6); and it must not depend on
    gamma."""
    R, lat, a0, om, rv = _cell(seed=21, N=3)
    Ed = _ts_direct(R, lat, a0, om, rv, sR, 20.0, Rmax=120.0)
    g, rc, kc = oracle.ewald_defaults(lat)
    Es = [oracle.ts(R, a0, om, rv, sR=sR, lattice=lat, gamma=g * s, rc=6 / (g * s), kc=10 * g * s)["energy"]
          for s in (0.7, 1.0, 1.4)]
    # the sharp sphere of the plain sum leaves ~1e-7 relative (lattice points
    # near its surface); the G = 0 term or the self term alone are ~1e-2 and ~1
    assert abs(Es[1] - Ed) < 1e-6 * abs(Ed)
    assert max(Es) - min(Es) < 1e-10 * abs(Ed)  # the cutoffs converge to ~1e-10 relative (Sec. 3.3)


def test_ts_gradients_fd():
    coords, a0, om, rv = _cluster(13, 6)
    R, lat, pa0, pom, prv = _cell(seed=22, N=3)
    for (X, A0, OM, RV, kw) in ((coords, a0, om, rv, {}), (R, pa0, pom, prv, {"lattice": lat})):
        out = oracle.ts(X, A0, OM, RV, sR=0.94, **kw)

        def E(x=X, a=A0, w=OM, v=RV):
            return oracle.ts(x, a, w, v, sR=0.94, **kw)["energy"]

        for idx in [(0, 0), (1, 2), (2, 1)]:
            np.testing.assert_allclose(out["grad_R"][idx], _fd(lambda x: E(x=x), X, idx, 1e-4), atol=1e-11)
        for i in range(2):
            np.testing.assert_allclose(out["grad_alpha0"][i], _fd(lambda x: E(a=x), A0, i, 1e-5), rtol=1e-7)
            np.testing.assert_allclose(out["grad_omega"][i], _fd(lambda x: E(w=x), OM, i, 1e-6), rtol=1e-7)
            np.testing.assert_allclose(out["grad_rvdw"][i], _fd(lambda x: E(v=x), RV, i, 1e-5),
                                       rtol=1e-6, atol=1e-12)
        assert abs(out["grad_R"].sum(axis=0)).max() < 1e-14


# --------------------------------------------------------------------------
# frequency route: eq:log-formula, eq:rpa, eq:gould-norm
# --------------------------------------------------------------------------

def test_freq_terms_log_formula_equals_eigen_route():
    """eq:log-formula equals eq:mbd-energy (the integral of
    ln((lambda + u^2)/(omega^2 + u^2)) over u is pi (sqrt(lambda) - omega)),
    for a finite cluster and for a periodic cell on a q mesh."""
    coords, a0, om, rv = _cluster(12, 7)
    t = oracle.freq_terms(coords, a0, om, rv, nfreq=40, norder=2)
    e = oracle.mbd_finite(coords, a0, om, rv, gradients=False)["energy"]
    assert abs(t["energy"] - e) < 1e-11 * abs(e)
    R, lat, pa0, pom, prv = _cell()
    qf = oracle.monkhorst_pack(2, 2, 1)
    t = oracle.freq_terms(R, pa0, pom, prv, nfreq=40, norder=2, lattice=lat, q_frac=qf)
    e = oracle.mbd_periodic(R, lat, qf, pa0, pom, prv, gradients=False)["energy"]
    assert abs(t["energy"] - e) < 1e-10 * abs(e)


def test_freq_terms_second_order_is_pairwise_with_g_squared():
    """eq:pairwise: the second-order term is the pairwise energy with
    f = R^6 Tr(T_lr^2)/6 = g^2 and C6_ij = (3/2) alpha_i alpha_j/(1/omega_i +
    1/omega_j); the first-order term vanishes for a finite system (T_ii = 0)."""
    coords, a0, om, rv = _cluster(14, 6)
    t = oracle.freq_terms(coords, a0, om, rv, nfreq=40, norder=2)
    E2 = 0.0
    for i in range(6):
        for j in range(6):
            if i == j:
                continue
            d = np.linalg.norm(coords[j] - coords[i])
            g = _fermi(d, 0.83 * (rv[i] + rv[j]))
            E2 += -0.5 * 1.5 * a0[i] * a0[j] / (1 / om[i] + 1 / om[j]) * g * g / d ** 6
    assert abs(t["orders"][1] - E2) < 1e-11 * abs(E2)
    assert abs(t["orders"][0]) < 1e-15


def test_freq_terms_series_sums_to_log():
    """Weak coupling (every |x_k| < 1): the many-body expansion eq:rpa,
    summed over orders, converges to eq:log-formula; the renormalisation of
    eq:gould-norm changes only the negative x_k, by O(|x|^9), and its -x~ term
    removes the first order: E_Gould = E - E^(1) to that order."""
    coords, a0, om, rv = _cluster(15, 6)
    t = oracle.freq_terms(coords, 0.2 * a0, om, rv, nfreq=30, norder=40)
    assert abs(t["orders"].sum() - t["energy"]) < 1e-13 * abs(t["energy"])
    # x~ - x = (pi/48) |x|^9 + ... for x < 0: with |x| <= 0.1 the two energies agree closely
    t = oracle.freq_terms(coords, 0.05 * a0, om, rv, nfreq=30, norder=2)
    assert abs(t["energy_gould"] - (t["energy"] - t["orders"][0])) < 1e-8 * abs(t["energy"])


def test_freq_terms_first_order_lorentz():
    """One atom per simple cubic cell at q = 0: T_ii(0) = -4 pi/(3 Omega) I
    (Lorentz field), so E^(1) = (1/2pi) int alpha(iu) du Tr T_ii = -pi
    alpha0 omega/Omega (using int_0^inf alpha(iu) du = pi alpha0 omega/2)."""
    L, a0, om = 40.0, 11.0, 0.6
    t = oracle.freq_terms(np.zeros((1, 3)), [a0], [om], [3.5], nfreq=40, norder=1, lattice=np.eye(3) * L,
                          q_frac=[[0.0, 0.0, 0.0]])
    assert abs(t["orders"][0] - (-np.pi * a0 * om / L ** 3)) < 1e-13


def test_freq_terms_collapse_gould_finite():
    """Inside the dipole collapse (some 1 + x_k <= 0) eq:log-formula has no
    real value, while the renormalised energy of eq:gould-norm stays finite."""
    coords = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]])
    # x = -2 alpha(iu)/R^3 for the mode along the axis: -1.48 at u = 0
    t = oracle.freq_terms(coords, [20.0, 20.0], [0.5, 0.5], [1.0, 1.0], beta=0.0, nfreq=15, norder=2)
    assert t["min_one_plus_x"] <= 0.0
    assert np.isnan(t["energy"])
    assert np.isfinite(t["energy_gould"]) and t["energy_gould"] < 0.0
    # a dimer just outside the collapse: renormalised and plain energies close
    t2 = oracle.freq_terms(coords, [12.0, 12.0], [0.5, 0.5], [1.0, 1.0], beta=0.0, nfreq=40, norder=2)
    assert t2["min_one_plus_x"] > 0.0
    assert abs(t2["energy_gould"] - t2["energy"]) < 0.05 * abs(t2["energy"])


# --------------------------------------------------------------------------
# self-consistent screening: eq:tgg, eq:mayer, eq:scs, eq:contraction,
# eq:casimir-polder, eq:scale-rvdw-scs
# --------------------------------------------------------------------------

def _hess(f, r, h=1e-4):
    return _num_hessian(f, np.asarray(r, float), h)


def test_tgg_is_minus_hessian_of_erf_over_r():
    """T^GG = -Hess(erf(r/s)/r) in the sign convention of the explicit dipole
    tensor (reading of eq:dipole), its r-derivative matches finite
    differences, and T^GG -> T when the widths vanish."""
    from scipy.special import erf
    r = np.array([1.3, -0.7, 2.1])
    s = 1.6
    T, dT = oracle.dipole_gg(r, s)
    H = _hess(lambda x: erf(np.linalg.norm(x) / s) / np.linalg.norm(x), r)
    np.testing.assert_allclose(T, -H, atol=2e-7)
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1e-5
        fd = (oracle.dipole_gg(r + e, s)[0] - oracle.dipole_gg(r - e, s)[0]) / 2e-5
        np.testing.assert_allclose(dT[c], fd, atol=1e-8)
    T0, _ = oracle.dipole(r)
    np.testing.assert_allclose(oracle.dipole_gg(r, 1e-3)[0], T0, atol=1e-13)


def test_scs_isolated_atom_and_far_apart():
    """One atom: alpha_bar = alpha, so the screened alpha0 is alpha0 and the
    Casimir-Polder C6 is (3/pi) int alpha(iu)^2 du = (3/4) alpha0^2 omega,
    giving back omega.  Atoms far beyond the damping radius: T^scs = (1-g) T^GG
    vanishes and nothing is screened."""
    o = oracle.scs(np.zeros((1, 3)), [12.0], [0.45], [3.5], nfreq=40)
    assert abs(o["alpha"][0] - 12.0) < 1e-13
    assert abs(o["c6"][0] - 0.75 * 12.0 ** 2 * 0.45) < 1e-11
    assert abs(o["omega"][0] - 0.45) < 1e-12 and abs(o["rvdw"][0] - 3.5) < 1e-14
    R = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 60.0], [0.0, 60.0, 0.0]])
    o = oracle.scs(R, [12.0, 20.0, 8.0], [0.45, 0.6, 0.5], [3.5, 3.9, 3.0], nfreq=40)
    np.testing.assert_allclose(o["alpha"], [12.0, 20.0, 8.0], rtol=1e-14)
    np.testing.assert_allclose(o["omega"], [0.45, 0.6, 0.5], rtol=1e-12)


def test_scs_dimer_closed_form():
    """A dimer along z: alpha^-1 + T^scs splits into three 2x2 blocks (x, y, z)
    with off-diagonal p_a = (1-g) T^GG_aa; inverting each block and contracting
    gives alpha_bar_1 = (1/3) sum_a (1/alpha_2 - p_a) / (1/(alpha_1 alpha_2) -
    p_a^2) at u = 0."""
    R0 = 4.0
    a1, a2, rv = 12.0, 20.0, (3.5, 3.9)
    o = oracle.scs(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R0]]), [a1, a2], [0.45, 0.6], list(rv), nfreq=15)
    sig = lambda a: (np.sqrt(2 / np.pi) * a / 3) ** (1 / 3)
    T, _ = oracle.dipole_gg(np.array([0.0, 0.0, R0]), np.hypot(sig(a1), sig(a2)))
    omg = 1.0 - _fermi(R0, 0.83 * (rv[0] + rv[1]))
    p = omg * np.diag(T)
    ab1 = np.mean([(1 / a2 - pa) / (1 / (a1 * a2) - pa * pa) for pa in p])
    ab2 = np.mean([(1 / a1 - pa) / (1 / (a1 * a2) - pa * pa) for pa in p])
    assert abs(o["alpha"][0] - ab1) < 1e-12 * ab1
    assert abs(o["alpha"][1] - ab2) < 1e-12 * ab2
    assert abs(o["rvdw"][0] - rv[0] * (ab1 / a1) ** (1 / 3)) < 1e-13


def test_mbd_rsscs_gradient_fd():
    """dE/dR of MBD@rsSCS (through the screened alpha0, omega and R_vdW, i.e.
    the derivative of eq:scs contracted as in eq:contraction) against central
    differences of the energy, Richardson-extrapolated; translation
    invariance."""
    coords, a0, om, rv = _cluster(12, 5)
    out = oracle.mbd_rsscs(coords, a0, om, rv)

    def E(x):
        return oracle.mbd_rsscs(x, a0, om, rv, gradients=False)["energy"]

    for idx in [(0, 0), (1, 2), (3, 1), (4, 0)]:
        # steps large enough that the energy's rounding (~1e-15 Ha) stays out
        f1, f2 = _fd(E, coords, idx, 1e-3), _fd(E, coords, idx, 2e-3)
        np.testing.assert_allclose(out["grad_R"][idx], (4 * f1 - f2) / 3, rtol=1e-7, atol=1e-12)
    assert abs(out["grad_R"].sum(axis=0)).max() < 1e-14


def test_mbd_rsscs_is_mbd_of_screened_parameters():
    coords, a0, om, rv = _cluster(16, 6)
    out = oracle.mbd_rsscs(coords, a0, om, rv, gradients=False)
    ref = oracle.mbd_finite(coords, out["alpha_scs"], out["omega_scs"], out["rvdw_scs"], gradients=False)
    assert abs(out["energy"] - ref["energy"]) < 1e-15
