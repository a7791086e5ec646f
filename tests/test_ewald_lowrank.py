"""CPU check of the identities behind the periodic reciprocal-space path.

The reciprocal term of T_ij(q) (Sec. 2.2, eq:ewald) is a sum of rank-one
blocks w(k) k k^T times the pair phase e^{iG.(R_j - R_i)}, k = G + q, so over
all pairs it equals U U^H with U_{ia,g} = sqrt(w_g) k_a e^{-iG_g.R_i}.  The
GPU path forms the matrix that way and contracts the adjoint through
W = M C U (M Hermitian, C = diag(c_i)): per atom k and column g, with
z = c_k sum_a conj(U_{ka,g}) W_{ka,g},
  sum over pairs of c_i c_j (P_ik + P_ki)     = 2 Re z        (dE/dalpha, dE/domega)
  dE/dR_k                                     = -2 G Im z
  dE/dA_vc = -Ainv_cv s - sum_d Ainv_dv [k_c k_d f s + 2 sqrt(w) k_c b_d
             + G_c sum_k R_kd (-2 Im z_k)],  s = sum_k Re z_k,
             b_d = sum_k c_k Re(conj(W_{kd,g}) e^{-iG.R_k}),
             f = -1/(2 gamma^2) - 2/k^2.
Here both sides are evaluated in numpy on a small random cell and a random
Hermitian M: the per-pair sums of the derivatives (of w(k), of k and the
phase through the lattice, of the prefactor through the volume) against the
low-rank forms.  The oracle is not involved; this pins the algebra the
kernels implement."""
import numpy as np


def _setup():
    rng = np.random.default_rng(1)
    N = 4
    A = np.array([[7.0, 0.3, 0.1], [0.2, 6.5, -0.4], [0.1, 0.5, 8.0]])   # rows: lattice vectors
    R = rng.uniform(0, 6, (N, 3))
    c = rng.uniform(0.5, 1.5, N)
    gamma, kc = 0.4, 2.2
    Ainv = np.linalg.inv(A)
    B = 2 * np.pi * Ainv.T
    q = np.array([0.125, -0.375, 0.25]) @ B
    Gs = []
    for m in np.ndindex(9, 9, 9):
        G = (np.array(m) - 4) @ B
        k2 = (G + q) @ (G + q)
        if 0 < k2 < kc * kc:
            Gs.append(G)
    X = rng.normal(size=(3 * N, 3 * N)) + 1j * rng.normal(size=(3 * N, 3 * N))
    return N, A, R, c, gamma, Ainv, q, np.array(Gs), X + X.conj().T


def _pairwise(N, A, R, c, gamma, Ainv, q, Gs, M):
    """Per-pair reciprocal sums of T and of its derivatives, contracted with M."""
    vol = np.linalg.det(A)
    pref, g4 = 4 * np.pi / vol, 1 / (4 * gamma ** 2)
    P = np.zeros((N, N)); dR = np.zeros((N, N, 3)); dA = np.zeros((N, N, 9))
    for i in range(N):
        for j in range(N):
            r = R[j] - R[i]
            rho = Ainv.T @ r
            Mab = M[3 * j:3 * j + 3, 3 * i:3 * i + 3].T    # Mab[a][b] = M_{jb,ia}
            for G in Gs:
                k = G + q; k2 = k @ k; E = np.exp(-k2 * g4)
                ph = np.exp(1j * G @ r)
                h = np.outer(k, k) * E / k2
                # d h_ab / d k_d, differentiated term by term
                dh = np.zeros((3, 3, 3))
                for d in range(3):
                    dh[d] = -2 * np.outer(k, k) * k[d] / k2 ** 2 * E - h * k[d] * 2 * g4
                    dh[d][d, :] += k / k2 * E
                    dh[d][:, d] += k / k2 * E
                Sh = np.sum(Mab * h)
                Sdh = np.array([np.sum(Mab * dh[d]) for d in range(3)])
                P[i, j] += (pref * Sh * ph).real
                for cc in range(3):
                    dR[i, j, cc] += (pref * 1j * G[cc] * Sh * ph).real
                    for v in range(3):
                        u = -Ainv[cc, v] * Sh - k[cc] * (Sdh @ Ainv[:, v])
                        dA[i, j, v * 3 + cc] += (pref * (u - 1j * G[cc] * rho[v] * Sh) * ph).real
    ga = np.array([sum(c[o] * c[k] * (P[o, k] + P[k, o]) for o in range(N)) for k in range(N)])
    g = np.array([sum(c[o] * c[k] * (dR[o, k] - dR[k, o]) for o in range(N) if o != k) for k in range(N)])
    la = sum(c[i] * c[j] * dA[i, j] for i in range(N) for j in range(N))
    return ga, g, la


def _lowrank(N, A, R, c, gamma, Ainv, q, Gs, M):
    vol = np.linalg.det(A)
    pref, g4 = 4 * np.pi / vol, 1 / (4 * gamma ** 2)
    ga = np.zeros(N); g = np.zeros((N, 3)); s = 0.0; L = np.zeros((3, 3))
    C3 = np.repeat(c, 3)
    for G in Gs:
        k = G + q; k2 = k @ k
        sw = np.sqrt(pref * np.exp(-k2 * g4) / k2)
        f = -2 * g4 - 2 / k2
        phi = np.exp(-1j * (R @ G))
        u = (sw * phi[:, None] * k[None, :]).reshape(-1)
        W = M @ (C3 * u)
        for a in range(N):
            z = c[a] * np.sum(np.conj(u[3 * a:3 * a + 3]) * W[3 * a:3 * a + 3])
            e = -2 * z.imag
            ga[a] += 2 * z.real
            g[a] += G * e
            s += z.real
            b = c[a] * (np.conj(W[3 * a:3 * a + 3]) * phi[a]).real
            L += f * z.real * np.outer(k, k) + 2 * sw * np.outer(k, b) + e * np.outer(G, R[a])
    la = np.array([-Ainv[cc, v] * s - Ainv[:, v] @ L[cc, :] for v in range(3) for cc in range(3)])
    return ga, g, la


def test_matrix_is_low_rank_product():
    N, A, R, c, gamma, Ainv, q, Gs, M = _setup()
    vol = np.linalg.det(A)
    pref, g4 = 4 * np.pi / vol, 1 / (4 * gamma ** 2)
    T = np.zeros((3 * N, 3 * N), complex)
    U = []
    for G in Gs:
        k = G + q; k2 = k @ k; E = np.exp(-k2 * g4)
        for i in range(N):
            for j in range(N):
                T[3 * i:3 * i + 3, 3 * j:3 * j + 3] += pref * np.outer(k, k) * E / k2 * np.exp(1j * G @ (R[j] - R[i]))
        U.append((np.sqrt(pref * E / k2) * np.exp(-1j * (R @ G))[:, None] * k[None, :]).reshape(-1))
    U = np.array(U).T
    assert np.abs(T - U @ U.conj().T).max() <= 1e-13 * np.abs(T).max()


def test_adjoint_low_rank_forms():
    args = _setup()
    ga_p, g_p, la_p = _pairwise(*args)
    ga_l, g_l, la_l = _lowrank(*args)
    assert np.abs(ga_l - ga_p).max() <= 1e-12 * np.abs(ga_p).max()
    assert np.abs(g_l - g_p).max() <= 1e-12 * np.abs(g_p).max()
    assert np.abs(la_l - la_p).max() <= 1e-12 * np.abs(la_p).max()
