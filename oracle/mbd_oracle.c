/*
 * mbd_oracle.c -- plain FP64 CPU oracle for the MBD energy and gradients.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  No product code may link or call it, and it
 * shares no code with the HIP path.
 *
 * Written from the paper (Hermann et al., arXiv:2308.03140):
 *   Sec. 2.1  eq:mbd-hamiltonian, eq:osc-param, eq:dipole, eq:q-matrix,
 *             eq:diagonalization, eq:mbd-energy
 *   Sec. 2.2  eq:brillouin-int, the Bloch sum of T, eq:ewald, eq:terfc
 *   Sec. 2.4  eq:mbd-gradient
 *   Sec. 2.5  eq:log-formula (frequency route), eq:dyn-pol
 *   Sec. 2.7  eq:fermi-damping, eq:mbd-lr-dipole (T^lr = g T, a = 6)
 *   Sec. 3.3  frequency grid map and Ewald defaults
 *
 * Readings where the paper is silent, ambiguous or at odds with itself:
 *   - T_ab = (delta_ab r^2 - 3 r_a r_b)/r^5, the explicit form of eq:dipole.
 *   - eq:terfc: T^erfc_ab = (delta_ab r^2 B - r_a r_b C)/r^5 (the printed 3 in
 *     front of r_a r_b C is already inside C; without it T^erfc -> T as
 *     gamma -> 0).
 *   - reciprocal phase exp(+i G.(R_j - R_i)) with k = G + q, consistent with
 *     the real-space phase exp(-i q.R_nij), R_nij = R_j + R_n - R_i.
 *   - the damped periodic tensor is the exact lattice sum of g T: the Ewald
 *     split of the bare T plus the real-space correction -(1-g) T, the latter
 *     summed over every image with (1-g) > 1e-18.
 *   - surface term and k = 0 omitted.
 *   - gradients as (1/4) Re Tr(Q^{-1/2} dQ/dX) - (3/2) d(sum omega)/dX.
 *
 * Eigenvalues come from the oracle's own cyclic Jacobi method (threshold
 * strategy, round-robin ordering so that disjoint rotations of one round can
 * be applied in parallel with OpenMP).  Hermitian matrices are handled by the
 * real embedding [[A, -B], [B, A]].
 */
#include "mbd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846264338327950288
#define DAMP_TAIL 1e-18

/* ------------------------------------------------------------------------- */
/* Pair tensors                                                               */
/* ------------------------------------------------------------------------- */

/* eq:dipole, explicit form; dT[c*9 + a*3 + b] = d T_ab / d r_c */
void orc_dipole(const double *r, double *T, double *dT)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double d = sqrt(r2);
    double r3 = r2 * d, r5 = r3 * r2, r7 = r5 * r2;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            T[a * 3 + b] = (a == b ? 1.0 / r3 : 0.0) - 3.0 * r[a] * r[b] / r5;
    if (!dT) return;
    for (int c = 0; c < 3; c++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double v = 15.0 * r[a] * r[b] * r[c] / r7;
                if (a == b) v -= 3.0 * r[c] / r5;
                if (a == c) v -= 3.0 * r[b] / r5;
                if (b == c) v -= 3.0 * r[a] / r5;
                dT[c * 9 + a * 3 + b] = v;
            }
}

/* eq:terfc (coefficient reading above). */
void orc_dipole_erfc(const double *r, double gamma, double *T, double *dT)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double d = sqrt(r2);
    double x = gamma * d;
    double ex = exp(-x * x);
    double B = erfc(x) + 2.0 * x / sqrt(PI) * ex;
    double C = 3.0 * erfc(x) + 2.0 * x / sqrt(PI) * (3.0 + 2.0 * x * x) * ex;
    double r3 = r2 * d, r5 = r3 * r2;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            T[a * 3 + b] = (a == b ? B / r3 : 0.0) - C * r[a] * r[b] / r5;
    if (!dT) return;
    /* dB/dd = -(4 gamma^3 d^2/sqrt(pi)) e^{-x^2};  dC/dd = -(8 gamma x^4/sqrt(pi)) e^{-x^2} */
    double dB = -4.0 * gamma * gamma * gamma * r2 / sqrt(PI) * ex;
    double dC = -8.0 * gamma * x * x * x * x / sqrt(PI) * ex;
    double db = dB / r3 - 3.0 * B / (r3 * d);     /* d(B/d^3)/dd */
    double dc = dC / r5 - 5.0 * C / (r5 * d);     /* d(C/d^5)/dd */
    for (int c = 0; c < 3; c++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double v = -dc * (r[c] / d) * r[a] * r[b];
                if (a == b) v += db * r[c] / d;
                if (a == c) v -= C * r[b] / r5;
                if (b == c) v -= C * r[a] / r5;
                dT[c * 9 + a * 3 + b] = v;
            }
}

/* eq:fermi-damping with s_R = beta (MBD: a = 6).  Returns g, 1-g (computed
 * without cancellation), dg/dd and dg/dR0 where R0 = beta (Rv_i + Rv_j). */
static void fermi(double d, double R0, double a, double *g, double *omg,
                  double *dg_dd, double *dg_dR0)
{
    if (R0 <= 0.0) { *g = 1.0; *omg = 0.0; *dg_dd = 0.0; *dg_dR0 = 0.0; return; }
    double x = a * (d / R0 - 1.0);
    if (x >= 0.0) { double e = exp(-x); *g = 1.0 / (1.0 + e); *omg = e / (1.0 + e); }
    else          { double e = exp(x);  *g = e / (1.0 + e);   *omg = 1.0 / (1.0 + e); }
    double gg = (*g) * (*omg);
    *dg_dd = a / R0 * gg;
    *dg_dR0 = -a * d / (R0 * R0) * gg;
}

/* ------------------------------------------------------------------------- */
/* Finite assembly, eq:q-matrix                                               */
/* ------------------------------------------------------------------------- */

void orc_assemble_finite(int N, const double *R, const double *alpha0,
                         const double *omega, const double *rvdw,
                         double beta, double a, double *Q)
{
    int n = 3 * N;
    memset(Q, 0, sizeof(double) * (size_t)n * n);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < N; i++) {
        double ci = omega[i] * sqrt(alpha0[i]);
        for (int j = 0; j < N; j++) {
            if (i == j) {
                for (int c = 0; c < 3; c++)
                    Q[(size_t)(3 * i + c) * n + 3 * i + c] = omega[i] * omega[i];
                continue;
            }
            double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1],
                           R[3 * j + 2] - R[3 * i + 2]};
            double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            double T[9], g, omg, gd, gR;
            orc_dipole(r, T, NULL);
            fermi(d, beta * (rvdw[i] + rvdw[j]), a, &g, &omg, &gd, &gR);
            double cc = ci * omega[j] * sqrt(alpha0[j]) * g;
            for (int p = 0; p < 3; p++)
                for (int s = 0; s < 3; s++)
                    Q[(size_t)(3 * i + p) * n + 3 * j + s] = cc * T[p * 3 + s];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Cyclic Jacobi (round-robin ordering)                                       */
/* ------------------------------------------------------------------------- */

int orc_jacobi(int n, double *A, double *w, double *V)
{
    if (n <= 0) return 0;
    if (V) {
        memset(V, 0, sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; i++) V[(size_t)i * n + i] = 1.0;
    }
    if (n == 1) { w[0] = A[0]; return 0; }
    int m = n + (n & 1);          /* players, one dummy if n is odd */
    int np = m / 2;
    int *pp = (int *)malloc(sizeof(int) * np), *qq = (int *)malloc(sizeof(int) * np);
    double *cs = (double *)malloc(sizeof(double) * np), *sn = (double *)malloc(sizeof(double) * np);
    int *slot = (int *)malloc(sizeof(int) * m);
    int sweeps = -1;
    for (int sweep = 0; sweep < 60; sweep++) {
        int rotated = 0;
        for (int rnd = 0; rnd < m - 1; rnd++) {
            slot[0] = 0;
            for (int s = 1; s < m; s++) slot[s] = 1 + (s - 1 + rnd) % (m - 1);
            int nact = 0;
            for (int k = 0; k < np; k++) {
                int p = slot[k], q = slot[m - 1 - k];
                if (p >= n || q >= n) continue;
                if (p > q) { int t = p; p = q; q = t; }
                double apq = A[(size_t)p * n + q];
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                if (fabs(apq) <= 1e-15 * sqrt(fabs(app * aqq)) || fabs(apq) < 1e-300)
                    continue;
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                pp[nact] = p; qq[nact] = q; cs[nact] = c; sn[nact] = t * c; nact++;
            }
            if (!nact) continue;
            rotated = 1;
            /* A <- A J (columns), V <- V J, row by row */
#pragma omp parallel for schedule(static)
            for (int r = 0; r < n; r++) {
                double *ar = A + (size_t)r * n;
                double *vr = V ? V + (size_t)r * n : NULL;
                for (int k = 0; k < nact; k++) {
                    int p = pp[k], q = qq[k];
                    double c = cs[k], s = sn[k];
                    double x = ar[p], y = ar[q];
                    ar[p] = c * x - s * y; ar[q] = s * x + c * y;
                    if (vr) { x = vr[p]; y = vr[q]; vr[p] = c * x - s * y; vr[q] = s * x + c * y; }
                }
            }
            /* A <- J^T A (rows), one pair per iteration */
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nact; k++) {
                int p = pp[k], q = qq[k];
                double c = cs[k], s = sn[k];
                double *ap = A + (size_t)p * n, *aq = A + (size_t)q * n;
                for (int col = 0; col < n; col++) {
                    double x = ap[col], y = aq[col];
                    ap[col] = c * x - s * y; aq[col] = s * x + c * y;
                }
                ap[q] = 0.0; aq[p] = 0.0;
            }
        }
        if (!rotated) { sweeps = sweep; break; }
    }
    for (int i = 0; i < n; i++) w[i] = A[(size_t)i * n + i];
    /* sort ascending (selection sort keeps it plain), permuting V columns */
    for (int i = 0; i < n - 1; i++) {
        int k = i;
        for (int j = i + 1; j < n; j++) if (w[j] < w[k]) k = j;
        if (k != i) {
            double t = w[i]; w[i] = w[k]; w[k] = t;
            if (V) for (int r = 0; r < n; r++) {
                double *vr = V + (size_t)r * n;
                t = vr[i]; vr[i] = vr[k]; vr[k] = t;
            }
        }
    }
    free(pp); free(qq); free(cs); free(sn); free(slot);
    return sweeps;
}

int orc_jacobi_hermitian(int n, const double *Are, const double *Aim,
                         double *w, double *V)
{
    int m = 2 * n;
    double *E = (double *)malloc(sizeof(double) * (size_t)m * m);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double re = Are[(size_t)i * n + j], im = Aim[(size_t)i * n + j];
            E[(size_t)i * m + j] = re;
            E[(size_t)(i + n) * m + j + n] = re;
            E[(size_t)i * m + j + n] = -im;
            E[(size_t)(i + n) * m + j] = im;
        }
    int s = orc_jacobi(m, E, w, V);
    free(E);
    return s;
}

/* M = V diag(lam^{-1/2}) V^T, plain triple loop */
static void inv_sqrt_from_eig(int n, const double *V, const double *lam, double *M)
{
    double *s = (double *)malloc(sizeof(double) * n);
    for (int k = 0; k < n; k++) s[k] = 1.0 / sqrt(lam[k]);
#pragma omp parallel for schedule(dynamic)
    for (int p = 0; p < n; p++)
        for (int q = 0; q < n; q++) {
            double acc = 0.0;
            const double *vp = V + (size_t)p * n, *vq = V + (size_t)q * n;
            for (int k = 0; k < n; k++) acc += vp[k] * s[k] * vq[k];
            M[(size_t)p * n + q] = acc;
        }
    free(s);
}

/* Neumaier-compensated sum of sqrt(lam) */
static double sum_sqrt(int n, const double *lam)
{
    double s = 0.0, c = 0.0;
    for (int k = 0; k < n; k++) {
        double x = sqrt(lam[k]);
        double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------- */
/* Finite energy and gradients                                                */
/* ------------------------------------------------------------------------- */

int orc_mbd_finite(int N, const double *R, const double *alpha0,
                   const double *omega, const double *rvdw, double beta,
                   double a, double *energy, double *grad_R,
                   double *grad_alpha0, double *grad_omega, double *grad_rvdw,
                   double *eigs)
{
    if (N < 1) return 1;
    int n = 3 * N;
    int want_grad = grad_R || grad_alpha0 || grad_omega || grad_rvdw;
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *lam = (double *)malloc(sizeof(double) * n);
    double *V = want_grad ? (double *)malloc(sizeof(double) * (size_t)n * n) : NULL;
    orc_assemble_finite(N, R, alpha0, omega, rvdw, beta, a, Q);
    int sw = orc_jacobi(n, Q, lam, V);
    if (eigs) memcpy(eigs, lam, sizeof(double) * n);
    int rc = 0;
    if (sw < 0) rc = 3;
    else if (lam[0] <= 0.0) rc = 2;
    if (rc) {
        if (energy) *energy = NAN;
        free(Q); free(lam); free(V);
        return rc;
    }
    double som = 0.0;
    for (int i = 0; i < N; i++) som += omega[i];
    if (energy) *energy = 0.5 * sum_sqrt(n, lam) - 1.5 * som;
    if (want_grad) {
        double *M = Q; /* reuse storage */
        inv_sqrt_from_eig(n, V, lam, M);
        double *gR = (double *)calloc((size_t)3 * N, sizeof(double));
        double *S = (double *)calloc(N, sizeof(double));
        double *U = (double *)calloc(N, sizeof(double));
        for (int i = 0; i < N; i++) {
            double ci = omega[i] * sqrt(alpha0[i]);
            for (int j = i + 1; j < N; j++) {
                double cj = omega[j] * sqrt(alpha0[j]);
                double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1],
                               R[3 * j + 2] - R[3 * i + 2]};
                double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                double T[9], dT[27], g, omg, gd, gR0;
                orc_dipole(r, T, dT);
                fermi(d, beta * (rvdw[i] + rvdw[j]), a, &g, &omg, &gd, &gR0);
                double f[3] = {0, 0, 0}, s = 0.0, u = 0.0;
                for (int p = 0; p < 3; p++)
                    for (int q = 0; q < 3; q++) {
                        double m = M[(size_t)(3 * i + p) * n + 3 * j + q];
                        s += m * g * T[p * 3 + q];
                        u += m * T[p * 3 + q];
                        for (int c = 0; c < 3; c++)
                            f[c] += m * (gd * r[c] / d * T[p * 3 + q] + g * dT[c * 9 + p * 3 + q]);
                    }
                for (int c = 0; c < 3; c++) {
                    double fc = 0.5 * ci * cj * f[c];
                    gR[3 * i + c] -= fc;
                    gR[3 * j + c] += fc;
                }
                S[i] += ci * cj * s; S[j] += ci * cj * s;
                double uu = 0.5 * ci * cj * beta * gR0 * u;
                U[i] += uu; U[j] += uu;
            }
        }
        for (int i = 0; i < N; i++) {
            double tr = 0.0;
            for (int c = 0; c < 3; c++) tr += M[(size_t)(3 * i + c) * n + 3 * i + c];
            if (grad_alpha0) grad_alpha0[i] = S[i] / (4.0 * alpha0[i]);
            if (grad_omega) grad_omega[i] = S[i] / (2.0 * omega[i]) + 0.5 * omega[i] * tr - 1.5;
            if (grad_rvdw) grad_rvdw[i] = U[i];
            if (grad_R) for (int c = 0; c < 3; c++) grad_R[3 * i + c] = gR[3 * i + c];
        }
        free(gR); free(S); free(U);
    }
    free(Q); free(lam); free(V);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Periodic: lattice helpers and Bloch sums                                  */
/* ------------------------------------------------------------------------- */

static double det3(const double *A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Ainv[d*3+u] = (A^{-1})_{du} */
static void inv3(const double *A, double *Ainv)
{
    double dt = det3(A);
    Ainv[0] = (A[4] * A[8] - A[5] * A[7]) / dt;
    Ainv[1] = (A[2] * A[7] - A[1] * A[8]) / dt;
    Ainv[2] = (A[1] * A[5] - A[2] * A[4]) / dt;
    Ainv[3] = (A[5] * A[6] - A[3] * A[8]) / dt;
    Ainv[4] = (A[0] * A[8] - A[2] * A[6]) / dt;
    Ainv[5] = (A[2] * A[3] - A[0] * A[5]) / dt;
    Ainv[6] = (A[3] * A[7] - A[4] * A[6]) / dt;
    Ainv[7] = (A[1] * A[6] - A[0] * A[7]) / dt;
    Ainv[8] = (A[0] * A[4] - A[1] * A[3]) / dt;
}

void orc_ewald_defaults(const double *lattice, double *gamma, double *rc, double *kc)
{
    double vol = fabs(det3(lattice));
    *gamma = 2.5 / cbrt(vol);
    *rc = 6.0 / *gamma;
    *kc = 10.0 * *gamma;
}

typedef struct {
    double A[9], Ainv[9], B[9]; /* B rows = reciprocal vectors b_u, B_ud = 2 pi Ainv_du */
    double vol;
    int nimg; int *img;         /* integer triplets n */
    int nrec; int *rec;         /* integer triplets m */
    double gamma, rc, kc;
} lattice_t;

static double norm3(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

static void lattice_setup(lattice_t *L, const double *lattice, double gamma,
                          double rc, double kc, double rreal, double rmaxpair,
                          double qmax)
{
    memcpy(L->A, lattice, sizeof(double) * 9);
    inv3(L->A, L->Ainv);
    for (int u = 0; u < 3; u++)
        for (int d = 0; d < 3; d++) L->B[u * 3 + d] = 2.0 * PI * L->Ainv[d * 3 + u];
    L->vol = fabs(det3(L->A));
    L->gamma = gamma; L->rc = rc; L->kc = kc;
    int nv[3], mv[3];
    for (int v = 0; v < 3; v++) {
        nv[v] = (int)ceil((rreal + rmaxpair) * norm3(L->B + 3 * v) / (2.0 * PI)) + 1;
        mv[v] = (int)ceil((kc + qmax) * norm3(L->A + 3 * v) / (2.0 * PI)) + 1;
    }
    L->nimg = (2 * nv[0] + 1) * (2 * nv[1] + 1) * (2 * nv[2] + 1);
    L->img = (int *)malloc(sizeof(int) * 3 * L->nimg);
    int t = 0;
    for (int x = -nv[0]; x <= nv[0]; x++)
        for (int y = -nv[1]; y <= nv[1]; y++)
            for (int z = -nv[2]; z <= nv[2]; z++) {
                L->img[3 * t] = x; L->img[3 * t + 1] = y; L->img[3 * t + 2] = z; t++;
            }
    L->nrec = (2 * mv[0] + 1) * (2 * mv[1] + 1) * (2 * mv[2] + 1);
    L->rec = (int *)malloc(sizeof(int) * 3 * L->nrec);
    t = 0;
    for (int x = -mv[0]; x <= mv[0]; x++)
        for (int y = -mv[1]; y <= mv[1]; y++)
            for (int z = -mv[2]; z <= mv[2]; z++) {
                L->rec[3 * t] = x; L->rec[3 * t + 1] = y; L->rec[3 * t + 2] = z; t++;
            }
}

static void lattice_free(lattice_t *L) { free(L->img); free(L->rec); }

/* Bloch-summed damped tensor for one ordered pair, r = R_j - R_i.
 * Outputs (each 9 complex = re/im arrays):
 *   T[ab]            T_ij(q)
 *   dR[c][ab]        d/dr_c
 *   dA[v][c][ab]     d/dA_vc (Cartesian positions, fractional q fixed)
 *   d0[ab]           d/dR0, R0 = beta (Rv_i + Rv_j) the damping radius (only
 *                    the damping correction -(1-g) T depends on it)
 * dR, dA, d0 may be NULL. */
static void bloch_pair(const lattice_t *L, const double *r, int self,
                       const double *q, double R0, double a,
                       double *Tre, double *Tim, double *dRre, double *dRim,
                       double *dAre, double *dAim, double *d0re, double *d0im)
{
    const double gamma = L->gamma;
    memset(Tre, 0, 9 * sizeof(double)); memset(Tim, 0, 9 * sizeof(double));
    if (dRre) { memset(dRre, 0, 27 * sizeof(double)); memset(dRim, 0, 27 * sizeof(double)); }
    if (dAre) { memset(dAre, 0, 81 * sizeof(double)); memset(dAim, 0, 81 * sizeof(double)); }
    if (d0re) { memset(d0re, 0, 9 * sizeof(double)); memset(d0im, 0, 9 * sizeof(double)); }
    double rho[3];
    for (int v = 0; v < 3; v++) {
        rho[v] = 0.0;
        for (int d = 0; d < 3; d++) rho[v] += L->Ainv[d * 3 + v] * r[d];
    }
    /* real space */
    for (int t = 0; t < L->nimg; t++) {
        const int *nn = L->img + 3 * t;
        double x[3];
        for (int d = 0; d < 3; d++)
            x[d] = r[d] + nn[0] * L->A[d] + nn[1] * L->A[3 + d] + nn[2] * L->A[6 + d];
        double dist = norm3(x);
        if (dist == 0.0) continue;  /* n = 0, i = j */
        double F[9] = {0}, dF[27] = {0}, F0[9] = {0};
        int any = 0;
        if (dist < L->rc) {
            double Te[9], dTe[27];
            orc_dipole_erfc(x, gamma, Te, dTe);
            for (int k = 0; k < 9; k++) F[k] += Te[k];
            for (int k = 0; k < 27; k++) dF[k] += dTe[k];
            any = 1;
        }
        double g, omg, gd, gR0;
        fermi(dist, R0, a, &g, &omg, &gd, &gR0);
        if (omg > DAMP_TAIL) {
            double T0[9], dT0[27];
            orc_dipole(x, T0, dT0);
            for (int k = 0; k < 9; k++) { F[k] -= omg * T0[k]; F0[k] = gR0 * T0[k]; }
            for (int c = 0; c < 3; c++)
                for (int k = 0; k < 9; k++)
                    dF[c * 9 + k] -= omg * dT0[c * 9 + k] - gd * x[c] / dist * T0[k];
            any = 1;
        }
        if (!any) continue;
        double ph = -(q[0] * x[0] + q[1] * x[1] + q[2] * x[2]);
        double cph = cos(ph), sph = sin(ph);
        for (int k = 0; k < 9; k++) { Tre[k] += F[k] * cph; Tim[k] += F[k] * sph; }
        if (d0re)
            for (int k = 0; k < 9; k++) { d0re[k] += F0[k] * cph; d0im[k] += F0[k] * sph; }
        if (dRre)
            for (int c = 0; c < 3; c++)
                for (int k = 0; k < 9; k++) {
                    /* (dF_c - i q_c F) e^{i ph} */
                    double are = dF[c * 9 + k], aim = -q[c] * F[k];
                    dRre[c * 9 + k] += are * cph - aim * sph;
                    dRim[c * 9 + k] += are * sph + aim * cph;
                }
        if (dAre)
            for (int v = 0; v < 3; v++)
                for (int c = 0; c < 3; c++)
                    for (int k = 0; k < 9; k++) {
                        /* (dF_c n_v + i q_c rho_v F) e^{i ph} */
                        double are = dF[c * 9 + k] * nn[v], aim = q[c] * rho[v] * F[k];
                        dAre[(v * 3 + c) * 9 + k] += are * cph - aim * sph;
                        dAim[(v * 3 + c) * 9 + k] += are * sph + aim * cph;
                    }
    }
    /* reciprocal space */
    double pref = 4.0 * PI / L->vol;
    for (int t = 0; t < L->nrec; t++) {
        const int *mm = L->rec + 3 * t;
        double G[3], k[3];
        for (int d = 0; d < 3; d++) {
            G[d] = mm[0] * L->B[d] + mm[1] * L->B[3 + d] + mm[2] * L->B[6 + d];
            k[d] = G[d] + q[d];
        }
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double kn = sqrt(k2);
        if (kn == 0.0 || kn >= L->kc) continue;
        double E = exp(-k2 / (4.0 * gamma * gamma));
        double h[9];
        for (int aa = 0; aa < 3; aa++)
            for (int bb = 0; bb < 3; bb++) h[aa * 3 + bb] = k[aa] * k[bb] / k2 * E;
        double ph = G[0] * r[0] + G[1] * r[1] + G[2] * r[2];
        double cph = cos(ph), sph = sin(ph);
        for (int kk = 0; kk < 9; kk++) { Tre[kk] += pref * h[kk] * cph; Tim[kk] += pref * h[kk] * sph; }
        if (dRre)
            for (int c = 0; c < 3; c++)
                for (int kk = 0; kk < 9; kk++) {
                    /* pref h (i G_c) e^{i ph} */
                    dRre[c * 9 + kk] += -pref * h[kk] * G[c] * sph;
                    dRim[c * 9 + kk] += pref * h[kk] * G[c] * cph;
                }
        if (dAre) {
            /* dh_ab/dk_d */
            double dh[27];
            for (int d = 0; d < 3; d++)
                for (int aa = 0; aa < 3; aa++)
                    for (int bb = 0; bb < 3; bb++) {
                        double v = -2.0 * k[aa] * k[bb] * k[d] / (k2 * k2) * E
                                   - k[aa] * k[bb] / k2 * E * k[d] / (2.0 * gamma * gamma);
                        if (aa == d) v += k[bb] / k2 * E;
                        if (bb == d) v += k[aa] / k2 * E;
                        dh[d * 9 + aa * 3 + bb] = v;
                    }
            for (int v = 0; v < 3; v++)
                for (int c = 0; c < 3; c++)
                    for (int kk = 0; kk < 9; kk++) {
                        double dhv = 0.0;
                        for (int d = 0; d < 3; d++) dhv += dh[d * 9 + kk] * L->Ainv[d * 3 + v];
                        /* d(pref)/dA_vc = -pref Ainv_cv ; dk_d/dA_vc = -Ainv_dv k_c ;
                           d(G.r)/dA_vc = -G_c rho_v */
                        double re = -L->Ainv[c * 3 + v] * h[kk] - k[c] * dhv;
                        double im = -h[kk] * G[c] * rho[v];
                        dAre[(v * 3 + c) * 9 + kk] += pref * (re * cph - im * sph);
                        dAim[(v * 3 + c) * 9 + kk] += pref * (re * sph + im * cph);
                    }
        }
    }
    if (self) {
        double s = 4.0 * gamma * gamma * gamma / (3.0 * sqrt(PI));
        Tre[0] -= s; Tre[4] -= s; Tre[8] -= s;
    }
}

static void pair_extent(int N, const double *R, double *maxd)
{
    double m = 0.0;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
            double d = norm3(r);
            if (d > m) m = d;
        }
    *maxd = m;
}

static double damp_range(int N, const double *rvdw, double beta, double a)
{
    if (beta <= 0.0) return 0.0;
    double mx = 0.0;
    for (int i = 0; i < N; i++) if (rvdw[i] > mx) mx = rvdw[i];
    /* (1-g) > DAMP_TAIL  <=>  eta < 1 + ln(1/DAMP_TAIL - 1)/a */
    return (1.0 + log(1.0 / DAMP_TAIL - 1.0) / a) * beta * 2.0 * mx * 1.0000001;
}

int orc_assemble_periodic(int N, const double *R, const double *lattice,
                          const double *q, double gamma, double rc, double kc,
                          const double *alpha0, const double *omega,
                          const double *rvdw, double beta, double a,
                          double *Qre, double *Qim)
{
    if (N < 1 || det3(lattice) <= 0.0) return 1;
    int n = 3 * N;
    double maxd;
    pair_extent(N, R, &maxd);
    double rreal = rc > damp_range(N, rvdw, beta, a) ? rc : damp_range(N, rvdw, beta, a);
    lattice_t L;
    lattice_setup(&L, lattice, gamma, rc, kc, rreal, maxd, norm3(q));
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < N; i++) {
        double ci = omega[i] * sqrt(alpha0[i]);
        for (int j = 0; j < N; j++) {
            double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
            double Tre[9], Tim[9];
            bloch_pair(&L, r, i == j, q, beta * (rvdw[i] + rvdw[j]), a, Tre, Tim,
                       NULL, NULL, NULL, NULL, NULL, NULL);
            double cc = ci * omega[j] * sqrt(alpha0[j]);
            for (int p = 0; p < 3; p++)
                for (int s = 0; s < 3; s++) {
                    Qre[(size_t)(3 * i + p) * n + 3 * j + s] =
                        cc * Tre[p * 3 + s] + (i == j && p == s ? omega[i] * omega[i] : 0.0);
                    Qim[(size_t)(3 * i + p) * n + 3 * j + s] = cc * Tim[p * 3 + s];
                }
        }
    }
    lattice_free(&L);
    return 0;
}

int orc_mbd_periodic(int N, const double *R, const double *lattice, int nq,
                     const double *q_frac, double gamma, double rc, double kc,
                     const double *alpha0, const double *omega,
                     const double *rvdw, double beta, double a,
                     double *energy, double *grad_R, double *grad_alpha0,
                     double *grad_omega, double *grad_rvdw,
                     double *grad_lattice, double *eigs)
{
    if (N < 1 || nq < 1 || det3(lattice) <= 0.0) return 1;
    int n = 3 * N, m = 2 * n;
    int want_grad = grad_R || grad_alpha0 || grad_omega || grad_rvdw || grad_lattice;
    double Ainv[9], B[9];
    inv3(lattice, Ainv);
    for (int u = 0; u < 3; u++)
        for (int d = 0; d < 3; d++) B[u * 3 + d] = 2.0 * PI * Ainv[d * 3 + u];
    double maxd;
    pair_extent(N, R, &maxd);
    double dr = damp_range(N, rvdw, beta, a);
    double rreal = rc > dr ? rc : dr;
    double qmax = 0.0;
    for (int t = 0; t < nq; t++) {
        double qq[3];
        for (int d = 0; d < 3; d++)
            qq[d] = q_frac[3 * t] * B[d] + q_frac[3 * t + 1] * B[3 + d] + q_frac[3 * t + 2] * B[6 + d];
        if (norm3(qq) > qmax) qmax = norm3(qq);
    }
    lattice_t L;
    lattice_setup(&L, lattice, gamma, rc, kc, rreal, maxd, qmax);
    double *Qre = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *Qim = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *lam = (double *)malloc(sizeof(double) * m);
    double *V = want_grad ? (double *)malloc(sizeof(double) * (size_t)m * m) : NULL;
    double *ME = want_grad ? (double *)malloc(sizeof(double) * (size_t)m * m) : NULL;
    double som = 0.0;
    for (int i = 0; i < N; i++) som += omega[i];
    double esum = 0.0;
    if (grad_R) memset(grad_R, 0, sizeof(double) * 3 * N);
    if (grad_alpha0) memset(grad_alpha0, 0, sizeof(double) * N);
    if (grad_omega) memset(grad_omega, 0, sizeof(double) * N);
    if (grad_rvdw) memset(grad_rvdw, 0, sizeof(double) * N);
    if (grad_lattice) memset(grad_lattice, 0, sizeof(double) * 9);
    int rc_out = 0;
    for (int t = 0; t < nq; t++) {
        double q[3];
        for (int d = 0; d < 3; d++)
            q[d] = q_frac[3 * t] * B[d] + q_frac[3 * t + 1] * B[3 + d] + q_frac[3 * t + 2] * B[6 + d];
        orc_assemble_periodic(N, R, lattice, q, gamma, rc, kc, alpha0, omega, rvdw,
                              beta, a, Qre, Qim);
        int sw = orc_jacobi_hermitian(n, Qre, Qim, lam, V);
        if (sw < 0) { rc_out = 3; break; }
        if (lam[0] <= 0.0) { rc_out = 2; break; }
        if (eigs) for (int k = 0; k < n; k++) eigs[(size_t)t * n + k] = lam[2 * k];
        esum += 0.25 * sum_sqrt(m, lam) - 1.5 * som;
        if (!want_grad) continue;
        inv_sqrt_from_eig(m, V, lam, ME);
        /* M = ME[0:n,0:n] + i ME[n:2n, 0:n] */
        double wq = 1.0 / nq;
        double *gRloc = (double *)calloc((size_t)3 * N, sizeof(double));
        double *galoc = (double *)calloc(N, sizeof(double));
        double *gwloc = (double *)calloc(N, sizeof(double));
        double *gvloc = (double *)calloc(N, sizeof(double));
        double gl[9] = {0};
#pragma omp parallel
        {
            double *gRt = (double *)calloc((size_t)3 * N, sizeof(double));
            double *gat = (double *)calloc(N, sizeof(double));
            double *gwt = (double *)calloc(N, sizeof(double));
            double *gvt = (double *)calloc(N, sizeof(double));
            double glt[9] = {0};
#pragma omp for schedule(dynamic)
            for (int i = 0; i < N; i++) {
                double ci = omega[i] * sqrt(alpha0[i]);
                for (int j = 0; j < N; j++) {
                    double cj = omega[j] * sqrt(alpha0[j]);
                    double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
                    double Tre[9], Tim[9], dRre[27], dRim[27], dAre[81], dAim[81], d0re[9], d0im[9];
                    bloch_pair(&L, r, i == j, q, beta * (rvdw[i] + rvdw[j]), a, Tre, Tim,
                               dRre, dRim, dAre, dAim, d0re, d0im);
                    double cc = ci * cj;
                    /* M_{jb,ia} */
                    double Mre[9], Mim[9];
                    for (int aa = 0; aa < 3; aa++)
                        for (int bb = 0; bb < 3; bb++) {
                            Mre[aa * 3 + bb] = ME[(size_t)(3 * j + bb) * m + 3 * i + aa];
                            Mim[aa * 3 + bb] = ME[(size_t)(n + 3 * j + bb) * m + 3 * i + aa];
                        }
                    double P = 0.0;
                    for (int k = 0; k < 9; k++) P += Mre[k] * Tre[k] - Mim[k] * Tim[k];
                    gat[i] += 0.25 * wq * cc * P / (2.0 * alpha0[i]);
                    gat[j] += 0.25 * wq * cc * P / (2.0 * alpha0[j]);
                    /* c_i = omega_i sqrt(alpha0_i): dc_i/domega_i = c_i/omega_i */
                    gwt[i] += 0.25 * wq * cc * P / omega[i];
                    gwt[j] += 0.25 * wq * cc * P / omega[j];
                    /* R0 = beta (Rv_i + Rv_j) */
                    double P0 = 0.0;
                    for (int k = 0; k < 9; k++) P0 += Mre[k] * d0re[k] - Mim[k] * d0im[k];
                    gvt[i] += 0.25 * wq * cc * beta * P0;
                    gvt[j] += 0.25 * wq * cc * beta * P0;
                    if (i != j)
                        for (int c = 0; c < 3; c++) {
                            double X = 0.0;
                            for (int k = 0; k < 9; k++)
                                X += Mre[k] * dRre[c * 9 + k] - Mim[k] * dRim[c * 9 + k];
                            gRt[3 * j + c] += 0.25 * wq * cc * X;
                            gRt[3 * i + c] -= 0.25 * wq * cc * X;
                        }
                    for (int vc = 0; vc < 9; vc++) {
                        double X = 0.0;
                        for (int k = 0; k < 9; k++)
                            X += Mre[k] * dAre[vc * 9 + k] - Mim[k] * dAim[vc * 9 + k];
                        glt[vc] += 0.25 * wq * cc * X;
                    }
                }
            }
#pragma omp critical
            {
                for (int k = 0; k < 3 * N; k++) gRloc[k] += gRt[k];
                for (int k = 0; k < N; k++) galoc[k] += gat[k];
                for (int k = 0; k < N; k++) gwloc[k] += gwt[k];
                for (int k = 0; k < N; k++) gvloc[k] += gvt[k];
                for (int k = 0; k < 9; k++) gl[k] += glt[k];
            }
            free(gRt); free(gat); free(gwt); free(gvt);
        }
        /* omega_i^2 on the diagonal of Q(q): (1/4) 2 omega_i Re Tr M_ii */
        for (int i = 0; i < N; i++) {
            double tr = 0.0;
            for (int c = 0; c < 3; c++) tr += ME[(size_t)(3 * i + c) * m + 3 * i + c];
            gwloc[i] += 0.25 * wq * 2.0 * omega[i] * tr;
        }
        if (grad_R) for (int k = 0; k < 3 * N; k++) grad_R[k] += gRloc[k];
        if (grad_alpha0) for (int k = 0; k < N; k++) grad_alpha0[k] += galoc[k];
        if (grad_omega) for (int k = 0; k < N; k++) grad_omega[k] += gwloc[k];
        if (grad_rvdw) for (int k = 0; k < N; k++) grad_rvdw[k] += gvloc[k];
        if (grad_lattice) for (int k = 0; k < 9; k++) grad_lattice[k] += gl[k];
        free(gRloc); free(galoc); free(gwloc); free(gvloc);
    }
    /* -(3/2) sum_i omega_i */
    if (grad_omega && !rc_out) for (int k = 0; k < N; k++) grad_omega[k] -= 1.5;
    if (energy) *energy = rc_out ? NAN : esum / nq;
    lattice_free(&L);
    free(Qre); free(Qim); free(lam); free(V); free(ME);
    return rc_out;
}

/* ------------------------------------------------------------------------- */
/* Frequency route (eq:log-formula) with the oracle's own Cholesky            */
/* ------------------------------------------------------------------------- */

void orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; i++) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= n; k++) {
                double p3 = p2; p2 = p1;
                p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* dot product with four partial sums (plain, but not latency-bound) */
static double dot4(const double *x, const double *y, int n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 3 < n; k += 4) {
        s0 += x[k] * y[k]; s1 += x[k + 1] * y[k + 1];
        s2 += x[k + 2] * y[k + 2]; s3 += x[k + 3] * y[k + 3];
    }
    for (; k < n; k++) s0 += x[k] * y[k];
    return (s0 + s1) + (s2 + s3);
}

/* In-place lower Cholesky of a row-major SPD matrix; returns 0 or 2 if not PD. */
static int cholesky(int n, double *A)
{
    for (int j = 0; j < n; j++) {
        double *aj = A + (size_t)j * n;
        double s = aj[j] - dot4(aj, aj, j);
        if (!(s > 0.0)) return 2;
        double l = sqrt(s);
        aj[j] = l;
#pragma omp parallel for schedule(static)
        for (int i = j + 1; i < n; i++) {
            double *ai = A + (size_t)i * n;
            ai[j] = (ai[j] - dot4(ai, aj, j)) / l;
        }
    }
    return 0;
}

/* Lower Cholesky of I + K (K row-major, overwritten by L) for the frequency
 * route, where I + K is close to the identity at large imaginary frequency:
 * each pivot is carried as its deviation e_j from 1, so that
 * ln det(I + K) = sum_j log1p(e_j) keeps its relative accuracy instead of
 * losing it to log(1 + tiny).  Returns 0, or 2 if not positive definite. */
static int cholesky_unit_shift(int n, double *K, double *logdet)
{
    double ld = 0.0;
    for (int j = 0; j < n; j++) {
        double *kj = K + (size_t)j * n;
        double e = kj[j] - dot4(kj, kj, j);
        if (!(1.0 + e > 0.0)) return 2;
        double l = sqrt(1.0 + e);
        kj[j] = l;
        ld += log1p(e);
#pragma omp parallel for schedule(static)
        for (int i = j + 1; i < n; i++) {
            double *ki = K + (size_t)i * n;
            ki[j] = (ki[j] - dot4(ki, kj, j)) / l;
        }
    }
    *logdet = ld;
    return 0;
}

int orc_is_positive_definite(int n, const double *A)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)n * n);
    memcpy(C, A, sizeof(double) * (size_t)n * n);
    int rc = cholesky(n, C);
    free(C);
    return rc == 0;
}

int orc_mbd_finite_freq(int N, const double *R, const double *alpha0,
                        const double *omega, const double *rvdw, double beta,
                        double a, int npts, double *energy, int nsample,
                        const int *atoms, double *grad_R_sample,
                        double *grad_alpha0_sample, double *grad_omega_sample)
{
    if (N < 1 || npts < 1) return 1;
    int n = 3 * N;
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *S = (double *)malloc(sizeof(double) * (size_t)n * n);
    orc_assemble_finite(N, R, alpha0, omega, rvdw, beta, a, Q);
    double *x = (double *)malloc(sizeof(double) * npts), *w = (double *)malloc(sizeof(double) * npts);
    orc_gauss_legendre(npts, x, w);
    double *Mrows = nsample > 0 ? (double *)calloc((size_t)nsample * 3 * n, sizeof(double)) : NULL;
    double *y = (double *)malloc(sizeof(double) * n);
    double *dsc = (double *)malloc(sizeof(double) * n);
    double etot = 0.0;
    int rc = 0;
    for (int t = 0; t < npts && !rc; t++) {
        double u = 0.6 * (1.0 + x[t]) / (1.0 - x[t]);
        double du = 0.6 * 2.0 / ((1.0 - x[t]) * (1.0 - x[t])) * w[t];
        /* I + alpha(iu)^{1/2} T alpha(iu)^{1/2} = D^{-1}(Q + u^2)D^{-1} = I + K,
         * D = (Omega^2 + u^2)^{1/2}, K = D^{-1}(Q - Omega^2)D^{-1} */
        for (int p = 0; p < n; p++) {
            double om = omega[p / 3];
            dsc[p] = 1.0 / sqrt(om * om + u * u);
        }
#pragma omp parallel for schedule(static)
        for (int p = 0; p < n; p++) {
            double om = omega[p / 3];
            for (int s = 0; s < n; s++)
                S[(size_t)p * n + s] = (Q[(size_t)p * n + s] - (p == s ? om * om : 0.0)) * dsc[p] * dsc[s];
        }
        double ld = 0.0;
        if (cholesky_unit_shift(n, S, &ld)) { rc = 2; break; }
        etot += du * ld / (2.0 * PI);
        /* rows of (Q + u^2)^{-1} = D^{-1} S^{-1} D^{-1} for the sampled atoms */
        for (int sa = 0; sa < nsample; sa++)
            for (int c = 0; c < 3; c++) {
                int col = 3 * atoms[sa] + c;
                for (int p = 0; p < n; p++) y[p] = (p == col) ? dsc[p] : 0.0;
                for (int p = 0; p < n; p++) {         /* L y = b */
                    double acc = y[p];
                    const double *sp = S + (size_t)p * n;
                    for (int k = 0; k < p; k++) acc -= sp[k] * y[k];
                    y[p] = acc / sp[p];
                }
                for (int p = n - 1; p >= 0; p--) {    /* L^T z = y */
                    double acc = y[p];
                    for (int k = p + 1; k < n; k++) acc -= S[(size_t)k * n + p] * y[k];
                    y[p] = acc / S[(size_t)p * n + p];
                }
                double *mr = Mrows + ((size_t)sa * 3 + c) * n;
                for (int p = 0; p < n; p++) mr[p] += (2.0 / PI) * du * y[p] * dsc[p];
            }
    }
    if (energy) *energy = rc ? NAN : etot;
    if (!rc && nsample > 0) {
        for (int sa = 0; sa < nsample; sa++) {
            int k = atoms[sa];
            double ck = omega[k] * sqrt(alpha0[k]);
            double gk[3] = {0, 0, 0}, Sk = 0.0;
            for (int j = 0; j < N; j++) {
                if (j == k) continue;
                double cj = omega[j] * sqrt(alpha0[j]);
                double r[3] = {R[3 * j] - R[3 * k], R[3 * j + 1] - R[3 * k + 1], R[3 * j + 2] - R[3 * k + 2]};
                double d = norm3(r);
                double T[9], dT[27], g, omg, gd, gR0;
                orc_dipole(r, T, dT);
                fermi(d, beta * (rvdw[k] + rvdw[j]), a, &g, &omg, &gd, &gR0);
                /* S_k = sum_j c_k c_j sum_ab M_{ka,jb} g T_ab */
                for (int p = 0; p < 3; p++)
                    for (int s2 = 0; s2 < 3; s2++)
                        Sk += ck * cj * Mrows[((size_t)sa * 3 + p) * n + 3 * j + s2] * g * T[p * 3 + s2];
                for (int c = 0; c < 3; c++) {
                    double acc = 0.0;
                    for (int p = 0; p < 3; p++)
                        for (int s = 0; s < 3; s++) {
                            double mm = Mrows[((size_t)sa * 3 + p) * n + 3 * j + s];
                            acc += mm * (gd * r[c] / d * T[p * 3 + s] + g * dT[c * 9 + p * 3 + s]);
                        }
                    gk[c] -= 0.5 * ck * cj * acc;
                }
            }
            if (grad_R_sample) for (int c = 0; c < 3; c++) grad_R_sample[3 * sa + c] = gk[c];
            /* dQ/dalpha0_k and dQ/domega_k through c_k and the omega_k^2
             * diagonal: (1/4) Tr(M dQ) as in the eigenvalue route */
            double tr = 0.0;
            for (int c = 0; c < 3; c++) tr += Mrows[((size_t)sa * 3 + c) * n + 3 * k + c];
            if (grad_alpha0_sample) grad_alpha0_sample[sa] = Sk / (4.0 * alpha0[k]);
            if (grad_omega_sample) grad_omega_sample[sa] = Sk / (2.0 * omega[k]) + 0.5 * omega[k] * tr - 1.5;
        }
    }
    free(Q); free(S); free(x); free(w); free(Mrows); free(y); free(dsc);
    return rc;
}

int orc_min_coupling_eig(int N, const double *R, const double *alpha0,
                         const double *rvdw, double beta, double a,
                         double *mu_min)
{
    int n = 3 * N;
    double *om = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; i++) om[i] = 1.0;
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *lam = (double *)malloc(sizeof(double) * n);
    /* with omega = 1: Q = I + alpha^{1/2} T alpha^{1/2} */
    orc_assemble_finite(N, R, alpha0, om, rvdw, beta, a, Q);
    for (int p = 0; p < n; p++) Q[(size_t)p * n + p] -= 1.0;
    int sw = orc_jacobi(n, Q, lam, NULL);
    *mu_min = lam[0];
    free(om); free(Q); free(lam);
    return sw < 0 ? 3 : 0;
}

/* ------------------------------------------------------------------------- */
/* Pairwise (TS) dispersion, Sec. 2.6 eq:pairwise with the Fermi damping of    */
/* eq:fermi-damping (TS: a = 20, s_R the damping parameter), and its lattice   */
/* sum by the Ewald split of eq:ts-ewald                                       */
/* ------------------------------------------------------------------------- */

/* C6_ij = (3/2) alpha_i alpha_j / (1/omega_i + 1/omega_j) */
static double c6_pair(double ai, double aj, double wi, double wj)
{
    return 1.5 * ai * aj / (1.0 / wi + 1.0 / wj);
}

/* sum over images of f/R^6 for one ordered pair, r = R_j - R_i, with its
 * gradient in r and its derivative in the damping radius R0.  Finite (L ==
 * NULL): the single term n = 0.  Periodic: the Ewald split of the undamped
 * lattice sum of R^-6 (real-space gamma^6 phi_r(gamma R) for 0 < R < rc,
 * reciprocal gamma^3 phi_k(G/gamma) cos(G.r)/Omega for |G| < kc with G = 0
 * included, -gamma^6/6 for i = j) minus the real-space sum of (1-f)/R^6 over
 * every image with (1-f) > DAMP_TAIL. */
static void ts_pair_sum(const lattice_t *L, const double *r, int self, double R0,
                        double a, double *S, double *dS, double *dS0)
{
    *S = 0.0; *dS0 = 0.0;
    dS[0] = dS[1] = dS[2] = 0.0;
    if (!L) {
        double d = norm3(r);
        double f, omf, fd, fR0;
        fermi(d, R0, a, &f, &omf, &fd, &fR0);
        double d6 = d * d * d * d * d * d;
        *S = f / d6;
        double dd = fd / d6 - 6.0 * f / (d6 * d);
        for (int c = 0; c < 3; c++) dS[c] = dd * r[c] / d;
        *dS0 = fR0 / d6;
        return;
    }
    const double g = L->gamma;
    for (int t = 0; t < L->nimg; t++) {
        const int *nn = L->img + 3 * t;
        double x[3];
        for (int c = 0; c < 3; c++)
            x[c] = r[c] + nn[0] * L->A[c] + nn[1] * L->A[3 + c] + nn[2] * L->A[6 + c];
        double d = norm3(x);
        if (d == 0.0) continue;
        if (d < L->rc) {
            /* gamma^6 phi_r(z), phi_r(z) = (z^-6 + z^-4 + z^-2/2) e^{-z^2} */
            double z = g * d, z2 = z * z, ez = exp(-z2);
            double phi = (1.0 / (z2 * z2 * z2) + 1.0 / (z2 * z2) + 0.5 / z2) * ez;
            double dphi = -(6.0 / (z2 * z2 * z2 * z) + 6.0 / (z2 * z2 * z) + 3.0 / (z2 * z) + 1.0 / z) * ez;
            double g6 = g * g * g * g * g * g;
            *S += g6 * phi;
            for (int c = 0; c < 3; c++) dS[c] += g6 * g * dphi * x[c] / d;
        }
        double f, omf, fd, fR0;
        fermi(d, R0, a, &f, &omf, &fd, &fR0);
        if (omf > DAMP_TAIL) {
            double d6 = d * d * d * d * d * d;
            /* -(1-f)/d^6 */
            *S -= omf / d6;
            double dd = fd / d6 + 6.0 * omf / (d6 * d);
            for (int c = 0; c < 3; c++) dS[c] += dd * x[c] / d;
            *dS0 += fR0 / d6;
        }
    }
    for (int t = 0; t < L->nrec; t++) {
        const int *mm = L->rec + 3 * t;
        double G[3];
        for (int c = 0; c < 3; c++) G[c] = mm[0] * L->B[c] + mm[1] * L->B[3 + c] + mm[2] * L->B[6 + c];
        double k = norm3(G);
        if (k >= L->kc) continue;
        /* phi_k(k) = (pi^{3/2}/12)((4 - 2k^2) e^{-k^2/4} + k^3 sqrt(pi) erfc(k/2)), k = G/gamma */
        double kk = k / g;
        double phik = pow(PI, 1.5) / 12.0 *
                      ((4.0 - 2.0 * kk * kk) * exp(-kk * kk / 4.0) + kk * kk * kk * sqrt(PI) * erfc(kk / 2.0));
        double w = g * g * g * phik / L->vol;
        double ph = G[0] * r[0] + G[1] * r[1] + G[2] * r[2];
        *S += w * cos(ph);
        for (int c = 0; c < 3; c++) dS[c] -= w * sin(ph) * G[c];
    }
    if (self) *S -= g * g * g * g * g * g / 6.0;
}

int orc_ts(int N, const double *R, const double *lattice, double gamma,
           double rc, double kc, const double *alpha0, const double *omega,
           const double *rvdw, double sR, double a, double *energy,
           double *grad_R, double *grad_alpha0, double *grad_omega,
           double *grad_rvdw)
{
    if (N < 1) return 1;
    lattice_t Lt, *L = NULL;
    if (lattice) {
        if (det3(lattice) <= 0.0) return 1;
        double maxd;
        pair_extent(N, R, &maxd);
        double dr = damp_range(N, rvdw, sR, a);
        lattice_setup(&Lt, lattice, gamma, rc, kc, rc > dr ? rc : dr, maxd, 0.0);
        L = &Lt;
    }
    double E = 0.0;
#pragma omp parallel for schedule(dynamic) reduction(+:E)
    for (int i = 0; i < N; i++) {
        double Ei = 0.0, gi[3] = {0, 0, 0}, wi = 0.0, vi = 0.0;
        for (int j = 0; j < N; j++) {
            if (j == i && !L) continue;
            double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
            double S, dS[3], dS0;
            ts_pair_sum(L, r, i == j, sR * (rvdw[i] + rvdw[j]), a, &S, dS, &dS0);
            double c6 = c6_pair(alpha0[i], alpha0[j], omega[i], omega[j]);
            /* E = -1/2 sum_ij C6_ij S_ij; each ordered pair's energy is
             * counted at i, and i's gradient gathers both orders */
            Ei += -0.5 * c6 * S;
            for (int c = 0; c < 3; c++) gi[c] += c6 * dS[c];
            wi += -c6 * S * omega[j] / (omega[i] * (omega[i] + omega[j]));
            vi += -sR * c6 * dS0;
        }
        E += Ei;
        if (grad_R) for (int c = 0; c < 3; c++) grad_R[3 * i + c] = gi[c];
        if (grad_alpha0) grad_alpha0[i] = 2.0 * Ei / alpha0[i];
        if (grad_omega) grad_omega[i] = wi;
        if (grad_rvdw) grad_rvdw[i] = vi;
    }
    if (energy) *energy = E;
    if (L) lattice_free(L);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Frequency route terms, Sec. 2.5: eq:log-formula, eq:rpa, eq:gould-norm      */
/* ------------------------------------------------------------------------- */

/* ln(1 + x~) - x~ of eq:gould-norm.  For x < 0, x~ = -erf(y)^{1/4} with
 * y = (sqrt(pi)/2) x^4.  ln erf(y) is taken as ln(erf(y)) for small y and as
 * ln(1 - erfc(y)) for large y, and 1 + x~ = -expm1(ln erf(y) / 4), so both
 * stay accurate when erf(y) is tiny or close to 1. */
static double gould_term(double x)
{
    if (x >= 0.0) return log1p(x) - x;
    double y = sqrt(PI) / 2.0 * x * x * x * x;
    double l = y < 0.5 ? log(erf(y)) : log1p(-erfc(y));   /* ln erf(y) */
    double xt = -exp(0.25 * l);
    double onep = -expm1(0.25 * l);      /* 1 + x~ */
    return log(onep) - xt;
}

int orc_mbd_freq_terms(int N, const double *R, const double *lattice, int nq,
                       const double *q_frac, double gamma, double rc, double kc,
                       const double *alpha0, const double *omega,
                       const double *rvdw, double beta, double a, int nfreq,
                       int norder, double *terms)
{
    if (N < 1 || nfreq < 1 || norder < 1) return 1;
    int periodic = lattice != NULL;
    if (!periodic) nq = 1;
    int n = 3 * N, m = periodic ? 2 * n : n;
    double *x = (double *)malloc(sizeof(double) * nfreq);
    double *wx = (double *)malloc(sizeof(double) * nfreq);
    orc_gauss_legendre(nfreq, x, wx);
    double *au = (double *)malloc(sizeof(double) * N);
    double *one = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; i++) one[i] = 1.0;
    double *K = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *Ki = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *lam = (double *)malloc(sizeof(double) * m);
    double B[9], Ainv[9];
    if (periodic) {
        inv3(lattice, Ainv);
        for (int u = 0; u < 3; u++)
            for (int d = 0; d < 3; d++) B[u * 3 + d] = 2.0 * PI * Ainv[d * 3 + u];
    }
    double Elog = 0.0, Eg = 0.0, xmin = 1e300;
    double *En = (double *)calloc(norder, sizeof(double));
    int rcode = 0;
    for (int f = 0; f < nfreq && !rcode; f++) {
        /* u = 0.6 (1+x)/(1-x) (Sec. 3.3), du = 1.2/(1-x)^2 dx */
        double u = 0.6 * (1.0 + x[f]) / (1.0 - x[f]);
        double du = 1.2 / ((1.0 - x[f]) * (1.0 - x[f])) * wx[f];
        /* eq:dyn-pol */
        for (int i = 0; i < N; i++) au[i] = alpha0[i] / (1.0 + u * u / (omega[i] * omega[i]));
        for (int t = 0; t < nq && !rcode; t++) {
            /* alpha(iu)^{1/2} T^lr alpha(iu)^{1/2}: Q of eq:q-matrix with omega = 1, minus I */
            int sw;
            if (!periodic) {
                orc_assemble_finite(N, R, au, one, rvdw, beta, a, K);
                for (int p = 0; p < n; p++) K[(size_t)p * n + p] -= 1.0;
                sw = orc_jacobi(n, K, lam, NULL);
            } else {
                double q[3];
                for (int d = 0; d < 3; d++)
                    q[d] = q_frac[3 * t] * B[d] + q_frac[3 * t + 1] * B[3 + d] + q_frac[3 * t + 2] * B[6 + d];
                orc_assemble_periodic(N, R, lattice, q, gamma, rc, kc, au, one, rvdw, beta, a, K, Ki);
                for (int p = 0; p < n; p++) K[(size_t)p * n + p] -= 1.0;
                sw = orc_jacobi_hermitian(n, K, Ki, lam, NULL);
            }
            if (sw < 0) { rcode = 3; break; }
            /* every Hermitian eigenvalue appears twice in the real embedding */
            double wgt = du / (2.0 * PI) / nq * (periodic ? 0.5 : 1.0);
            for (int k = 0; k < m; k++) {
                double xk = lam[k];
                if (1.0 + xk < xmin) xmin = 1.0 + xk;
                Elog += wgt * (1.0 + xk > 0.0 ? log1p(xk) : NAN);
                Eg += wgt * gould_term(xk);
                /* eq:rpa: E^(n) = -(1/2pi) int du ((-1)^n / n) Tr (alpha T)^n */
                double pw = 1.0;
                for (int o = 1; o <= norder; o++) {
                    pw *= xk;
                    En[o - 1] += wgt * ((o % 2) ? 1.0 : -1.0) / o * pw;
                }
            }
        }
    }
    terms[0] = Elog;
    terms[1] = Eg;
    terms[2] = xmin;
    for (int o = 0; o < norder; o++) terms[3 + o] = En[o];
    free(x); free(wx); free(au); free(one); free(K); free(Ki); free(lam); free(En);
    return rcode;
}

/* ------------------------------------------------------------------------- */
/* Self-consistent screening (MBD@rsSCS), Sec. 2.3 and 2.7                     */
/* ------------------------------------------------------------------------- */

/* T^GG of eq:tgg for widths sigma_i, sigma_j: with zeta = r/s,
 * s = sqrt(sigma_i^2 + sigma_j^2), Theta = (2 zeta/sqrt(pi)) e^{-zeta^2},
 *   T^GG_ab = (erf(zeta) - Theta) T_ab + 2 zeta^2 Theta r_a r_b / r^5
 * with T the explicit dipole tensor of eq:dipole.  As C1 delta_ab + C2 r_a r_b:
 *   C1 = (erf - Theta)/r^3,  C2 = (2 zeta^2 Theta - 3 (erf - Theta))/r^5,
 * and (d erf/dr = Theta/r, d Theta/dr = Theta (1 - 2 zeta^2)/r)
 *   C1' = (2 zeta^2 Theta - 3 (erf - Theta))/r^4,
 *   C2' = (15 (erf - Theta) - 10 zeta^2 Theta - 4 zeta^4 Theta)/r^6.
 * dT[c][a][b] = d T^GG_ab / d r_c (may be NULL). */
void orc_dipole_gg(const double *r, double s, double *T, double *dT)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double d = sqrt(r2);
    double z = d / s;
    double th = 2.0 * z / sqrt(PI) * exp(-z * z);
    double ef = erf(z);
    double c1 = (ef - th) / (r2 * d);
    double c2 = (2.0 * z * z * th - 3.0 * (ef - th)) / (r2 * r2 * d);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) T[a * 3 + b] = (a == b ? c1 : 0.0) + c2 * r[a] * r[b];
    if (!dT) return;
    double c1p = (2.0 * z * z * th - 3.0 * (ef - th)) / (r2 * r2);
    double c2p = (15.0 * (ef - th) - 10.0 * z * z * th - 4.0 * z * z * z * z * th) / (r2 * r2 * r2);
    for (int c = 0; c < 3; c++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double v = c2p * r[c] / d * r[a] * r[b];
                if (a == b) v += c1p * r[c] / d;
                if (a == c) v += c2 * r[b];
                if (b == c) v += c2 * r[a];
                dT[c * 9 + a * 3 + b] = v;
            }
}

/* eq:mayer */
static double mayer_sigma(double alpha)
{
    return cbrt(sqrt(2.0 / PI) * alpha / 3.0);
}

/* A(u) = diag(1/alpha(iu)) + T^scs, T^scs_ij = (1 - g_ij) T^GG_ij (i != j),
 * g the Fermi damping with a and s_R = beta on the unscaled R_vdW
 * (eq:scs-sr-dipole); row-major n x n */
static void scs_matrix(int N, const double *R, const double *au, const double *rvdw,
                       double beta, double a, double *A)
{
    int n = 3 * N;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            double blk[9] = {0};
            if (i == j) {
                for (int c = 0; c < 3; c++) blk[c * 4] = 1.0 / au[i];
            } else {
                double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
                double s = sqrt(mayer_sigma(au[i]) * mayer_sigma(au[i]) + mayer_sigma(au[j]) * mayer_sigma(au[j]));
                double g, omg, gd, gR0;
                fermi(norm3(r), beta * (rvdw[i] + rvdw[j]), a, &g, &omg, &gd, &gR0);
                double T[9];
                orc_dipole_gg(r, s, T, NULL);
                for (int k = 0; k < 9; k++) blk[k] = omg * T[k];
            }
            for (int p = 0; p < 3; p++)
                for (int q = 0; q < 3; q++) A[(size_t)(3 * i + p) * n + 3 * j + q] = blk[p * 3 + q];
        }
}

/* inverse of a symmetric positive definite matrix (row-major, n x n) by the
 * oracle's Cholesky and triangular solves; returns 2 if not positive definite */
static int spd_inverse(int n, const double *A, double *Ainv)
{
    double *L = (double *)malloc(sizeof(double) * (size_t)n * n);
    memcpy(L, A, sizeof(double) * (size_t)n * n);
    if (cholesky(n, L)) { free(L); return 2; }
#pragma omp parallel for schedule(dynamic)
    for (int col = 0; col < n; col++) {
        double *y = (double *)malloc(sizeof(double) * n);
        for (int p = 0; p < n; p++) {
            double acc = (p == col) ? 1.0 : 0.0;
            for (int k = 0; k < p; k++) acc -= L[(size_t)p * n + k] * y[k];
            y[p] = acc / L[(size_t)p * n + p];
        }
        for (int p = n - 1; p >= 0; p--) {
            double acc = y[p];
            for (int k = p + 1; k < n; k++) acc -= L[(size_t)k * n + p] * y[k];
            y[p] = acc / L[(size_t)p * n + p];
        }
        for (int p = 0; p < n; p++) Ainv[(size_t)p * n + col] = y[p];
        free(y);
    }
    free(L);
    return 0;
}

/* the SCS stage on nfreq Gauss-Legendre points (map of Sec. 3.3) plus u = 0:
 * alpha_bar(u) = (alpha(iu)^{-1} + T^scs)^{-1} (eq:scs), contracted
 * (eq:contraction); C6 by eq:casimir-polder, omega = 4 C6/(3 alpha0^2), R_vdW
 * scaled by (alpha_bar0/alpha0)^{1/3} (eq:scale-rvdw-scs).  abar
 * [(nfreq+1) x N] (row 0: u = 0) and the inverses Abar [(nfreq+1) x n x n]
 * are kept when non-NULL. */
static int scs_stage(int N, const double *R, const double *alpha0, const double *omega,
                     const double *rvdw, double beta, double a, int nfreq,
                     double *a_scs, double *c6_scs, double *w_scs, double *rv_scs,
                     double *abar, double *Abar, double *uw)
{
    int n = 3 * N;
    double *x = (double *)malloc(sizeof(double) * nfreq), *wx = (double *)malloc(sizeof(double) * nfreq);
    orc_gauss_legendre(nfreq, x, wx);
    double *au = (double *)malloc(sizeof(double) * N);
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *Ai = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *ab = (double *)malloc(sizeof(double) * (size_t)(nfreq + 1) * N);
    int rc = 0;
    for (int f = 0; f <= nfreq && !rc; f++) {
        double u = f == 0 ? 0.0 : 0.6 * (1.0 + x[f - 1]) / (1.0 - x[f - 1]);
        if (uw && f > 0) uw[f - 1] = 1.2 / ((1.0 - x[f - 1]) * (1.0 - x[f - 1])) * wx[f - 1];
        for (int i = 0; i < N; i++) au[i] = alpha0[i] / (1.0 + u * u / (omega[i] * omega[i]));
        scs_matrix(N, R, au, rvdw, beta, a, A);
        if (spd_inverse(n, A, Ai)) { rc = 2; break; }
        for (int i = 0; i < N; i++) {
            double s = 0.0;
            for (int j = 0; j < N; j++)
                for (int c = 0; c < 3; c++) s += Ai[(size_t)(3 * i + c) * n + 3 * j + c];
            ab[(size_t)f * N + i] = s / 3.0;
        }
        if (Abar) memcpy(Abar + (size_t)f * n * n, Ai, sizeof(double) * (size_t)n * n);
    }
    if (!rc)
        for (int i = 0; i < N; i++) {
            double c6 = 0.0;
            for (int f = 1; f <= nfreq; f++) {
                double u_w = 1.2 / ((1.0 - x[f - 1]) * (1.0 - x[f - 1])) * wx[f - 1];
                c6 += u_w * ab[(size_t)f * N + i] * ab[(size_t)f * N + i];
            }
            c6 *= 3.0 / PI;
            double a0s = ab[i];
            if (a_scs) a_scs[i] = a0s;
            if (c6_scs) c6_scs[i] = c6;
            if (w_scs) w_scs[i] = 4.0 * c6 / (3.0 * a0s * a0s);
            if (rv_scs) rv_scs[i] = rvdw[i] * cbrt(a0s / alpha0[i]);
        }
    if (abar) memcpy(abar, ab, sizeof(double) * (size_t)(nfreq + 1) * N);
    free(x); free(wx); free(au); free(A); free(Ai); free(ab);
    return rc;
}

int orc_scs(int N, const double *R, const double *alpha0, const double *omega,
            const double *rvdw, double beta, double a, int nfreq,
            double *alpha_scs, double *c6_scs, double *omega_scs, double *rvdw_scs,
            double *alpha_dyn)
{
    if (N < 1 || nfreq < 1) return 1;
    return scs_stage(N, R, alpha0, omega, rvdw, beta, a, nfreq, alpha_scs, c6_scs, omega_scs,
                     rvdw_scs, alpha_dyn, NULL, NULL);
}

/* MBD@rsSCS: the SCS stage, then the MBD energy of Sec. 2.1 with the screened
 * alpha0, omega and R_vdW (T^lr = g T with the scaled radii, eq:mbd-lr-dipole).
 * dE/dR by the chain rule through the screened parameters: for every
 * coordinate R_mc, d alpha_bar(u)/dR_mc = -alpha_bar (dT^scs/dR_mc) alpha_bar
 * (the derivative of eq:scs), contracted as in eq:contraction, at u = 0 and
 * at every frequency point. */
int orc_mbd_rsscs(int N, const double *R, const double *alpha0, const double *omega,
                  const double *rvdw, double beta, double a, int nfreq,
                  double *energy, double *grad_R, double *alpha_scs, double *omega_scs,
                  double *rvdw_scs)
{
    if (N < 1 || nfreq < 1) return 1;
    int n = 3 * N, nf1 = nfreq + 1;
    double *as = (double *)malloc(sizeof(double) * N), *ws = (double *)malloc(sizeof(double) * N);
    double *rs = (double *)malloc(sizeof(double) * N), *c6 = (double *)malloc(sizeof(double) * N);
    double *ab = (double *)malloc(sizeof(double) * (size_t)nf1 * N);
    double *uw = (double *)malloc(sizeof(double) * nfreq);
    double *Ab = grad_R ? (double *)malloc(sizeof(double) * (size_t)nf1 * n * n) : NULL;
    int rc = scs_stage(N, R, alpha0, omega, rvdw, beta, a, nfreq, as, c6, ws, rs, ab, Ab, uw);
    double *gR = (double *)calloc((size_t)3 * N, sizeof(double));
    double *ga = (double *)calloc(N, sizeof(double)), *gw = (double *)calloc(N, sizeof(double));
    double *gv = (double *)calloc(N, sizeof(double));
    if (!rc) rc = orc_mbd_finite(N, R, as, ws, rs, beta, a, energy, grad_R ? gR : NULL,
                                 grad_R ? ga : NULL, grad_R ? gw : NULL, grad_R ? gv : NULL, NULL);
    if (!rc && grad_R) {
        /* weights of d alpha_bar_i(u)/dX in dE/dX: u = 0 (alpha0, and through
         * omega and R_vdW), u_f (through C6 and omega) */
        double *w = (double *)malloc(sizeof(double) * (size_t)nf1 * N);
        for (int i = 0; i < N; i++) {
            w[i] = ga[i] - 2.0 * ws[i] / as[i] * gw[i] + gv[i] * rs[i] / (3.0 * as[i]);
            for (int f = 1; f <= nfreq; f++)
                w[(size_t)f * N + i] = gw[i] * 4.0 / (3.0 * as[i] * as[i]) * (3.0 / PI) * uw[f - 1] * 2.0 *
                                       ab[(size_t)f * N + i];
        }
        double *x = (double *)malloc(sizeof(double) * nfreq), *wx = (double *)malloc(sizeof(double) * nfreq);
        orc_gauss_legendre(nfreq, x, wx);
        double *au = (double *)malloc(sizeof(double) * N);
        double *D = (double *)malloc(sizeof(double) * (size_t)N * 9);   /* dA block (m, l) per l */
        double *cs = (double *)malloc(sizeof(double) * (size_t)n * 3);  /* sum_j Abar_{k, ja} */
        double *Z = (double *)malloc(sizeof(double) * (size_t)n * 3);
        for (int f = 0; f <= nfreq; f++) {
            double u = f == 0 ? 0.0 : 0.6 * (1.0 + x[f - 1]) / (1.0 - x[f - 1]);
            for (int i = 0; i < N; i++) au[i] = alpha0[i] / (1.0 + u * u / (omega[i] * omega[i]));
            const double *Ai = Ab + (size_t)f * n * n;
            for (int k = 0; k < n; k++)
                for (int aa = 0; aa < 3; aa++) {
                    double t = 0.0;
                    for (int j = 0; j < N; j++) t += Ai[(size_t)k * n + 3 * j + aa];
                    cs[3 * k + aa] = t;
                }
            for (int m = 0; m < N; m++)
                for (int c = 0; c < 3; c++) {
                    /* dA/dR_mc is nonzero in blocks (m, l) = D_l and (l, m) = D_l^T,
                     * with D_l = d/dR_mc (1 - g) T^GG (R_l - R_m) = -d/dr_c of it */
                    for (int l = 0; l < N; l++) {
                        double *Dl = D + 9 * l;
                        memset(Dl, 0, 9 * sizeof(double));
                        if (l == m) continue;
                        double r[3] = {R[3 * l] - R[3 * m], R[3 * l + 1] - R[3 * m + 1], R[3 * l + 2] - R[3 * m + 2]};
                        double d = norm3(r);
                        double sm = mayer_sigma(au[m]), sl = mayer_sigma(au[l]);
                        double T[9], dT[27], g, omg, gd, gR0;
                        orc_dipole_gg(r, sqrt(sm * sm + sl * sl), T, dT);
                        fermi(d, beta * (rvdw[m] + rvdw[l]), a, &g, &omg, &gd, &gR0);
                        for (int k = 0; k < 9; k++) Dl[k] = -(-gd * r[c] / d * T[k] + omg * dT[c * 9 + k]);
                    }
                    /* (Abar dA Abar)_{ia,ja} summed over j: sum_k Abar_{ia,k} (dA cs)_{k,a};
                     * (dA cs) has rows of block m: Y[p] = sum_l D_l[p][q] cs_{lq}, and rows
                     * (l, q): Z = sum_p D_l[p][q] cs_{mp} */
                    double Y[9] = {0};
                    for (int l = 0; l < N; l++)
                        for (int pp = 0; pp < 3; pp++)
                            for (int q = 0; q < 3; q++)
                                for (int aa = 0; aa < 3; aa++)
                                    Y[pp * 3 + aa] += D[9 * l + pp * 3 + q] * cs[3 * (3 * l + q) + aa];
                    for (int l = 0; l < N; l++)
                        for (int q = 0; q < 3; q++)
                            for (int aa = 0; aa < 3; aa++) {
                                double t = 0.0;
                                for (int pp = 0; pp < 3; pp++) t += D[9 * l + pp * 3 + q] * cs[3 * (3 * m + pp) + aa];
                                Z[3 * (3 * l + q) + aa] = t;
                            }
                    double acc = 0.0;
                    for (int i = 0; i < N; i++) {
                        double wi = w[(size_t)f * N + i];
                        if (wi == 0.0) continue;
                        for (int aa = 0; aa < 3; aa++) {
                            const double *ar = Ai + (size_t)(3 * i + aa) * n;
                            double sacc = 0.0;
                            for (int pp = 0; pp < 3; pp++) sacc += ar[3 * m + pp] * Y[pp * 3 + aa];
                            for (int k = 0; k < n; k++) sacc += ar[k] * Z[3 * k + aa];
                            acc += wi * (-sacc / 3.0);
                        }
                    }
                    gR[3 * m + c] += acc;
                }
        }
        free(x); free(wx); free(au); free(D); free(cs); free(Z); free(w);
    }
    if (grad_R && !rc) memcpy(grad_R, gR, sizeof(double) * 3 * N);
    if (alpha_scs && !rc) memcpy(alpha_scs, as, sizeof(double) * N);
    if (omega_scs && !rc) memcpy(omega_scs, ws, sizeof(double) * N);
    if (rvdw_scs && !rc) memcpy(rvdw_scs, rs, sizeof(double) * N);
    if (rc && energy) *energy = NAN;
    free(as); free(ws); free(rs); free(c6); free(ab); free(uw); free(Ab);
    free(gR); free(ga); free(gw); free(gv);
    return rc;
}
