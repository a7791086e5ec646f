/*
 * mbd_oracle.h -- plain FP64 CPU oracle for the MBD energy and its gradients.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may call into this library.  It shares no code
 * with the HIP path (paper_2308_03140_amd/) and never imports it.
 *
 * Everything is in Hartree atomic units (bohr, Ha).  Arrays are row-major.
 * The paper is Hermann et al., "libMBD: A general-purpose package for scalable
 * quantum many-body dispersion calculations" (arXiv:2308.03140); citations
 * name its sections and equation labels.
 *
 * Return codes: 0 ok, 1 invalid argument, 2 negative eigenvalue of Q
 * (dipole collapse, Sec. 2.1 after eq:mbd-energy), 3 Jacobi not converged.
 */
#ifndef MBD_ORACLE_H
#define MBD_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

/* Q of eq:q-matrix for a finite system, T^lr = g T (eq:mbd-lr-dipole with the
 * bare tensor of eq:dipole, Fermi damping eq:fermi-damping with s_R = beta).
 * beta == 0 means no damping (g == 1).  Q is n x n, n = 3N, row-major,
 * index p = 3*i + a. */
void orc_assemble_finite(int N, const double *R, const double *alpha0,
                         const double *omega, const double *rvdw,
                         double beta, double a, double *Q);

/* Cyclic Jacobi for a real symmetric n x n matrix (row-major, destroyed).
 * w: eigenvalues ascending; V (may be NULL): V[i*n + k] = component i of
 * eigenvector k.  Returns number of sweeps used, or -1 if not converged. */
int orc_jacobi(int n, double *A, double *w, double *V);

/* Hermitian eigenvalues (and optionally eigenvectors) via the real embedding
 * [[Re, -Im], [Im, Re]] of size 2n; w gets the 2n embedded eigenvalues
 * (each Hermitian eigenvalue twice), V the 2n x 2n embedded eigenvectors. */
int orc_jacobi_hermitian(int n, const double *Are, const double *Aim,
                         double *w, double *V);

/* Finite MBD: energy eq:mbd-energy, gradients as (1/4) Re Tr(Q^{-1/2} dQ)
 * (eq:mbd-gradient read with the full derivative of Q).  Any output pointer
 * may be NULL.  eigs: 3N eigenvalues of Q ascending. */
int orc_mbd_finite(int N, const double *R, const double *alpha0,
                   const double *omega, const double *rvdw, double beta,
                   double a, double *energy, double *grad_R,
                   double *grad_alpha0, double *grad_omega, double *grad_rvdw,
                   double *eigs);

/* Ewald defaults of Sec. 3.3: gamma = 2.5/Omega^(1/3), Rc = 6/gamma,
 * kc = 10 gamma.  lattice rows are the lattice vectors (bohr). */
void orc_ewald_defaults(const double *lattice, double *gamma, double *rc,
                        double *kc);

/* Periodic Q(q) of eq:q-matrix with T^lr(q) the Bloch sum of g T evaluated
 * with the Ewald split of eq:ewald/eq:terfc plus the damping correction
 * -(1-g) T summed in real space.  q is Cartesian (1/bohr).  Qre/Qim n x n. */
int orc_assemble_periodic(int N, const double *R, const double *lattice,
                          const double *q, double gamma, double rc, double kc,
                          const double *alpha0, const double *omega,
                          const double *rvdw, double beta, double a,
                          double *Qre, double *Qim);

/* Periodic MBD per unit cell: E = mean over the q list of E(q)
 * (eq:brillouin-int).  q_frac [nq][3] fractional in the reciprocal basis.
 * Gradients (each may be NULL) are q-averages of (1/4) Re Tr(M(q) dQ(q)),
 * M = Q^{-1/2}, minus (3/2) d(sum omega): dE/dR [N][3], dE/dalpha0,
 * dE/domega and dE/dRv [N] (through the damping correction), and
 * grad_lattice [3][3] = dE/dA_{vc} with Cartesian positions, fractional q,
 * gamma and the term sets fixed.  eigs: nq x 3N Hermitian eigenvalues. */
int orc_mbd_periodic(int N, const double *R, const double *lattice, int nq,
                     const double *q_frac, double gamma, double rc, double kc,
                     const double *alpha0, const double *omega,
                     const double *rvdw, double beta, double a,
                     double *energy, double *grad_R, double *grad_alpha0,
                     double *grad_omega, double *grad_rvdw,
                     double *grad_lattice, double *eigs);

/* Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n). */
void orc_gauss_legendre(int n, double *x, double *w);

/* Finite MBD energy by the imaginary-frequency route eq:log-formula, with the
 * Hermitian form alpha^{1/2} T alpha^{1/2}, eq:dyn-pol and the grid map
 * u = 0.6 (1+x)/(1-x) of Sec. 3.3; ln det by the oracle's own Cholesky.
 * Optionally (nsample > 0) the gradients dE/dR [nsample][3], dE/dalpha0 and
 * dE/domega [nsample] of the listed atoms from the rows of
 * Q^{-1/2} = (2/pi) int_0^inf (Q + u^2)^{-1} du, reusing the same factors
 * (each gradient output may be NULL).
 * Returns 2 if a Cholesky factorisation fails (collapse). */
int orc_mbd_finite_freq(int N, const double *R, const double *alpha0,
                        const double *omega, const double *rvdw, double beta,
                        double a, int npts, double *energy, int nsample,
                        const int *atoms, double *grad_R_sample,
                        double *grad_alpha0_sample, double *grad_omega_sample);

/* Pairwise (TS) energy of Sec. 2.6 eq:pairwise, E = -1/2 sum_{i != j}
 * C6_ij f(R_ij)/R_ij^6 with C6_ij = (3/2) alpha_i alpha_j/(1/omega_i +
 * 1/omega_j) and f the Fermi damping of eq:fermi-damping (steepness a, s_R =
 * sR; TS uses a = 20).  lattice == NULL: finite system.  Otherwise the energy
 * per cell, sum over all images (n = 0, i = j excluded), by the Ewald split of
 * eq:ts-ewald for the undamped R^-6 sum (read with the G = 0 term included,
 * the self term -gamma^6/6 and cos(G.R_ij)) minus the real-space sum of
 * (1-f)/R^6.  Gradients (each may be NULL): dE/dR [N][3], dE/dalpha0,
 * dE/domega, dE/dRv [N]. */
int orc_ts(int N, const double *R, const double *lattice, double gamma,
           double rc, double kc, const double *alpha0, const double *omega,
           const double *rvdw, double sR, double a, double *energy,
           double *grad_R, double *grad_alpha0, double *grad_omega,
           double *grad_rvdw);

/* Frequency route of Sec. 2.5 with the eigenvalues x_k of
 * K(u) = alpha(iu)^{1/2} T^lr alpha(iu)^{1/2} (eq:dyn-pol; periodic: K(u, q)
 * on the q list, averaged): nfreq Gauss-Legendre points on the map of
 * Sec. 3.3, the oracle's Jacobi for the x_k.  terms [3 + norder]:
 *   [0] E = (1/2pi) int du sum_k ln(1 + x_k)      (eq:log-formula; NaN if
 *                                                   some 1 + x_k <= 0)
 *   [1] (1/2pi) int du sum_k (ln(1 + x~_k) - x~_k) (eq:gould-norm)
 *   [2] min over u, q, k of 1 + x_k
 *   [3 + n - 1] E^(n) = -(1/2pi) int du ((-1)^n/n) sum_k x_k^n, n = 1..norder
 *               (eq:rpa; E^(1) vanishes for finite systems)
 * lattice == NULL: finite (nq, q_frac, gamma, rc, kc unused). */
int orc_mbd_freq_terms(int N, const double *R, const double *lattice, int nq,
                       const double *q_frac, double gamma, double rc, double kc,
                       const double *alpha0, const double *omega,
                       const double *rvdw, double beta, double a, int nfreq,
                       int norder, double *terms);

/* Gaussian-smeared dipole tensor T^GG of eq:tgg (explicit-T sign convention)
 * for r and s = sqrt(sigma_i^2 + sigma_j^2); dT[c][a][b] = d/dr_c (may be NULL). */
void orc_dipole_gg(const double *r, double s, double *T, double *dT);

/* Self-consistent screening of Sec. 2.3 (finite systems): at u = 0 and at
 * nfreq Gauss-Legendre points (map of Sec. 3.3), alpha_bar(u) = (alpha(iu)^-1
 * + T^scs)^-1 (eq:scs, eq:dyn-pol), T^scs = (1 - g) T^GG with Mayer widths
 * (eq:scs-sr-dipole, eq:tgg, eq:mayer; g with steepness a and s_R = beta on
 * the unscaled R_vdW), contracted per atom (eq:contraction).  Outputs [N]
 * (each may be NULL): alpha_scs = alpha_bar(0), c6_scs by eq:casimir-polder,
 * omega_scs = 4 C6/(3 alpha_scs^2), rvdw_scs = R_vdW (alpha_scs/alpha0)^{1/3}
 * (eq:scale-rvdw-scs); alpha_dyn [(nfreq+1) x N], row 0 at u = 0.
 * Returns 2 if some alpha(iu)^-1 + T^scs is not positive definite. */
int orc_scs(int N, const double *R, const double *alpha0, const double *omega,
            const double *rvdw, double beta, double a, int nfreq,
            double *alpha_scs, double *c6_scs, double *omega_scs, double *rvdw_scs,
            double *alpha_dyn);

/* MBD@rsSCS energy (SCS stage, then the MBD energy with the screened alpha0,
 * omega, R_vdW and T^lr = g T) and dE/dR [N][3] through the chain rule of the
 * screened parameters (may be NULL); screened parameters out (may be NULL). */
int orc_mbd_rsscs(int N, const double *R, const double *alpha0, const double *omega,
                  const double *rvdw, double beta, double a, int nfreq,
                  double *energy, double *grad_R, double *alpha_scs, double *omega_scs,
                  double *rvdw_scs);

/* Smallest eigenvalue of alpha0^{1/2} T^lr alpha0^{1/2} (finite). */
int orc_min_coupling_eig(int N, const double *R, const double *alpha0,
                         const double *rvdw, double beta, double a,
                         double *mu_min);

/* 1 if the symmetric matrix (row-major) has a Cholesky factor, else 0. */
int orc_is_positive_definite(int n, const double *A);

/* Pairwise tensors for tests: bare T (eq:dipole), T^erfc (eq:terfc, with the
 * coefficient reading -r_a r_b C), and their first derivatives dT[c][a][b]. */
void orc_dipole(const double *r, double *T, double *dT);
void orc_dipole_erfc(const double *r, double gamma, double *T, double *dT);

#ifdef __cplusplus
}
#endif
#endif
