// Per-system device descriptor and MBD stage launchers (internal).
#pragma once
#include "mbd_internal.h"

struct SysDesc {
    const double* coords;
    const double* alpha0;
    const double* omega_or_c6;
    const double* rvdw;
    int N;
    int param_kind;          // 0 omega, 1 C6
    double beta, a;
    int mat0, nmat;          // matrices of this system in the batch (periodic: one per q)
    double weight;           // energy weight per sqrt(lambda) (1/2, or 1/(4 n_q) for embedded)
    int embed;               // 1: matrices are 2n real embeddings of Hermitian Q(q)
    int atom_off;            // offset of this system in the per-atom workspaces
    double* energy;
    double* grad_coords;
    double* grad_alpha0;
    double* grad_omega;
    double* grad_rvdw;
    double* grad_lattice;
    double* eigvals;
    double* errors;
    // periodic data
    double lat[9], linv[9], recip[9];
    double vol, gamma, rc, kc, rdamp;
};

void mbd_prep_launch(hipStream_t st, const SysDesc* sd, int nsys, int Nmax, double* om, double* cc,
                     unsigned* status);
void mbd_assemble_finite_launch(hipStream_t st, const SysDesc* sd, int nsys, int Nmax, const double* om,
                                const double* cc, MatBatch<double> Q, MatBatch<float> Q32, unsigned* status);
// mmult (may be null: all 1): weight of each matrix's eigenvalue sum, a
// multiple of the system's weight
void mbd_energy_launch(hipStream_t st, const SysDesc* sd, int nsys, const int* ns, const double* lam,
                       long long sL, const double* om, unsigned* status, double* lmin, const int* conv,
                       const double* mmult = nullptr);
void mbd_errors_launch(hipStream_t st, const SysDesc* sd, int nsys, int nmat, const double* stats, const int* one);
void mbd_invsqrt4_launch(hipStream_t st, const int* ns, int nmax, int nbatch, const double* lam, long long sL,
                         double* sc);
// lower triangle of M = X diag(sc)^2 X^T; the columns of X are scaled in place
void mbd_inv_sqrt_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> X,
                         const double* sc, long long sL, MatBatch<double> M);
void mbd_mirror_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> M,
                       const int* skip = nullptr);
void mbd_grad_finite_launch(hipStream_t st, const SysDesc* sd, int nsys, int Nmax, const double* om,
                            const double* cc, MatBatch<double> M);

// Ogita-Aishima refinement (one step per call; see k_refine.hip)
#define OA_KMAX 32  // largest window of close eigenvalues solved by Rayleigh-Ritz
// Default remainder threshold of the first refinement step (rho_next
// overrides when > 0) and the factor by which the second step must end below
// the threshold in force.  After a second step rho no longer overstates the
// error the column rescaling leaves: the dE/domega error measured about 1.2
// rho (order 24000: rho 1.2e-6, error 0.6-1.0e-6; a wide band of identical
// weakly coupled atoms: rho 2.2e-6, error 2.7e-6), so 1.5e-6 keeps it within
// 2e-6 and dE/dR three orders below that.
#define OA_RHO_NEXT 3e-5
#define OA_RHO_FINAL_DIV 20.0
struct OaWork {
    double* colpart;  // [nbatch][nmax][6] per-column partial sums
    unsigned* nclust; // [nbatch] runs of linked columns the last step cut into windows
    int* wstart;      // [nbatch][nmax] first column of each column's window
    int* wlen;        // [nbatch][nmax] window length
    double* wv;       // [nbatch][nmax][OA_KMAX] window rotation, per column
    double* gdiag;    // [nbatch][nmax] diagonal of X^T X
    int* fexp;        // [nbatch][nmax] power-of-two scale of each F_small column (first step)
    double rho_next;  // threshold on the step's remainder estimate (<= 0: default OA_RHO_NEXT)
};
size_t oa_colpart_doubles(int nmax, int nbatch);
void oa_f2d_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<float> X32, MatBatch<double> Xd);
// X (in) -> T1 (out, refined); T2 and G are scratch; stats[4b..4b+3] =
// {delta, max|I - X^T X|, rho, max|X|}; next[b] = 1 where no further step is
// needed; matrices with skip[b] != 0 get T1 = X and keep lam.  X32.p != nullptr
// states that X holds exactly the FP32 matrix X32, whose products the update
// then runs on the FP16 matrix cores (split operands)
void oa_step_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> Q, MatBatch<double> X,
                    MatBatch<double> T1, MatBatch<double> T2, MatBatch<double> G, double* lam, long long sL,
                    const OaWork& w, double* stats, const int* skip, int* next, MatBatch<float> X32);
void copy_mat_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> src,
                     MatBatch<double> dst);
void fill_u32_launch(hipStream_t st, unsigned* p, int n, unsigned v);
template <typename T>
void fill_sym_random_launch(hipStream_t st, int n, T* A, int ld, unsigned seed);

// periodic (Ewald) assembly and adjoint; the adjoint keeps PER_PART doubles
// per (q, i, j): {P, dR[3], dA[9], P0} of the real-space and self terms
#define PER_PART 14
// Work of the Ewald sums.  Reciprocal-space term as a product of the basis
// U(q) (one column per reciprocal vector G with 0 < |G + q| < kc, embedded
// [Re; Im], 2n x ncol per q, ld ldz, stride sZ; columns past a q point's
// count are zero) with itself (assembly) or with M(q) C (adjoint, into W,
// same layout); real-space phases e^{-i q.R_n} per image n and q.
struct PerEwald {
    const int* rec;    // reciprocal lattice vectors, integer triplets
    const int* col;    // [nq][ncol]: index into rec of each column, -1 past the q point's count
    int ncol;          // columns per q point (the largest count)
    double* Z;         // basis U(q)
    double* W;         // M C U (adjoint only)
    int ldz;
    long long sZ;
    double* phase;     // [nimg][nq] (cos, sin) of -q.R_n
};
// U(q) for every q and the real-space phase table (before the assembly; the
// adjoint reuses both)
void per_recip_basis_launch(hipStream_t st, const SysDesc* sd, const double* qcart, int nq, const int* img,
                            int nimg, const PerEwald& pr);
// Writes the whole embedded Q(q) (and its FP32 copy when Q32.p is set); with
// cc and om null, the lattice sum T(q) itself (c = 1, no omega^2 diagonal)
void mbd_assemble_periodic_launch(hipStream_t st, const SysDesc* sd, const double* om, const double* cc,
                                  const double* qcart, int nq, const int* img, int nimg, const PerEwald& pr,
                                  MatBatch<double> Q, MatBatch<float> Q32, unsigned* status, int N);
// column chunks of the reciprocal adjoint: rq holds 4 N doubles and rl 10 per
// (q, chunk); latpart 9 N doubles
int per_recip_chunks(int ncol);
// qmult[q]: weight of q point q (2 where it stands for its time-reversed
// partner); wq: the Brillouin-zone weight 1/4 per mesh point of all of them
void mbd_grad_periodic_launch(hipStream_t st, const SysDesc* sd, const double* om, const double* cc,
                              const double* qcart, const double* qmult, double wq, int nq, const int* img,
                              int nimg, const PerEwald& pr, MatBatch<double> M, double* partial, double* rq,
                              double* rl, double* latpart, int N);

// pairwise (TS) dispersion: per-atom energy shares into eatom, gradients into
// the descriptor's outputs, then the energy (and errors[0..3] = 0); with
// launch profiling on, the pair kernel is timed as kind 11
struct LaunchProfiler;
void mbd_ts_launch(hipStream_t st, const SysDesc* sd, int N, const double* om, const int* img, int nimg,
                   const int* rec, int nrec, int periodic, double* eatom, unsigned* status,
                   LaunchProfiler* prof = nullptr);

// frequency route: per-frequency coefficients (descriptor 0 = the system,
// 1..nfreq = one per frequency), then the per-matrix eigenvalue sums and the
// weighted terms {E, E_Gould, min(1+x), E^(1..norder)}
void mbd_freq_coeff_launch(hipStream_t st, const SysDesc* sd, const double* om0, const double* u, int nfreq, int N,
                           double* om_f, double* cc_f);
// periodic K(u_f, q) = C_f T(q) C_f for every frequency f and q (T: the
// embedded lattice sums, as the periodic assembly writes them without c, omega)
void mbd_freq_scale_launch(hipStream_t st, const double* cc_f, int N, int nfreq, int nq, MatBatch<double> T,
                           MatBatch<double> K);
void mbd_freq_terms_launch(hipStream_t st, const int* ns, int nmat, const double* lam, long long sL, int norder,
                           double* part, const double* wf, int nfreq, int nq, int embed, double* terms);

// self-consistent screening (see k_scs.hip)
void scs_assemble_launch(hipStream_t st, const SysDesc* sd, int N, const double* om, const double* u, int nf,
                         MatBatch<double> A, unsigned* status);
void scs_rhs_launch(hipStream_t st, int N, int nf, const double* w, double* R);
void scs_contract_launch(hipStream_t st, int N, int nf, const double* V, double* abar);
void scs_params_launch(hipStream_t st, const SysDesc* sd, int N, const double* abar, const double* wq, int nf,
                       double* out);
void scs_weights_launch(hipStream_t st, int N, int nf, const double* par, const double* abar, const double* wq,
                        const double* ga, const double* gw, const double* gv, double* w);
void scs_grad_launch(hipStream_t st, const SysDesc* sd, int N, int nf, const double* om, const double* u,
                     const double* U, const double* V, double* UV, double* grad);
// batched Cholesky (k_chol.hip): factor in place (lower), diagonal-block
// inverses in Linv (chol_linv_stride(n) per matrix); solves with three
// right-hand sides, layout [nbatch][n][3] with per-matrix stride sR
long long chol_linv_stride(int n);
void chol_factor_launch(hipStream_t st, MatBatch<double> A, int n, int nbatch, double* Linv, unsigned* status);
void chol_solve_launch(hipStream_t st, MatBatch<double> A, int n, int nbatch, const double* Linv, double* R, double* Y,
                       double* X, long long sR);
