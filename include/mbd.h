/*
 * mbd.h -- C ABI of libmbd_hip.so: many-body dispersion (MBD) energy and
 * analytic gradients on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Hermann et al., "libMBD: A general-purpose package
 * for scalable quantum many-body dispersion calculations" (arXiv:2308.03140):
 *
 *   Q_ij = delta_ij omega_i^2 I + omega_i omega_j sqrt(alpha0_i alpha0_j) T^lr_ij
 *                                                        (Sec. 2.1, eq:q-matrix)
 *   Q = C Lambda C^T                                     (eq:diagonalization)
 *   E = sum_k sqrt(lambda_k)/2 - 3 sum_i omega_i/2        (eq:mbd-energy)
 *   T^lr = g T, g the Fermi function with a and beta     (Sec. 2.7,
 *                                eq:mbd-lr-dipole, eq:fermi-damping, a = 6)
 *   periodic: E = mean over the q mesh of E(q), T^lr(q) by Ewald summation
 *                                (Sec. 2.2, eq:brillouin-int, eq:ewald, eq:terfc;
 *                                 defaults of Sec. 3.3)
 *   gradients: dE/dX = (1/4) Re Tr(Q^{-1/2} dQ/dX) - (3/2) d(sum omega)/dX
 *                                (Sec. 2.4, eq:mbd-gradient)
 *
 * Conventions
 *   - Hartree atomic units: lengths in bohr, energies in Ha, alpha0 in bohr^3,
 *     omega in Ha, C6 in Ha bohr^6.
 *   - Every array argument is FP64, contiguous, and a DEVICE pointer on the
 *     context's device, unless marked (host).  Coordinates are [N][3]
 *     row-major; the lattice is [3][3] with row v = lattice vector v.
 *   - Ownership: the caller owns all input and output buffers.  The library
 *     never frees them and does not keep them past the call.  The context owns
 *     its device workspaces (grown to the largest problem seen, reused).
 *   - Streams: all device work is enqueued on the context's stream.  A call
 *     returns after one synchronisation of that stream (it reads one status
 *     word back).  A context is not thread-safe; use one per host thread.
 *   - Errors: every call returns an mbd_status; no exceptions cross the ABI
 *     and the library never exits.  mbd_last_error() gives (code, origin,
 *     message) of the last failure on the context, like get_exception of the
 *     paper's Fortran API (Sec. 3.1).  On any error the outputs are undefined
 *     except where stated.
 */
#ifndef MBD_H
#define MBD_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbd_ctx mbd_ctx;

typedef enum {
    MBD_OK = 0,
    MBD_ERR_INVALID_ARGUMENT = 1,   /* bad pointer, size, flag or input value */
    MBD_ERR_NEGATIVE_EIGENVALUE = 2,/* Q not positive definite: the "dipole
                                       collapse" of Sec. 2.1 (complex energy) */
    MBD_ERR_NOT_CONVERGED = 3,      /* MBD_FP32_REFINED: the FP64 refinement
                                       missed its target and the FP64 fallback
                                       is disabled (env MBD_REFINE_FALLBACK=0) */
    MBD_ERR_OUT_OF_MEMORY = 4,      /* device allocation failed or exceeded
                                       MBD_WORKSPACE_LIMIT (bytes, env var)   */
    MBD_ERR_DEVICE = 5,             /* HIP runtime error                      */
    MBD_ERR_UNSUPPORTED = 6         /* valid request this build does not do  */
} mbd_status;

/* Arithmetic of the diagonalisation.  MBD_FP64: everything in FP64.
 * MBD_FP32_REFINED: Householder reduction, tridiagonal solve and
 * back-transform in FP32 on matrix cores with FP32 accumulation, then one
 * Ogita-Aishima refinement step of the eigenpairs in FP64 against the FP64 Q
 * (a second one where the first leaves a large remainder estimate or cuts a
 * run of linked near-degenerate columns into windows, which must end 20
 * times below the threshold); the sqrt(lambda)
 * energy sum, the gradients and the Ewald sums stay FP64.  A system whose
 * refinement still misses its target after the second step is re-evaluated
 * on the MBD_FP64 path (then errors[2] = 0), or, with the environment
 * variable MBD_REFINE_FALLBACK=0 at mbd_create, reported as
 * MBD_ERR_NOT_CONVERGED.  MBD_REFINE_TOL (at mbd_create) overrides the
 * remainder threshold, default 3e-5. */
typedef enum { MBD_FP64 = 0, MBD_FP32_REFINED = 1 } mbd_precision;

/* Environment variables read by the library (once per process unless noted):
 *   MBD_REFINE_TOL, MBD_REFINE_FALLBACK   see mbd_precision (at mbd_create)
 *   MBD_WORKSPACE_LIMIT    cap on a context's device workspace, bytes (at
 *                          mbd_create)
 *   MBD_NO_GRAPH=1         mbd_evaluate_batch runs eagerly instead of
 *                          replaying a captured graph (read per call)
 *   MBD_Q_PAIRS=1          periodic evaluations fold time-reversed q points
 *                          (see mbd_system.n_q; read per call)
 *   MBD_SYTRD_FUSED_MAXN   largest trailing order reduced by one fused launch
 *                          per column (default 4000 in FP32, 0 in FP64)
 *   MBD_SYTRD_WG_MIN_BATCH smallest batch of matrices of order <= 1024 that
 *                          is reduced with one workgroup per matrix (default
 *                          256 in FP64; FP32 only when set; 0: never)
 * The last two choose between reduction paths of equal results (to
 * rounding); they exist for measurement and tests. */

/* Second oscillator parameter: omega (Ha) or C6 (Ha bohr^6), related by
 * 4 C6 = 3 omega alpha0^2 (Sec. 2.1, eq:osc-param). */
typedef enum { MBD_PARAM_OMEGA = 0, MBD_PARAM_C6 = 1 } mbd_param_kind;

enum {
    MBD_WANT_ENERGY = 1,
    MBD_WANT_GRAD_COORDS = 2,
    MBD_WANT_GRAD_ALPHA0 = 4,
    MBD_WANT_GRAD_OMEGA = 8,       /* gradient w.r.t. omega or C6 (param_kind) */
    MBD_WANT_GRAD_RVDW = 16,       /* through the damping radius beta(Rv_i+Rv_j) */
    MBD_WANT_GRAD_LATTICE = 32,    /* periodic systems only                    */
    MBD_WANT_EIGVALS = 64,
    MBD_WANT_ERRORS = 128
};

typedef struct {
    int32_t n_atoms;              /* N >= 1                                      */
    const double *coords;         /* [N][3] bohr                                 */
    const double *lattice;        /* [3][3] bohr, rows = lattice vectors, or NULL
                                     for a finite system (HOST pointer)          */
    int32_t n_q;                  /* periodic: number of q points in q_frac, or 0
                                     to use the Monkhorst-Pack mesh kgrid/kshift.
                                     Every point is evaluated (at most 65535,
                                     else MBD_ERR_UNSUPPORTED).  Points q, q'
                                     with q + q' an integer vector (time-
                                     reversed partners) give the same energy and
                                     gradient contributions: with MBD_Q_PAIRS=1
                                     (and no eigenvalue output) one of each
                                     pair is evaluated, with weight 2 */
    const double *q_frac;         /* [n_q][3] fractional coordinates in the
                                     reciprocal basis (HOST pointer)             */
    int32_t kgrid[3];             /* periodic mesh size when n_q == 0 (each >= 1) */
    double kshift[3];             /* added to the Monkhorst-Pack fractions
                                     (2r - n - 1)/(2n), r = 1..n                 */
    const double *alpha0;         /* [N] static polarisabilities, > 0           */
    const double *omega_or_c6;    /* [N] omega (Ha) or C6, > 0                  */
    mbd_param_kind param_kind;
    const double *rvdw;           /* [N] vdW radii, > 0                          */
    double beta;                  /* damping s_R >= 0 (0: undamped, g == 1)      */
    double a;                     /* damping steepness > 0 (MBD: 6)              */
    double ewald_gamma, ewald_rc, ewald_kc; /* <= 0: gamma = 2.5/Omega^(1/3),
                                     Rc = 6/gamma, kc = 10 gamma (Sec. 3.3)      */
} mbd_system;

typedef struct {
    double *energy;               /* [1] Ha (per unit cell if periodic)          */
    double *grad_coords;          /* [N][3] dE/dR, Ha/bohr                        */
    double *grad_alpha0;          /* [N]                                          */
    double *grad_omega_or_c6;     /* [N] w.r.t. the given parameter kind          */
    double *grad_rvdw;            /* [N]                                          */
    double *grad_lattice;         /* [3][3] dE/dA_vc, Cartesian positions and
                                     fractional q fixed                           */
    double *eigvals;              /* [n_q or 1][3N] eigenvalues of Q ascending    */
    double *errors;               /* [4]: lambda_min; for MBD_FP32_REFINED also
                                     max|X^T X - I| of the FP32 eigenvectors, the
                                     number of refinement steps taken (1 or 2) and
                                     the estimated largest element error left in
                                     Q^{-1/2} after the last step; [1..3] are 0
                                     for MBD_FP64 and for a system re-evaluated
                                     on the FP64 path after the refinement missed
                                     its target.  Written on the device.        */
} mbd_result;

/* Create a context on HIP device `device` with the given precision.
 * hip_stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream),
 * or NULL for the default stream.  Returns MBD_ERR_DEVICE if the device
 * cannot be used. */
mbd_status mbd_create(mbd_ctx **ctx, int device, mbd_precision prec, void *hip_stream);

/* Release the context and all its device workspaces. */
mbd_status mbd_destroy(mbd_ctx *ctx);

/* Change the stream of an existing context (same device). */
mbd_status mbd_set_stream(mbd_ctx *ctx, void *hip_stream);

/* Energy and the requested gradients of one system (finite or periodic).
 * `want` is a bit set of MBD_WANT_*; an output pointer must be non-NULL when
 * its bit is set.  Collapse (some eigenvalue <= 0, Sec. 2.1) returns
 * MBD_ERR_NEGATIVE_EIGENVALUE with energy = NaN and, if MBD_WANT_ERRORS,
 * errors[0] = lambda_min; gradients are then not written.  Coincident atoms
 * (distance < 1e-8 bohr) and non-finite or non-positive per-atom inputs give
 * MBD_ERR_INVALID_ARGUMENT.  MBD_ERR_NOT_CONVERGED: see mbd_precision.
 * Periodic systems: the host reads coords and rvdw back once, ordered after
 * the work already queued on the context's stream, to build the image and
 * reciprocal-vector lists. */
mbd_status mbd_evaluate(mbd_ctx *ctx, const mbd_system *sys, unsigned want, mbd_result *out);

/* Many independent finite systems (molecules of uneven size) in one batched
 * launch sequence.  sys and out are HOST arrays of n_sys entries whose device
 * pointers follow mbd_evaluate; status (HOST, [n_sys]) receives each system's
 * mbd_status.  Periodic systems are not accepted here (MBD_ERR_UNSUPPORTED).
 * The launch sequence is captured once per batch signature (sizes, want,
 * precision) in a HIP graph and replayed on later calls with the same
 * signature.  Returns MBD_OK if every system succeeded, else the first
 * failing code.  At most 65535 systems per call (MBD_ERR_UNSUPPORTED). */
mbd_status mbd_evaluate_batch(mbd_ctx *ctx, int32_t n_sys, const mbd_system *sys, unsigned want,
                              mbd_result *out, int32_t *status);

/* No-allocation variant of mbd_evaluate, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * mbd_evaluate, for finite systems of at most MBD_NOALLOC_MAX_ATOMS atoms
 * (larger ones: MBD_ERR_INVALID_ARGUMENT; periodic: MBD_ERR_UNSUPPORTED).
 * Every workspace comes from one static device array of
 * MBD_NOALLOC_SCRATCH_BYTES per device (held until the process ends; its
 * address is resolved by mbd_create); the call makes no hipMalloc, hipFree or
 * other allocating call.  All calls on one device share that array, which
 * keeps the last call's contents (the kernels clear what must start at
 * zero): calls that overlap in time on one device, from any context or
 * stream, race and give undefined results. */
#define MBD_NOALLOC_MAX_ATOMS 256
#define MBD_NOALLOC_SCRATCH_BYTES (128ull << 20)
mbd_status mbd_evaluate_noalloc(mbd_ctx *ctx, const mbd_system *sys, unsigned want, mbd_result *out);

/* Pairwise (TS) dispersion energy and gradients (Sec. 2.6 eq:pairwise):
 *   E = -1/2 sum_{i != j} C6_ij f(R_ij)/R_ij^6,
 *   C6_ij = (3/2) alpha0_i alpha0_j / (1/omega_i + 1/omega_j),
 * f the Fermi damping of eq:fermi-damping with s_R = sys->beta and steepness
 * sys->a (the TS method uses a = 20).  Periodic (sys->lattice != NULL): the
 * energy per cell, summed over all images with the Ewald split of
 * eq:ts-ewald for the undamped R^-6 sum (ewald_gamma/rc/kc as for
 * mbd_evaluate, G = 0 term included) minus the real-space sum of (1-f)/R^6;
 * the q mesh fields are ignored.  want: MBD_WANT_ENERGY, _GRAD_COORDS,
 * _GRAD_ALPHA0, _GRAD_OMEGA (omega or C6 per param_kind), _GRAD_RVDW,
 * _ERRORS (all four set to 0); _GRAD_LATTICE and _EIGVALS give
 * MBD_ERR_UNSUPPORTED.  Input validation and errors as for mbd_evaluate. */
mbd_status mbd_ts_evaluate(mbd_ctx *ctx, const mbd_system *sys, unsigned want, mbd_result *out);

/* Frequency route of the MBD energy (Sec. 2.5), from the eigenvalues x_k of
 * K(u) = alpha(iu)^{1/2} T^lr alpha(iu)^{1/2}, alpha(iu) = alpha0/(1 +
 * u^2/omega^2) (eq:dyn-pol), on n_freq Gauss-Legendre points mapped by
 * u = 0.6 (1 + x)/(1 - x) (Sec. 3.3; the paper's default is 15), and for
 * periodic systems on every q of the mesh (averaged).  terms (DEVICE,
 * [3 + n_order]) receives
 *   [0] E = (1/2pi) int du sum_k ln(1 + x_k)            (eq:log-formula;
 *       NaN inside the dipole collapse, where some 1 + x_k <= 0)
 *   [1] (1/2pi) int du sum_k (ln(1 + x~_k) - x~_k)       (eq:gould-norm, the
 *       renormalised energy; finite inside the collapse)
 *   [2] the smallest 1 + x_k over all u (and q): the collapse indicator
 *   [2 + n] E^(n) = -(1/2pi) int du ((-1)^n/n) sum_k x_k^n, n = 1..n_order
 *       (eq:rpa; E^(1) vanishes for finite systems)
 * 1 <= n_freq <= 512, 1 <= n_order <= 60, and n_freq times the number of q
 * points at most 65535 (MBD_ERR_UNSUPPORTED).  The eigenvalues are computed in
 * FP64 whatever the context's precision (no eigenvectors are formed).
 * Inputs, validation and Ewald parameters as for mbd_evaluate; the outputs
 * of mbd_result are not used. */
mbd_status mbd_freq_evaluate(mbd_ctx *ctx, const mbd_system *sys, int32_t n_freq, int32_t n_order, double *terms);

/* MBD@rsSCS (Secs. 2.3 and 2.7), finite systems: the self-consistent
 * screening stage followed by the MBD energy with the screened parameters.
 * At u = 0 and at n_freq Gauss-Legendre points (map of Sec. 3.3; the paper's
 * default is 15), alpha_bar(u) = (alpha(iu)^-1 + T^scs)^-1 (eq:scs) with
 * T^scs = (1 - g) T^GG (eq:scs-sr-dipole, eq:tgg, Mayer widths eq:mayer; g
 * with steepness sys->a and s_R = sys->beta on the input R_vdW), contracted
 * per atom (eq:contraction); C6 by eq:casimir-polder, omega = 4 C6/(3
 * alpha_bar0^2), R_vdW scaled by (alpha_bar0/alpha0)^{1/3}
 * (eq:scale-rvdw-scs).  The MBD energy (T^lr = g T with the scaled radii,
 * eq:mbd-lr-dipole) runs at the context's precision; the screening stage is
 * always FP64.  want: MBD_WANT_ENERGY, _GRAD_COORDS (dE/dR through the
 * screened parameters: the derivative of eq:scs contracted as in
 * eq:contraction), _EIGVALS, _ERRORS; other bits give MBD_ERR_UNSUPPORTED,
 * as does a lattice.  scs_params (DEVICE, may be NULL): [4][N] screened
 * alpha0, C6, omega, R_vdW.  alpha_bar(u) is never formed: the contraction
 * and the gradient need it only applied to three columns, which come from a
 * Cholesky factorisation of alpha(iu)^-1 + T^scs per frequency.  A matrix
 * that is not positive definite (a non-positive pivot) gives
 * MBD_ERR_NEGATIVE_EIGENVALUE. */
mbd_status mbd_rsscs_evaluate(mbd_ctx *ctx, const mbd_system *sys, int32_t n_freq, unsigned want, mbd_result *out,
                              double *scs_params);

/* Dense symmetric eigensolver of the MBD path, exposed for testing and reuse:
 * the Householder reduction, divide-and-conquer tridiagonal solve and
 * back-transform used for Q.  A: [nbatch] matrices of order n, column-major
 * with leading dimension lda, consecutive matrices `stride` elements apart,
 * lower triangle read (copied into a library workspace first; A itself is
 * not modified).  w: [nbatch][n] eigenvalues ascending.
 * Z (may be NULL): [nbatch] n x n eigenvector matrices, leading dimension ldz,
 * stride `zstride`.  dtype: 0 = FP64, 1 = FP32 (then A, w, Z are float).
 * A matrix whose reduction yields a non-finite entry (NaN or Inf in A) gives
 * MBD_ERR_INVALID_ARGUMENT; its w and Z are then not meaningful (the other
 * matrices of the batch are solved as usual).  In mbd_evaluate and its
 * variants the same condition fails the system with that code.  At most
 * 65535 matrices per call (MBD_ERR_UNSUPPORTED). */
mbd_status mbd_eigh(mbd_ctx *ctx, int32_t dtype, int32_t n, int32_t nbatch, void *A, int32_t lda,
                    int64_t stride, void *w, void *Z, int32_t ldz, int64_t zstride);

/* Measure the launch-shape choices of the path for the problem sizes given
 * (HOST array sizes[nsizes] of matrix orders) and store the fastest in the
 * context; if table_json_path is non-NULL the table is written there.  An
 * existing table can be loaded with mbd_load_tuning.  Two choices are
 * measured per order: the reduction's SYMV work-item target (kernel time
 * summed separately over the upper quarter of trailing sizes and below it)
 * and the general GEMM's output tile (64 or 128, an FP64 n x n x n product
 * timed with both).  Table format, per precision of the context
 * ("fp64" / "fp32"): {"<order>": [upper_target, lower_target, gemm_tile]};
 * the loader also takes [upper, lower] or a single target (then the GEMM
 * tile is chosen by order) and rejects tiles other than 0, 64 and 128.  An
 * evaluation uses the row of the tuned order nearest its matrix order (on a
 * log scale), the GEMM tile only when that order is within a factor 2.
 * Both calls retire the batch launch graphs the context has captured (they
 * hold the previous shapes); the next mbd_evaluate_batch captures anew. */
mbd_status mbd_autotune(mbd_ctx *ctx, const int32_t *sizes, int32_t nsizes, const char *table_json_path);
mbd_status mbd_load_tuning(mbd_ctx *ctx, const char *table_json_path);

/* Launch timing for measurement tools.  While enabled, every per-column
 * launch of the Householder reduction and every trailing SYR2K launch (kind 1,
 * the matrix-core BLAS-3 phase) is bracketed by two HIP events on the context
 * stream, and so is each phase of an evaluation: 2 input preparation and
 * assembly, 3 Householder reduction, 4 divide and conquer, 5 back-transform,
 * 6 refinement (FP32 path), 7 energy, Q^{-1/2} and gradients.  The per-column
 * launches are kind 0 where a column takes a SYMV launch and a finish launch
 * (large trailing orders), kind 8 where one fused launch finishes the previous
 * column and runs the column's SYMV (FP32, trailing order up to 4000).
 * Kind 9 is the screening stage of mbd_rsscs_evaluate (assembly, Cholesky
 * factorisation and solves, contraction; and the chain rule of its gradient).
 * Kind 10 is the single launch that reduces a batch of small matrices with
 * one workgroup per matrix (FP64 batches of 256 or more matrices of
 * order <= 1024).  Kind 11 is the pair kernel of mbd_ts_evaluate.  Enabling
 * clears earlier records.  mbd_get_profile synchronises
 * the stream and returns, for one kind (0..11), the summed event time (ms),
 * the number of records and the summed algorithmic work: bytes of the lower
 * trailing triangle read (kinds 0, 8 and 10), flops of the rank-2k update
 * (kind 1), pair terms (kind 11: N (N - 1) ordered pairs for a finite system,
 * N^2 times the image and reciprocal terms for a cell), 0 for the phases.
 * enable = 2 records the
 * phases only, without timing events (which would slow every launch): the
 * stream is synchronised at each phase boundary and the host clock read. */
mbd_status mbd_set_profiling(mbd_ctx *ctx, int enable);

/* Host-only self-check of the divide-and-conquer workspace for matrices of
 * order <= n_max (no device needed): FP32 merges of order 2048 and more
 * gather their operands into buffers of ldz * n_max + 64 elements per matrix
 * (ldz = n_max rounded up to 64).  *needed gets the furthest element, from a
 * matrix's base, that the gather and the split product touch (0 when no such
 * merge exists), *allocated the buffer size.  Returns MBD_OK if the one fits
 * the other, MBD_ERR_UNSUPPORTED if not (the eigensolver refuses such an
 * order with the same code), MBD_ERR_INVALID_ARGUMENT for n_max < 1 or NULL
 * outputs. */
mbd_status mbd_check_dc_buffers(int32_t n_max, int64_t *needed, int64_t *allocated);
mbd_status mbd_get_profile(mbd_ctx *ctx, int32_t kind, double *total_ms, int64_t *launches, double *work);

/* (code, origin, message) of the last error on the context; returns code.
 * origin and message stay valid until the next call on the context. */
int mbd_last_error(const mbd_ctx *ctx, const char **origin, const char **message);

#ifdef __cplusplus
}
#endif
#endif
