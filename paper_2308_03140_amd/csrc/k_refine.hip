// Refinement of approximate eigenpairs in FP64 against the FP64 Q, applied to
// the eigenvectors of the FP32 diagonalisation (Ogita & Aishima, "Iterative
// refinement for symmetric eigenvalue decomposition", 2018, with the treatment
// of close eigenvalues of their 2019 sequel, "... II: clustered eigenvalues",
// in Rayleigh-Ritz form).  One step on X (n x n, columns ~ eigenvectors):
//
//   S = X^T Q X, G = X^T X (both symmetric, lower triangles formed),
//   R = I - G, lam_i = S_ii / G_ii
//   delta = 2 (||S - diag(lam)||_F + max|lam| ||R||_F)   (Frobenius bounds of
//           the spectral norms in the method's separation threshold; reported,
//           not used: with FP32 eigenvectors of large matrices it exceeds the
//           typical eigenvalue spacing, and grouping by it merges the spectrum)
//   windows: column i joins the window of column i-1 when the linear
//           correction between i and one of the OA_LINK previous columns,
//           |S_ji + lam_i R_ji| / |lam_i - lam_j|, exceeds OA_TAU (the step is
//           only second-order accurate for such pairs), or when their lam
//           agree to rounding; windows are cut at OA_KMAX columns
//   per window J: the generalised problem S_JJ v = mu G_JJ v (Cholesky of
//           G_JJ, cyclic Jacobi), W_JJ = [v] (G-orthonormal), lam_J <- mu
//   in the rotated basis X' = X W:  S' = W^T S W, R' = -W^T G W off the
//           diagonal blocks, and
//             E'_ij = (S'_ij + lam_j R'_ij) / (lam_j - lam_i)  i, j in different
//                     windows with |lam_i - lam_j| above rounding level
//             E'_ij = R'_ij / 2   other pairs of different windows (unresolved)
//             E'_ii = R_ii / 2    single-column windows, 0 inside windows
//   X <- (X' + X' E') D = X + X F,  F = ((W - I) + W E') D + (D - I),
//           D = diag(1/sqrt(1 + eta_j)), eta_j = sum_{i != j} E'_ij^2
//   lam_j <- Rayleigh quotient of the refined column j, expanded from S', G'
//           and E' (no further product with Q)
//
// The leftover of a step is second order in the cross-window correction:
// column j grows in norm by eta_j = sum_{i != j} E'_ij^2, and
// rho = max_j eta_j max_r|X_rj|^2 / sqrt(lam_j) estimates the largest element
// error it leaves in Q^{-1/2} = X diag(lam^{-1/2}) X^T before the column
// rescaling below.  A matrix takes a second step when rho > OA_RHO_NEXT or
// when the step cut a run of linked columns into windows of OA_KMAX (a cut
// between columns whose lam agree to rounding is harmless and not counted):
// the second step's runs then form around the old cut, where the pairs left
// over sit.  If the second step ends with rho above the threshold divided by
// OA_RHO_FINAL_DIV (there rho measures the error left, where after the first
// step it overstates it), or with a cut, the matrix is reported as not
// converged.  The decisions stay on
// the device (per-matrix flags), so captured launch graphs remain valid.
#include "mbd_internal.h"
#include "gemm_mfma.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

// The default threshold OA_RHO_NEXT = 3e-5 (OaWork::rho_next overrides when
// > 0): rho estimates the remainder before the column rescaling, which
// removes most of it (measured factor 3-6 on FP32 eigenvectors of n =
// 100..6000); at 3e-5 the element error left in Q^{-1/2} stays near 6e-6 or
// below, which keeps the gradients within 1e-6 and the energy within 1e-12
// Ha/atom of FP64.
#define OA_TAU 1e-4
#define OA_LINK 4
#define OA_CP 6  // per-column partials: s2 (then eta), r2, max|R|, |lam|, max|x|, spare

// one workgroup per column (rows in steps of 256): grid (nmax, 1, nbatch)
__global__ __launch_bounds__(256) void oa_f2d_kernel(const int* ns, MatBatch<float> X32, MatBatch<double> Xd) {
    const int b = blockIdx.z;
    const int n = ns[b];
    const int c = blockIdx.x;
    if (c >= n) return;
    const float* src = X32.at(b) + (long long)c * X32.ld;
    double* dst = Xd.at(b) + (long long)c * Xd.ld;
    for (int r = threadIdx.x; r < n; r += 256) dst[r] = (double)src[r];
}

// dst = src; with only_skipped, just for the matrices whose skip flag is set;
// one workgroup per column: grid (nmax, 1, nbatch)
__global__ __launch_bounds__(256) void copy_mat_kernel(const int* ns, MatBatch<double> src, MatBatch<double> dst,
                                                         const int* only_skipped = nullptr) {
    const int b = blockIdx.z;
    if (only_skipped && !only_skipped[b]) return;
    const int n = ns[b];
    const int c = blockIdx.x;
    if (c >= n) return;
    const double* sc = src.at(b) + (long long)c * src.ld;
    double* dc = dst.at(b) + (long long)c * dst.ld;
    for (int r = threadIdx.x; r < n; r += 256) dc[r] = sc[r];
}

__global__ void fill_u32_kernel(unsigned* p, int n, unsigned v) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ double sym_lower(const double* G, int ld, int r, int c) {
    return r >= c ? G[r + (long long)c * ld] : G[c + (long long)r * ld];
}

// lam_c = S_cc / G_cc and per-column partials of ||S - diag(lam)||_F^2 and
// ||R||_F^2 (the strictly lower part counted twice, plus the diagonal), max|R|,
// |lam| and max|X|.  S and G hold their lower triangles, read contiguously.
__global__ __launch_bounds__(256) void oa_colstats_kernel(const int* ns, MatBatch<double> S, MatBatch<double> G,
                                                            MatBatch<double> X, double* lam, long long sL,
                                                            double* colpart, double* gdiag, const int* skip) {
    __shared__ double red[4];
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int c = blockIdx.x;
    if (c >= n) return;
    const double* Sc = S.at(b) + (long long)c * S.ld;
    const double* Gc = G.at(b) + (long long)c * G.ld;
    const double* Xc = X.at(b) + (long long)c * X.ld;
    double s2 = 0.0, r2 = 0.0, rmax = 0.0, xmax = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) {
        if (r > c) {
            const double sv = Sc[r], rv = Gc[r];
            s2 += 2.0 * sv * sv;
            r2 += 2.0 * rv * rv;
            rmax = fmax(rmax, fabs(rv));
        }
        xmax = fmax(xmax, fabs(Xc[r]));
    }
    s2 = block_sum256(s2, red);
    r2 = block_sum256(r2, red);
    rmax = block_max256(rmax, red);
    xmax = block_max256(xmax, red);
    if (threadIdx.x == 0) {
        const double scc = Sc[c], gcc = Gc[c];
        const double l = scc / gcc;
        const double rcc = 1.0 - gcc;
        lam[(long long)b * sL + c] = l;
        gdiag[(long long)b * sL + c] = gcc;
        double* cp = colpart + ((long long)b * sL + c) * OA_CP;
        cp[0] = s2 + (scc - l) * (scc - l);
        cp[1] = r2 + rcc * rcc;
        cp[2] = fmax(rmax, fabs(rcc));
        cp[3] = fabs(l);
        cp[4] = xmax;
    }
}

// per matrix: stats = {delta, max|R|, (rho), max|X|}; clears the unresolved
// pair counter and the per-column accumulators of the correction
__global__ __launch_bounds__(256) void oa_delta_kernel(const int* ns, double* colpart, long long sL,
                                                         double* stats, unsigned* nclust, const int* skip) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (skip && skip[b]) return;
    const int n = ns[b];
    double s2 = 0, r2 = 0, rmax = 0, lmax = 0, xmax = 0;
    for (int c = threadIdx.x; c < n; c += 256) {
        double* cp = colpart + ((long long)b * sL + c) * OA_CP;
        s2 += cp[0];
        r2 += cp[1];
        rmax = fmax(rmax, cp[2]);
        lmax = fmax(lmax, cp[3]);
        xmax = fmax(xmax, cp[4]);
        // reused by the E' kernel: [0] eta, [1] and [2] the numerator terms,
        // [5] the denominator term of the refined Rayleigh quotient ([3] is
        // cleared by the windows kernel after it has read |lam|)
        cp[0] = 0.0;
        cp[1] = 0.0;
        cp[2] = 0.0;
        cp[5] = 0.0;
    }
    s2 = block_sum256(s2, red);
    r2 = block_sum256(r2, red);
    rmax = block_max256(rmax, red);
    lmax = block_max256(lmax, red);
    xmax = block_max256(xmax, red);
    if (threadIdx.x == 0) {
        stats[4 * b] = 2.0 * (sqrt(s2) + lmax * sqrt(r2));
        stats[4 * b + 1] = rmax;
        stats[4 * b + 2] = 0.0;
        stats[4 * b + 3] = xmax;
        nclust[b] = 0u;
    }
}

// Windows: a new run starts at column i unless it links to one of the
// OA_LINK previous columns; runs are cut into chunks of OA_KMAX columns.
// One block per matrix; each thread scans a contiguous segment, with carries
// across segments taken from LDS.  wstart[i] = first column of i's window,
// wlen[i] = its length.
__device__ __forceinline__ bool oa_break(const double* Sb, int lds, const double* Gb, int ldg, const double* L,
                                         int i, double tiny) {
    if (i == 0) return true;
    const double li = L[i];
    for (int d = 1; d <= OA_LINK && i - d >= 0; d++) {
        const int j = i - d;
        const double dl = fabs(li - L[j]);
        const double sji = Sb[i + (long long)j * lds];  // i > j: lower triangle
        const double rji = -Gb[i + (long long)j * ldg];
        if (dl <= tiny || fabs(sji + li * rji) > OA_TAU * dl) return false;
    }
    return true;
}

__global__ __launch_bounds__(256) void oa_windows_kernel(const int* ns, MatBatch<double> S, MatBatch<double> G,
                                                           const double* lam, long long sL, double* colpart,
                                                           int* wstart, int* wlen, unsigned* nclust,
                                                           const int* skip) {
    __shared__ int last[256], first[256];
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const double* L = lam + (long long)b * sL;
    const double* Sb = S.at(b);
    const double* Gb = G.at(b);
    const int t = threadIdx.x;
    double lmax = 0.0;
    for (int c = t; c < n; c += 256) {
        double* cp3 = colpart + ((long long)b * sL + c) * OA_CP + 3;
        lmax = fmax(lmax, *cp3);
        *cp3 = 0.0;
    }
    const double tiny = 64.0 * num_limits<double>::eps * block_max256(lmax, red);
    const int seg = (n + 255) / 256;
    const int i0 = min(n, t * seg), i1 = min(n, i0 + seg);
    int* ws = wstart + (long long)b * sL;
    int* wl = wlen + (long long)b * sL;
    int lst = -1, fst = n;
    for (int i = i0; i < i1; i++) {
        const bool brk = oa_break(Sb, S.ld, Gb, G.ld, L, i, tiny);
        wl[i] = brk ? 1 : 0;
        if (brk) {
            lst = i;
            if (fst == n) fst = i;
        }
    }
    last[t] = lst;
    first[t] = fst;
    __syncthreads();
    int run = -1, nxt = n;
    for (int u = 0; u < t; u++) run = max(run, last[u]);
    for (int u = t + 1; u < 256; u++) nxt = min(nxt, first[u]);
    for (int i = i0; i < i1; i++) {  // run starts
        if (wl[i]) run = i;
        ws[i] = run;
    }
    unsigned ncut = 0;
    for (int i = i1 - 1; i >= i0; i--) {  // run ends, then chunks
        const bool brk = wl[i] != 0;
        const int rs = ws[i];
        const int cs = rs + OA_KMAX * ((i - rs) / OA_KMAX);
        // a chunk boundary inside a run: the linked pair (i - 1, i) is
        // left to the linear correction, which the link test judged
        // inaccurate for it (harmless only when their lam agree to rounding)
        if (cs == i && i != rs && fabs(L[i] - L[i - 1]) > tiny) ncut++;
        ws[i] = cs;
        wl[i] = min(cs + OA_KMAX, nxt) - cs;
        if (brk) nxt = i;
    }
    if (ncut) atomicAdd(&nclust[b], ncut);
}

// Rayleigh-Ritz per window of k >= 2 columns: one 64-lane block, k <= 32.
// S_JJ (symmetrised) and G_JJ -> L = chol(G_JJ), A = L^-1 S_JJ L^-T, cyclic
// Jacobi A = U diag(mu) U^T, V = L^-T U; columns ordered by ascending mu.
// wv[(b sL + cs + r) * OA_KMAX + p] = V_pr, lam[cs + r] = mu_r.
__global__ __launch_bounds__(64) void oa_rr_kernel(const int* ns, MatBatch<double> S, MatBatch<double> G,
                                                     double* lam, long long sL, const int* wstart, const int* wlen,
                                                     double* wv, const int* skip) {
    __shared__ double Am[OA_KMAX][OA_KMAX + 1], Lm[OA_KMAX][OA_KMAX + 1], Im[OA_KMAX][OA_KMAX + 1],
        Um[OA_KMAX][OA_KMAX + 1];
    __shared__ int rank[OA_KMAX];
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int cs = blockIdx.x;
    if (cs >= n) return;
    const long long o = (long long)b * sL;
    const int k = wlen[o + cs];
    if (wstart[o + cs] != cs || k < 2) return;
    const int tid = threadIdx.x;
    const double* Sb = S.at(b);
    const double* Gb = G.at(b);
    for (int e = tid; e < k * k; e += 64) {
        const int r = e % k, c = e / k;
        Am[r][c] = sym_lower(Sb, S.ld, cs + r, cs + c);
        Lm[r][c] = sym_lower(Gb, G.ld, cs + r, cs + c);
        Um[r][c] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    // Cholesky of G_JJ in place (lower)
    for (int j = 0; j < k; j++) {
        if (tid == 0) {
            double d = Lm[j][j];
            for (int p = 0; p < j; p++) d -= Lm[j][p] * Lm[j][p];
            Lm[j][j] = sqrt(fmax(d, 1e-300));
        }
        __syncthreads();
        if (tid > j && tid < k) {
            double v = Lm[tid][j];
            for (int p = 0; p < j; p++) v -= Lm[tid][p] * Lm[j][p];
            Lm[tid][j] = v / Lm[j][j];
        }
        __syncthreads();
    }
    // L^-1, one column per lane
    if (tid < k) {
        const int c = tid;
        for (int r = 0; r < k; r++) {
            if (r < c) {
                Im[r][c] = 0.0;
                continue;
            }
            double v = r == c ? 1.0 : 0.0;
            for (int p = c; p < r; p++) v -= Lm[r][p] * Im[p][c];
            Im[r][c] = v / Lm[r][r];
        }
    }
    __syncthreads();
    // T = S_JJ L^-T into Lm, then A = L^-1 T into Am
    for (int e = tid; e < k * k; e += 64) {
        const int r = e % k, c = e / k;
        double v = 0.0;
        for (int m = 0; m <= c; m++) v += Am[r][m] * Im[c][m];
        Lm[r][c] = v;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += 64) {
        const int r = e % k, c = e / k;
        double v = 0.0;
        for (int m = 0; m <= r; m++) v += Im[r][m] * Lm[m][c];
        Am[r][c] = v;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += 64) {
        const int r = e % k, c = e / k;
        if (r < c) {
            const double v = 0.5 * (Am[r][c] + Am[c][r]);
            Am[r][c] = v;
            Am[c][r] = v;
        }
    }
    __syncthreads();
    // cyclic Jacobi: rotation (p, q) zeroes A_pq; lanes 0..31 update A,
    // lanes 32..63 update U.  Every lane evaluates the same rotation test on
    // the same LDS values, so the control flow stays uniform.
    for (int sweep = 0; sweep < 40; sweep++) {
        int rotated = 0;
        for (int p = 0; p < k - 1; p++)
            for (int q = p + 1; q < k; q++) {
                const double app = Am[p][p], aqq = Am[q][q], apq = Am[p][q];
                if (apq == 0.0 || !(fabs(apq) > 1e-17 * sqrt(fabs(app * aqq)))) continue;
                rotated = 1;
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                __syncthreads();
                if (tid < k) {  // A <- A J
                    const double arp = Am[tid][p], arq = Am[tid][q];
                    Am[tid][p] = c * arp - s * arq;
                    Am[tid][q] = s * arp + c * arq;
                } else if (tid >= 32 && tid - 32 < k) {  // U <- U J
                    const int r = tid - 32;
                    const double urp = Um[r][p], urq = Um[r][q];
                    Um[r][p] = c * urp - s * urq;
                    Um[r][q] = s * urp + c * urq;
                }
                __syncthreads();
                if (tid < k) {  // A <- J^T A
                    const double apr = Am[p][tid], aqr = Am[q][tid];
                    Am[p][tid] = c * apr - s * aqr;
                    Am[q][tid] = s * apr + c * aqr;
                }
                __syncthreads();
                if (tid == 0) {
                    Am[p][q] = 0.0;
                    Am[q][p] = 0.0;
                }
                __syncthreads();
            }
        if (!rotated) break;
    }
    if (tid < k) {
        const double mu = Am[tid][tid];
        int rk = 0;
        for (int s2 = 0; s2 < k; s2++) {
            const double ms = Am[s2][s2];
            rk += (ms < mu || (ms == mu && s2 < tid)) ? 1 : 0;
        }
        rank[tid] = rk;
        lam[o + cs + rk] = mu;
    }
    __syncthreads();
    // V = L^-T U, written per output column
    for (int e = tid; e < k * k; e += 64) {
        const int p = e % k, r = e / k;
        double v = 0.0;
        for (int m = p; m < k; m++) v += Im[m][p] * Um[m][r];
        wv[(o + cs + rank[r]) * OA_KMAX + p] = v;
    }
}

// E' (in the rotated basis) into Eo, one workgroup per column j (grid
// (nmax, 1, nbatch)); counts unresolved close pairs and sums over the rows
// the column terms below.  S and G hold both triangles (mirrored).  The
// rotated entries S'_ij = sum_p sum_q W(p, i) S(wi + p, wj + q) W(q, j) are
// formed in two steps: the column s1 = sum_q W(q, j) S(:, wj + q) (and g1 from
// G) is built once per chunk of OA_ECH rows, plus the OA_KMAX rows on either
// side that windows of the chunk's rows can reach, in LDS; each row then
// applies its own window's coefficients to s1 and g1.
#define OA_ECH 2048
__global__ __launch_bounds__(256) void oa_e_kernel(const int* ns, MatBatch<double> S, MatBatch<double> G,
                                                     MatBatch<double> Eo, const double* lam, long long sL,
                                                     const int* wstart, const int* wlen, const double* wv,
                                                     const double* stats, unsigned* nclust, double* colpart,
                                                     const double* gdiag, const int* skip) {
    __shared__ double red[4];
    __shared__ double s1[OA_ECH + 2 * OA_KMAX], g1[OA_ECH + 2 * OA_KMAX];
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int j = blockIdx.x;
    if (j >= n) return;
    const long long o = (long long)b * sL;
    const double* Sb = S.at(b);
    const double* Gb = G.at(b);
    double* Ej = Eo.at(b) + (long long)j * Eo.ld;
    const int wj = wstart[o + j], kj = wlen[o + j];
    const double lj = lam[o + j];
    const double* vj = wv + (o + j) * OA_KMAX;
    // per column j: eta = sum_i E'_ij^2 (cross-window) and the terms of the
    // Rayleigh quotient of the refined column, x_j' = sum_i x'_i (I + E')_ij:
    //   num = S'_jj + sum_i (2 E'_ij S'_ij + E'_ij^2 S'_ii),
    //   den = G'_jj + sum_i (2 E'_ij G'_ij + E'_ij^2 G'_ii)
    double e2 = 0.0, a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int r0 = 0; r0 < n; r0 += OA_ECH) {
        const int lo = max(0, r0 - OA_KMAX), hi = min(n, r0 + OA_ECH + OA_KMAX);
        __syncthreads();  // the previous chunk's readers are done
        for (int r = lo + threadIdx.x; r < hi; r += 256) {
            double sv = 0.0, gv = 0.0;
            for (int q = 0; q < kj; q++) {
                const double cq = kj == 1 ? 1.0 : vj[q];
                sv += cq * Sb[r + (long long)(wj + q) * S.ld];
                gv += cq * Gb[r + (long long)(wj + q) * G.ld];
            }
            s1[r - lo] = sv;
            g1[r - lo] = gv;
        }
        __syncthreads();
        const int rend = min(n, r0 + OA_ECH);
        // four rows per thread and round, their loads issued together (rows
        // clamped into the chunk, results of rows past its end discarded)
        constexpr int RU = 4;
        for (int i0 = r0 + threadIdx.x; i0 < rend; i0 += RU * 256) {
            int wiu[RU], kiu[RU];
            double liu[RU], gdu[RU];
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int i = min(i0 + 256 * u, rend - 1);
                wiu[u] = wstart[o + i];
                kiu[u] = wlen[o + i];
                liu[u] = lam[o + i];
                gdu[u] = gdiag[o + i];
            }
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int i = i0 + 256 * u;
                if (i >= rend) continue;
                const int wi = wiu[u], ki = kiu[u];
                double e;
                if (wi == wj) {
                    if (ki == 1) {  // i == j, single-column window
                        const double gjj = g1[i - lo], sjj = s1[i - lo];
                        e = 0.5 * (1.0 - gjj);
                        a1 += 2.0 * e * sjj;
                        a2 += e * e * sjj;
                        b1 += 2.0 * e * gjj;
                        b2 += e * e * gjj;
                    } else {
                        e = 0.0;
                    }
                } else {
                    double sp, gp;
                    if (ki == 1) {
                        sp = s1[i - lo];
                        gp = g1[i - lo];
                    } else {
                        const double* vi = wv + (o + i) * OA_KMAX;
                        sp = 0.0;
                        gp = 0.0;
                        for (int p = 0; p < ki; p++) {
                            const double cp_ = vi[p];
                            sp += cp_ * s1[wi + p - lo];
                            gp += cp_ * g1[wi + p - lo];
                        }
                    }
                    const double li = liu[u];
                    const double dl = lj - li;
                    if (fabs(dl) > 64.0 * num_limits<double>::eps * fmax(fabs(li), fabs(lj))) {
                        e = (sp - lj * gp) / dl;
                    } else {
                        // lam agree to rounding: the pair's rotation leaves
                        // Q^{-1/2} unchanged, only its symmetric part is kept
                        e = -0.5 * gp;
                    }
                    const double ee = e * e;
                    const double gii = ki == 1 ? gdu[u] : 1.0;
                    e2 += ee;
                    a1 += 2.0 * e * sp;
                    a2 += ee * li * gii;
                    b1 += 2.0 * e * gp;
                    b2 += ee * gii;
                }
                Ej[i] = e;
            }
        }
    }
    e2 = block_sum256(e2, red);
    a1 = block_sum256(a1, red);
    a2 = block_sum256(a2, red);
    b1 = block_sum256(b1, red);
    b2 = block_sum256(b2, red);
    if (threadIdx.x == 0) {
        // zeroed by the delta and window passes; this workgroup is the only writer
        double* cp = colpart + (o + j) * OA_CP;
        cp[0] = e2;
        cp[1] = a1;
        cp[2] = a2;
        cp[3] = b1;
        cp[5] = b2;
    }
}

// F = ((W - I) + W E') D + (D - I) into Fo, W block diagonal over the windows,
// D = diag(1/sqrt(1 + eta_j)): the cross-window corrections are orthogonal to
// column j, so they lengthen it by eta_j = sum_i E'_ij^2 (accumulated by the
// E' kernel); rescaling removes that second-order term without a further
// product, so X + X F has columns of unit length to that order.
__global__ __launch_bounds__(256) void oa_f_kernel(const int* ns, MatBatch<double> Ei, MatBatch<double> Fo,
                                                     long long sL, const int* wstart, const int* wlen,
                                                     const double* wv, const double* colpart, const int* skip) {
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int j = blockIdx.x;
    if (j >= n) return;
    const long long o = (long long)b * sL;
    const double* Ej = Ei.at(b) + (long long)j * Ei.ld;
    double* Fj = Fo.at(b) + (long long)j * Fo.ld;
    const int wsj = wstart[o + j];
    const double d = 1.0 / sqrt(1.0 + colpart[(o + j) * OA_CP]);
    for (int i = threadIdx.x; i < n; i += 256) {
        const int wi = wstart[o + i], ki = wlen[o + i];
        double f;
        if (ki == 1) {
            f = Ej[i];
        } else {
            const int p = i - wi;
            f = (wsj == wi) ? wv[(o + j) * OA_KMAX + p] - (i == j ? 1.0 : 0.0) : 0.0;
            for (int a = 0; a < ki; a++) f += wv[(o + wi + a) * OA_KMAX + p] * Ej[wi + a];
        }
        Fj[i] = f * d + (i == j ? d - 1.0 : 0.0);
    }
}

// Update of the first step, whose X holds the FP32 eigenvectors exactly:
// F = F_blk + F_small, with
//   F_blk   the entries inside multi-column windows, (W - I)_ij d_j +
//           delta_ij (d_j - 1): order one (the Rayleigh-Ritz rotations);
//   F_small everything else, (W E')_ij d_j and the single-window diagonal
//           E'_jj d_j + (d_j - 1): at most the linear correction's size.
// X + X F_blk is formed exactly in FP64 (at most OA_KMAX columns per output
// column); X F_small = X32 fl32(F_small) runs on the matrix cores in split
// FP16 (below) and is added in FP64.  fexp[j] is the power of two that brings
// the largest |F_small(:, j)| into [2^14, 2^15) for that split.
__global__ __launch_bounds__(256) void oa_fsmall_kernel(const int* ns, MatBatch<double> Ei, MatBatch<float> Fs,
                                                          int* fexp, long long sL, const int* wstart, const int* wlen,
                                                          const double* wv, const double* colpart, const int* skip) {
    __shared__ float red[4];
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int j = blockIdx.x;
    if (j >= n) return;
    const long long o = (long long)b * sL;
    const double* Ej = Ei.at(b) + (long long)j * Ei.ld;
    float* Fj = Fs.at(b) + (long long)j * Fs.ld;
    const int wsj = wstart[o + j];
    const double d = 1.0 / sqrt(1.0 + colpart[(o + j) * OA_CP]);
    float fmx = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) {
        const int wi = wstart[o + i], ki = wlen[o + i];
        double f;
        if (ki == 1) {
            f = Ej[i] * d + (i == j ? d - 1.0 : 0.0);
        } else if (wi == wsj) {
            f = 0.0;  // inside column j's window: F_blk
        } else {
            const int p = i - wi;
            f = 0.0;
            for (int a = 0; a < ki; a++) f += wv[(o + wi + a) * OA_KMAX + p] * Ej[wi + a];
            f *= d;
        }
        Fj[i] = (float)f;
        fmx = fmaxf(fmx, fabsf((float)f));
    }
    fmx = block_max256(fmx, red);
    if (threadIdx.x == 0) fexp[o + j] = fmx > 0.0f ? min(110, max(-60, 14 - ilogbf(fmx))) : 0;
}

// T1 = X + X F_blk, one workgroup per column j
__global__ __launch_bounds__(256) void oa_fblock_kernel(const int* ns, MatBatch<double> X, MatBatch<double> T1,
                                                          long long sL, const int* wstart, const int* wlen,
                                                          const double* wv, const double* colpart, const int* skip) {
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int j = blockIdx.x;
    if (j >= n) return;
    const long long o = (long long)b * sL;
    const int wsj = wstart[o + j], kj = wlen[o + j];
    const double* Xb = X.at(b);
    double* Tj = T1.at(b) + (long long)j * T1.ld;
    const double* Xj = Xb + (long long)j * X.ld;
    if (kj == 1) {
        for (int r = threadIdx.x; r < n; r += 256) Tj[r] = Xj[r];
        return;
    }
    const double d = 1.0 / sqrt(1.0 + colpart[(o + j) * OA_CP]);
    const double* vj = wv + (o + j) * OA_KMAX;
    for (int r = threadIdx.x; r < n; r += 256) {
        double t = Xj[r];
        for (int p = 0; p < kj; p++) {
            const int i = wsj + p;
            const double fb = (vj[p] - (i == j ? 1.0 : 0.0)) * d + (i == j ? d - 1.0 : 0.0);
            t += Xb[r + (long long)i * X.ld] * fb;
        }
        Tj[r] = t;
    }
}

// T1 += X32 F_small: FP32 operands on the matrix cores, FP64 accumulation of
// the result into T1
// ---------------------------------------------------------------------------
// C += X32 F_small on the FP16 matrix cores (v_mfma_f32_16x16x32_f16: lane l
// holds A(m = l % 16, k = 8 (l / 16) + e) and B(k = 8 (l / 16) + e, n = l % 16),
// e = 0..7, and result rows 4 (l / 16) + r of column l % 16).
//
// Each FP32 operand y is split as y = yh + yl, yh = fp16(y), yl = fp16(y - yh),
// after exact power-of-two scalings that keep both parts in FP16's normal
// range: X by 2^14 (|x| <= 1 in orthonormal columns), column j of F_small by
// 2^fexp[j].  X F is taken as Xh Fh + Xh Fl + Xl Fh with FP32 accumulation;
// the dropped Xl Fl and the parts' rounding leave about 2^-22 |X| |F_small|
// per term, below the FP32 accumulation error that follows and far below the
// step's second-order remainder |F_small|^2.  Three FP16 MFMA
// products cost less than one FP32 one.  The accumulators are unscaled and
// added to C in FP64.
//
// TS x TS tiles, 2 x 2 wavefronts, K in slabs of 32 staged through LDS
// (double buffered) as rows of k-contiguous FP16 values, so that each MFMA
// fragment is one 16-byte LDS read.
// ---------------------------------------------------------------------------
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int TS>
__global__ __launch_bounds__(256) void xf_small_f16_kernel(MatBatch<float> X, MatBatch<float> F, const int* fexp,
                                                             long long sL, MatBatch<double> C, const int* ns,
                                                             const int* skip, int tiles_n) {
    constexpr int BK = 32;              // K of one MFMA step and of one slab
    constexpr int WT = TS / 2;          // wavefront tile
    constexpr int MI = WT / 16, NJ = WT / 16;
    constexpr int LDK = BK + 8;         // halfs per LDS row: 80 bytes, 16-byte aligned
    constexpr int KPT = BK * TS / 256;  // k values per thread and operand in a slab
    static_assert(KPT % 8 == 0 && TS * (BK / KPT) == 256, "whole 16-byte LDS row pieces per thread");
    constexpr int TSZ = TS * LDK;
    __shared__ __align__(16) _Float16 lds[2][4][TSZ];  // [buffer][Xh, Xl, Fh, Fl]
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    int ti, tj;
    band_tile(xcd_virtual(blockIdx.x, gridDim.x), tiles_n, tiles_n, ti, tj);
    const int m0 = ti * TS, n0 = tj * TS;
    if (m0 >= n || n0 >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const long long o = (long long)b * sL;

    // staging: thread (rr, kq) loads row m0 + rr of X and column n0 + rr of
    // F for k = k0 + kq .. k0 + kq + KPT - 1; rows and columns past the order
    // read a clamped address and are zeroed, and so is k past the order
    const int rr = tid % TS, kq = (tid / TS) * KPT;
    const int mr = m0 + rr, nc = n0 + rr;
    const float* xrow = X.at(b) + (mr < n ? mr : n - 1);
    const float* fcol = F.at(b) + (long long)(nc < n ? nc : n - 1) * F.ld;
    const float xsc = mr < n ? 16384.0f : 0.0f;
    const float fsc = nc < n ? ldexpf(1.0f, fexp[o + nc]) : 0.0f;
    float xa[KPT], fa[KPT];
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < KPT; e++) {
            const int k = k0 + kq + e;
            xa[e] = xrow[(long long)(k < n ? k : n - 1) * X.ld];
        }
        // F's rows up to the next multiple of 32 lie inside its column (the
        // leading dimension is a multiple of 64): 16-byte loads
#pragma unroll
        for (int e = 0; e < KPT; e += 4) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(fcol + k0 + kq + e);
            fa[e] = v[0]; fa[e + 1] = v[1]; fa[e + 2] = v[2]; fa[e + 3] = v[3];
        }
    };
    // masking, scaling and the split happen here, after the slab's MFMAs,
    // so that the loads of the next slab are not waited for before them
    auto sstore = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < KPT / 8; q++) {
            half8 xh, xl, fh, fl;
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const bool ok = k0 + kq + 8 * q + e < n;
                const float x = ok ? xa[8 * q + e] * xsc : 0.0f, f = ok ? fa[8 * q + e] * fsc : 0.0f;
                const _Float16 h = (_Float16)x, g = (_Float16)f;
                xh[e] = h; xl[e] = (_Float16)(x - (float)h);
                fh[e] = g; fl[e] = (_Float16)(f - (float)g);
            }
            const int off = rr * LDK + kq + 8 * q;
            *reinterpret_cast<half8*>(&lds[buf][0][off]) = xh;
            *reinterpret_cast<half8*>(&lds[buf][1][off]) = xl;
            *reinterpret_cast<half8*>(&lds[buf][2][off]) = fh;
            *reinterpret_cast<half8*>(&lds[buf][3][off]) = fl;
        }
    };

    f32x4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int fo = (lane & 15) * LDK + 8 * (lane >> 4);  // fragment offset inside a 16-row group
    const int nk = (n + BK - 1) / BK;
    gload(0);
    sstore(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        half8 ah[MI], al[MI], bh[NJ], bl[NJ];
#pragma unroll
        for (int i = 0; i < MI; i++) {
            const int r = (wm * WT + 16 * i) * LDK + fo;
            ah[i] = *reinterpret_cast<const half8*>(&lds[buf][0][r]);
            al[i] = *reinterpret_cast<const half8*>(&lds[buf][1][r]);
        }
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int r = (wn * WT + 16 * j) * LDK + fo;
            bh[j] = *reinterpret_cast<const half8*>(&lds[buf][2][r]);
            bl[j] = *reinterpret_cast<const half8*>(&lds[buf][3][r]);
        }
        // the two small cross terms first, then the leading one
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        if (kt + 1 < nk) sstore(buf ^ 1, (kt + 1) * BK);
        __syncthreads();
    }
    double* Cb = C.at(b);
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int col = n0 + wn * WT + 16 * j + (lane & 15);
        if (col >= n) continue;
        const double sc = ldexp(1.0, -(14 + fexp[o + col]));
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int row = m0 + wm * WT + 16 * i + 4 * (lane >> 4) + r;
                if (row < n) Cb[row + (long long)col * C.ld] += (double)acc[i][j][r] * sc;
            }
    }
}

static void xf_small_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<float> X32,
                            MatBatch<float> Fs, const int* fexp, long long sL, MatBatch<double> T1,
                            const int* skip) {
    if (nmax >= GEMM_TS128_MIN_ORDER) {
        const int t = (nmax + 127) / 128;
        hipLaunchKernelGGL(xf_small_f16_kernel<128>, dim3(t * t, 1, nbatch), dim3(256), 0, st, X32, Fs, fexp, sL,
                           T1, ns, skip, t);
    } else {
        const int t = (nmax + 63) / 64;
        hipLaunchKernelGGL(xf_small_f16_kernel<64>, dim3(t * t, 1, nbatch), dim3(256), 0, st, X32, Fs, fexp, sL,
                           T1, ns, skip, t);
    }
}

// rho = max_c eta_c max|x_c|^2 / sqrt(lam_c) -> stats[4b+2]; next[b] = 1
// (skip the next step) unless rho > the threshold or the step left pairs it
// could not treat accurately (runs of linked columns cut into windows, pairs
// of different windows whose lam agree to rounding); lam <- Rayleigh
// quotients of the refined columns
__global__ __launch_bounds__(256) void oa_next_kernel(const int* ns, const double* colpart, double* lam,
                                                        long long sL, MatBatch<double> G, const int* wlen,
                                                        double* stats, const unsigned* nclust, const int* skip,
                                                        int* next, double rho_next) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    if (skip && skip[b]) {
        if (threadIdx.x == 0) next[b] = 1;
        return;
    }
    const int n = ns[b];
    const long long o = (long long)b * sL;
    const double* Gb = G.at(b);
    double rho = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) {
        const double* cp = colpart + (o + c) * OA_CP;
        const double l = lam[o + c];
        if (l > 0.0) rho = fmax(rho, cp[0] * cp[4] * cp[4] / sqrt(l));
        // Rayleigh quotient of the refined column (the rescaling by D leaves it unchanged)
        const double g = wlen[o + c] == 1 ? Gb[c + (long long)c * G.ld] : 1.0;
        lam[o + c] = (l * g + cp[1] + cp[2]) / (g + cp[3] + cp[5]);
    }
    rho = block_max256(rho, red);
    if (threadIdx.x == 0) {
        stats[4 * b + 2] = rho;
        next[b] = (rho > rho_next || nclust[b] != 0u) ? 0 : 1;
    }
}

void oa_f2d_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<float> X32, MatBatch<double> Xd) {
    hipLaunchKernelGGL(oa_f2d_kernel, dim3(nmax, 1, nbatch), dim3(256), 0, st, ns, X32, Xd);
}

void copy_mat_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> src,
                     MatBatch<double> dst) {
    hipLaunchKernelGGL(copy_mat_kernel, dim3(nmax, 1, nbatch), dim3(256), 0, st, ns, src, dst);
}

void fill_u32_launch(hipStream_t st, unsigned* p, int n, unsigned v) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
}

size_t oa_colpart_doubles(int nmax, int nbatch) { return (size_t)nbatch * nmax * OA_CP; }

void oa_step_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> Q, MatBatch<double> X,
                    MatBatch<double> T1, MatBatch<double> T2, MatBatch<double> G, double* lam, long long sL,
                    const OaWork& w, double* stats, const int* skip, int* next, MatBatch<float> X32) {
    const dim3 gc(nmax, 1, nbatch);  // one workgroup per column
    gemm_batched<double>(st, false, false, ns, nmax, nbatch, Q.p, Q.ld, Q.stride, X.p, X.ld, X.stride, T1.p,
                         T1.ld, T1.stride, 1.0, 0.0, false, skip);                             // T1 = Q X
    // S = X^T Q X and G = X^T X (lower triangles) in one launch
    const GemmSecond<double> g2 = {X.p, X.ld, X.stride, G.p, G.ld, G.stride};
    gemm_batched_pair<double>(st, true, false, ns, nmax, nbatch, X.p, X.ld, X.stride, T1.p, T1.ld, T1.stride, T2.p,
                              T2.ld, T2.stride, g2, 1.0, 0.0, true, skip);
    hipLaunchKernelGGL(oa_colstats_kernel, dim3(nmax, 1, nbatch), dim3(256), 0, st, ns, T2, G, X, lam, sL,
                       w.colpart, w.gdiag, skip);
    hipLaunchKernelGGL(oa_delta_kernel, dim3(nbatch), dim3(256), 0, st, ns, w.colpart, sL, stats, w.nclust, skip);
    hipLaunchKernelGGL(oa_windows_kernel, dim3(nbatch), dim3(256), 0, st, ns, T2, G, lam, sL, w.colpart, w.wstart,
                       w.wlen, w.nclust, skip);
    hipLaunchKernelGGL(oa_rr_kernel, dim3(nmax, 1, nbatch), dim3(64), 0, st, ns, T2, G, lam, sL, w.wstart,
                       w.wlen, w.wv, skip);
    // both triangles of S and G for the column-contiguous reads of the E' pass
    mbd_mirror_launch(st, ns, nmax, nbatch, T2, skip);
    mbd_mirror_launch(st, ns, nmax, nbatch, G, skip);
    hipLaunchKernelGGL(oa_e_kernel, gc, dim3(256), 0, st, ns, T2, G, T1, lam, sL, w.wstart, w.wlen, w.wv, stats,
                       w.nclust, w.colpart, w.gdiag, skip);                                    // E' -> T1
    if (X32.p) {
        // X is the FP32 eigenvectors: T1 = X + X F_blk (FP64), then
        // T1 += X32 fl32(F_small) on the FP16 matrix cores; F_small in T2's memory
        const MatBatch<float> Fs = {(float*)T2.p, T2.ld, 2 * T2.stride};
        hipLaunchKernelGGL(oa_fsmall_kernel, gc, dim3(256), 0, st, ns, T1, Fs, w.fexp, sL, w.wstart, w.wlen,
                           w.wv, w.colpart, skip);                                             // F_small -> T2
        hipLaunchKernelGGL(oa_next_kernel, dim3(nbatch), dim3(256), 0, st, ns, w.colpart, lam, sL, G, w.wlen, stats,
                           w.nclust, skip, next, w.rho_next > 0.0 ? w.rho_next : OA_RHO_NEXT);
        hipLaunchKernelGGL(oa_fblock_kernel, gc, dim3(256), 0, st, ns, X, T1, sL, w.wstart, w.wlen, w.wv,
                           w.colpart, skip);                                                   // T1 = X + X F_blk
        xf_small_launch(st, ns, nmax, nbatch, X32, Fs, w.fexp, sL, T1, skip);                  // T1 += X F_small
    } else {
        hipLaunchKernelGGL(oa_f_kernel, gc, dim3(256), 0, st, ns, T1, T2, sL, w.wstart, w.wlen, w.wv, w.colpart,
                           skip);                                                              // F -> T2
        hipLaunchKernelGGL(oa_next_kernel, dim3(nbatch), dim3(256), 0, st, ns, w.colpart, lam, sL, G, w.wlen, stats,
                           w.nclust, skip, next, w.rho_next > 0.0 ? w.rho_next : OA_RHO_NEXT);
        gemm_batched<double>(st, false, false, ns, nmax, nbatch, X.p, X.ld, X.stride, T2.p, T2.ld, T2.stride, T1.p,
                             T1.ld, T1.stride, 1.0, 1.0, false, skip, X.p, X.ld, X.stride);    // T1 = X + X F
    }
    // a matrix that skips this step passes X through unchanged
    if (skip) hipLaunchKernelGGL(copy_mat_kernel, gc, dim3(256), 0, st, ns, X, T1, skip);
}

// symmetric pseudo-random test matrix (autotuner input): A_rc = A_cr in [-1, 1)
template <typename T>
__global__ __launch_bounds__(256) void fill_sym_random_kernel(int n, T* A, int ld, unsigned seed) {
    const int c = blockIdx.y;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n || c >= n) return;
    unsigned x = (unsigned)min(r, c) * 2654435761u ^ ((unsigned)max(r, c) * 2246822519u) ^ seed;
    x ^= x >> 15; x *= 2654435761u; x ^= x >> 13; x *= 3266489917u; x ^= x >> 16;
    A[r + (long long)c * ld] = (T)((double)x * (2.0 / 4294967296.0) - 1.0);
}

template <typename T>
void fill_sym_random_launch(hipStream_t st, int n, T* A, int ld, unsigned seed) {
    hipLaunchKernelGGL(fill_sym_random_kernel<T>, dim3((n + 255) / 256, n), dim3(256), 0, st, n, A, ld, seed);
}
template void fill_sym_random_launch<double>(hipStream_t, int, double*, int, unsigned);
template void fill_sym_random_launch<float>(hipStream_t, int, float*, int, unsigned);
