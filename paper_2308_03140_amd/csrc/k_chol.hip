// Batched Cholesky factorisation A = L L^T of symmetric positive definite
// FP64 matrices and solves with a few right-hand sides.  The screening of
// MBD@rsSCS (Sec. 2.3, eq:scs) needs alpha_bar(u) = A(u)^-1 only through
// alpha_bar B, with B = 1 (x) I_3 for the contraction (eq:contraction) and
// B = w (x) I_3 for the gradient, so one factorisation per frequency and
// two three-column solves replace the inverse.  A non-positive pivot (A not
// positive definite: the screening collapses) sets MBD_ST_COLLAPSE.
//
// Right-looking, panels of CHOL_NB = 64 columns:
//   diagonal block   one workgroup per matrix factors the 64 x 64 block in
//                    LDS and inverts its factor, L11^-1, kept for the
//                    panel solve and the triangular solves;
//   panel            L21 = A21 L11^-T as a matrix-core product, in place;
//   trailing update  A22 -= L21 L21^T on the lower tiles (matrix cores).
// The triangular solves go block row by block row, one launch per block:
// every workgroup forms the block's solution from the (final) residual and
// L11^-1, the first stores it, the others update the residual of their own
// block row.
#include <algorithm>

#include "gemm_mfma.h"
#include "mbd_internal.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

#define CHOL_NB 64
#define CHOL_NR 3  // right-hand sides per solve

// ---------------------------------------------------------------------------
// diagonal block: factor, invert the factor; identity padding past n
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chol_diag_kernel(MatBatch<double> A, double* Linv, long long sLi, int n,
                                                         int k0, unsigned* status) {
    __shared__ double L[CHOL_NB][CHOL_NB + 1];
    __shared__ double X[CHOL_NB][CHOL_NB + 1];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int w = min(CHOL_NB, n - k0);
    double* Ab = A.at(b) + k0 + (long long)k0 * A.ld;
    const long long ld = A.ld;
    for (int t = tid; t < CHOL_NB * CHOL_NB; t += 256) {
        const int i = t & (CHOL_NB - 1), j = t / CHOL_NB;
        L[i][j] = (i < w && j < w) ? (i >= j ? Ab[i + j * ld] : 0.0) : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    bool bad = false;
    for (int j = 0; j < w; j++) {
        const double d = L[j][j];
        const bool nb = !(d > 0.0);
        bad = bad || nb;
        const double s = nb ? 1.0 : sqrt(d);
        __syncthreads();
        if (tid == 0) L[j][j] = s;
        for (int i = j + 1 + tid; i < CHOL_NB; i += 256) L[i][j] /= s;
        __syncthreads();
        for (int t = tid; t < CHOL_NB * CHOL_NB; t += 256) {
            const int i = t & (CHOL_NB - 1), l = t / CHOL_NB;
            if (l > j && i >= l) L[i][l] -= L[i][j] * L[l][j];
        }
        __syncthreads();
    }
    if (bad && tid == 0) atomicOr(status, MBD_ST_COLLAPSE);
    // X = L^-1 (lower), one column per thread: X(c,c) = 1/L(c,c),
    // X(i,c) = -(sum_{l=c}^{i-1} L(i,l) X(l,c)) / L(i,i)
    if (tid < CHOL_NB) {
        const int c = tid;
        for (int i = 0; i < c; i++) X[i][c] = 0.0;
        X[c][c] = 1.0 / L[c][c];
        for (int i = c + 1; i < CHOL_NB; i++) {
            double s = 0.0;
            for (int l = c; l < i; l++) s += L[i][l] * X[l][c];
            X[i][c] = -s / L[i][i];
        }
    }
    __syncthreads();
    for (int t = tid; t < CHOL_NB * CHOL_NB; t += 256) {
        const int i = t & (CHOL_NB - 1), j = t / CHOL_NB;
        if (i < w && j < w && i >= j) Ab[i + j * ld] = L[i][j];
    }
    double* Xo = Linv + (long long)b * sLi + (long long)(k0 / CHOL_NB) * CHOL_NB * CHOL_NB;
    for (int t = tid; t < CHOL_NB * CHOL_NB; t += 256) {
        const int i = t & (CHOL_NB - 1), j = t / CHOL_NB;
        Xo[i + j * CHOL_NB] = X[i][j];  // column-major, leading dimension 64
    }
}

// ---------------------------------------------------------------------------
// panel: L21 = A21 X^T (X = L11^-1), rows k0 + 64 .. n-1, in place.  A tile
// spans the panel's 64 columns, so a workgroup reads only the rows it writes.
// ---------------------------------------------------------------------------
struct CholPanelProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = true;
    MatBatch<double> A;
    const double* Linv; long long sLi;
    int k0, rows;  // rows = n - k0 - 64
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        t.batch = bz;
        t.m0 = bx * CHOL_NB; t.n0 = 0; t.K = CHOL_NB;
        return t.m0 < rows;
    }
    __device__ double a(const GemmTile& t, int m, int k) const {
        if (m >= rows) return 0.0;
        return A.at(t.batch)[(k0 + CHOL_NB + m) + (long long)(k0 + k) * A.ld];
    }
    __device__ double b(const GemmTile& t, int k, int c) const {
        // X^T(k, c) = X(c, k)
        return Linv[(long long)t.batch * sLi + (long long)(k0 / CHOL_NB) * CHOL_NB * CHOL_NB + c + k * CHOL_NB];
    }
    __device__ void store(const GemmTile& t, int m, int c, double v) const {
        if (m < rows) A.at(t.batch)[(k0 + CHOL_NB + m) + (long long)(k0 + c) * A.ld] = v;
    }
};

// ---------------------------------------------------------------------------
// trailing update: A22 -= L21 L21^T on the lower tiles (elements on and below
// the diagonal), TS x TS tiles in the XCD-aware banded order
// ---------------------------------------------------------------------------
template <int TS>
struct CholSyrkProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = true;
    MatBatch<double> A;
    int k0, m;  // panel start, trailing order m = n - k0 - 64
    int tiles;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        t.batch = bz;
        int ti, tj;
        band_lower_tile(xcd_virtual(bx, gridDim.x), tiles, ti, tj);
        t.m0 = ti * TS; t.n0 = tj * TS; t.K = CHOL_NB;
        return t.m0 < m && t.n0 < m;
    }
    __device__ double a(const GemmTile& t, int r, int k) const {
        if (r >= m) return 0.0;
        return A.at(t.batch)[(k0 + CHOL_NB + r) + (long long)(k0 + k) * A.ld];
    }
    __device__ double b(const GemmTile& t, int k, int c) const {
        if (c >= m) return 0.0;
        return A.at(t.batch)[(k0 + CHOL_NB + c) + (long long)(k0 + k) * A.ld];
    }
    __device__ void store(const GemmTile& t, int r, int c, double v) const {
        if (r >= m || c > r) return;
        A.at(t.batch)[(k0 + CHOL_NB + r) + (long long)(k0 + CHOL_NB + c) * A.ld] -= v;
    }
};

// ---------------------------------------------------------------------------
// triangular solves; right-hand sides row-major [n][CHOL_NR] per matrix
// ---------------------------------------------------------------------------
// forward step for block kb: y_kb = X_kb r_kb; workgroup 0 stores it, workgroup
// j >= 1 updates the residual of block kb + j: r -= L(kb + j, kb) y_kb
__global__ __launch_bounds__(256) void chol_fwd_kernel(MatBatch<double> A, const double* Linv, long long sLi, int n,
                                                        int kb, double* R, double* Y, long long sR) {
    __shared__ double Xs[CHOL_NB][CHOL_NB + 1];
    __shared__ double rs[CHOL_NB][CHOL_NR];
    __shared__ double ys[CHOL_NB][CHOL_NR];
    const int b = blockIdx.z, j = blockIdx.x, tid = threadIdx.x;
    const int r0 = kb * CHOL_NB;
    const double* Xg = Linv + (long long)b * sLi + (long long)kb * CHOL_NB * CHOL_NB;
    double* Rb = R + (long long)b * sR;
    for (int t = tid; t < CHOL_NB * CHOL_NB; t += 256) Xs[t & (CHOL_NB - 1)][t / CHOL_NB] = Xg[t];
    for (int t = tid; t < CHOL_NB * CHOL_NR; t += 256) {
        const int i = t / CHOL_NR, c = t % CHOL_NR;
        rs[i][c] = r0 + i < n ? Rb[(long long)(r0 + i) * CHOL_NR + c] : 0.0;
    }
    __syncthreads();
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid / CHOL_NR, c = tid % CHOL_NR;
        double s = 0.0;
        for (int l = 0; l <= i; l++) s += Xs[i][l] * rs[l][c];
        ys[i][c] = s;
    }
    __syncthreads();
    if (j == 0) {
        for (int t = tid; t < CHOL_NB * CHOL_NR; t += 256) {
            const int i = t / CHOL_NR, c = t % CHOL_NR;
            if (r0 + i < n) Y[(long long)b * sR + (long long)(r0 + i) * CHOL_NR + c] = ys[i][c];
        }
        return;
    }
    const int q0 = (kb + j) * CHOL_NB;
    const double* Ab = A.at(b);
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid % CHOL_NB, c = tid / CHOL_NB;
        const int q = q0 + i;
        if (q < n) {
            double s = 0.0;
            for (int l = 0; l < CHOL_NB && r0 + l < n; l++) s += Ab[q + (long long)(r0 + l) * A.ld] * ys[l][c];
            Rb[(long long)q * CHOL_NR + c] -= s;
        }
    }
}

// backward step for block kb: x_kb = X_kb^T y_kb; workgroup 0 stores it,
// workgroup j >= 1 updates block kb - j: y -= L(kb, kb - j)^T x_kb
__global__ __launch_bounds__(256) void chol_bwd_kernel(MatBatch<double> A, const double* Linv, long long sLi, int n,
                                                        int kb, double* Yr, double* Xo, long long sR) {
    __shared__ double Xs[CHOL_NB][CHOL_NB + 1];
    __shared__ double rs[CHOL_NB][CHOL_NR];
    __shared__ double xs[CHOL_NB][CHOL_NR];
    const int b = blockIdx.z, j = blockIdx.x, tid = threadIdx.x;
    const int r0 = kb * CHOL_NB;
    const double* Xg = Linv + (long long)b * sLi + (long long)kb * CHOL_NB * CHOL_NB;
    double* Yb = Yr + (long long)b * sR;
    for (int t = tid; t < CHOL_NB * CHOL_NB; t += 256) Xs[t & (CHOL_NB - 1)][t / CHOL_NB] = Xg[t];
    for (int t = tid; t < CHOL_NB * CHOL_NR; t += 256) {
        const int i = t / CHOL_NR, c = t % CHOL_NR;
        rs[i][c] = r0 + i < n ? Yb[(long long)(r0 + i) * CHOL_NR + c] : 0.0;
    }
    __syncthreads();
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid / CHOL_NR, c = tid % CHOL_NR;
        double s = 0.0;
        for (int l = i; l < CHOL_NB; l++) s += Xs[l][i] * rs[l][c];
        xs[i][c] = s;
    }
    __syncthreads();
    if (j == 0) {
        for (int t = tid; t < CHOL_NB * CHOL_NR; t += 256) {
            const int i = t / CHOL_NR, c = t % CHOL_NR;
            if (r0 + i < n) Xo[(long long)b * sR + (long long)(r0 + i) * CHOL_NR + c] = xs[i][c];
        }
        return;
    }
    const int q0 = (kb - j) * CHOL_NB;
    const double* Ab = A.at(b);
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid % CHOL_NB, c = tid / CHOL_NB;
        const int q = q0 + i;
        double s = 0.0;
        for (int l = 0; l < CHOL_NB && r0 + l < n; l++) s += Ab[(r0 + l) + (long long)q * A.ld] * xs[l][c];
        Yb[(long long)q * CHOL_NR + c] -= s;
    }
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
long long chol_linv_stride(int n) { return (long long)((n + CHOL_NB - 1) / CHOL_NB) * CHOL_NB * CHOL_NB; }

void chol_factor_launch(hipStream_t st, MatBatch<double> A, int n, int nbatch, double* Linv, unsigned* status) {
    const long long sLi = chol_linv_stride(n);
    for (int k0 = 0; k0 < n; k0 += CHOL_NB) {
        hipLaunchKernelGGL(chol_diag_kernel, dim3(nbatch), dim3(256), 0, st, A, Linv, sLi, n, k0, status);
        const int rows = n - k0 - CHOL_NB;
        if (rows <= 0) break;
        CholPanelProb pp;
        pp.A = A; pp.Linv = Linv; pp.sLi = sLi; pp.k0 = k0; pp.rows = rows;
        hipLaunchKernelGGL((gemm_mfma_kernel<double, CholPanelProb>), dim3((rows + CHOL_NB - 1) / CHOL_NB, 1, nbatch),
                           dim3(256), 0, st, pp);
        if (rows >= GEMM_TS128_MIN_ORDER) {
            typedef Gemm128Shape<double> S;
            CholSyrkProb<128> ps;
            ps.A = A; ps.k0 = k0; ps.m = rows; ps.tiles = (rows + 127) / 128;
            hipLaunchKernelGGL((gemm_mfma_kernel<double, CholSyrkProb<128>, 128, 128, S::BK, S::WM, S::WN>),
                               dim3(ps.tiles * (ps.tiles + 1) / 2, 1, nbatch), dim3(64 * S::WM * S::WN), 0, st, ps);
        } else {
            CholSyrkProb<64> ps;
            ps.A = A; ps.k0 = k0; ps.m = rows; ps.tiles = (rows + 63) / 64;
            hipLaunchKernelGGL((gemm_mfma_kernel<double, CholSyrkProb<64>>), dim3(ps.tiles * (ps.tiles + 1) / 2, 1, nbatch),
                               dim3(256), 0, st, ps);
        }
    }
}

// X = A^-1 B from the factor: B in R (overwritten), Y scratch, X out; all
// [nbatch][n][CHOL_NR] with per-matrix stride sR
void chol_solve_launch(hipStream_t st, MatBatch<double> A, int n, int nbatch, const double* Linv, double* R, double* Y,
                       double* X, long long sR) {
    const long long sLi = chol_linv_stride(n);
    const int nblk = (n + CHOL_NB - 1) / CHOL_NB;
    for (int kb = 0; kb < nblk; kb++)
        hipLaunchKernelGGL(chol_fwd_kernel, dim3(nblk - kb, 1, nbatch), dim3(256), 0, st, A, Linv, sLi, n, kb, R, Y,
                           sR);
    for (int kb = nblk - 1; kb >= 0; kb--)
        hipLaunchKernelGGL(chol_bwd_kernel, dim3(kb + 1, 1, nbatch), dim3(256), 0, st, A, Linv, sLi, n, kb, Y, X, sR);
}
