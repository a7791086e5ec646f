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
//   trailing update  A22 -= L21 L21^T on the lower tiles (matrix cores),
//                    once per superpanel of two panels (K = 128).
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
// One workgroup per matrix, the block in LDS; thread (i, j0) = (tid & 63,
// tid >> 6) works on row i and columns j0, j0 + 4, ...  (A single-wavefront
// variant without barriers, the row in LDS, measured 171 us against 100 us.)
__global__ __launch_bounds__(256) void chol_diag_kernel(MatBatch<double> A, double* Linv, long long sLi, int n,
                                                         int k0, unsigned* status) {
    __shared__ double L[CHOL_NB][CHOL_NB + 1];
    __shared__ double X[CHOL_NB][CHOL_NB + 1];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int w = min(CHOL_NB, n - k0);
    double* Ab = A.at(b) + k0 + (long long)k0 * A.ld;
    const long long ld = A.ld;
    constexpr int PER = CHOL_NB * CHOL_NB / 256;
    const int ri = tid & (CHOL_NB - 1), j0 = tid >> 6;
    {
        // all 16 loads in flight together (rows and columns clamped, values masked)
        double v[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int j = j0 + 4 * u;
            v[u] = Ab[min(ri, w - 1) + (long long)min(j, w - 1) * ld];
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int j = j0 + 4 * u;
            L[ri][j] = (ri < w && j < w) ? (ri >= j ? v[u] : 0.0) : (ri == j ? 1.0 : 0.0);
        }
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
        if (tid > j && tid < CHOL_NB) L[tid][j] /= s;
        __syncthreads();
        // trailing update L(i, l) -= L(i, j) L(l, j), j < l <= i
        const double lij = L[ri][j];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int l = j0 + 4 * u;
            if (l > j && ri >= l) L[ri][l] -= lij * L[l][j];
        }
        __syncthreads();
    }
    if (bad && tid == 0) atomicOr(status, MBD_ST_COLLAPSE);
    // X = L^-1 row by row: X(r, c) = -(sum_{l=c}^{r-1} L(r,l) X(l,c)) / L(r,r)
    // for c < r; four threads per column c split the sum over l
    {
        const int c = tid >> 2, part = tid & 3;
        if (part == 0) {
            for (int r = 0; r < CHOL_NB; r++) X[r][c] = r == c ? 1.0 / L[c][c] : 0.0;
        }
        __syncthreads();
        for (int r = 1; r < CHOL_NB; r++) {
            double sacc = 0.0;
            if (c < r)
                for (int l = c + part; l < r; l += 4) sacc += L[r][l] * X[l][c];
            sacc += __shfl_xor(sacc, 1, 64);
            sacc += __shfl_xor(sacc, 2, 64);
            if (c < r && part == 0) X[r][c] = -sacc / L[r][r];
            __syncthreads();
        }
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int j = j0 + 4 * u;
        if (ri < w && j < w && ri >= j) Ab[ri + j * ld] = L[ri][j];
    }
    double* Xo = Linv + (long long)b * sLi + (long long)(k0 / CHOL_NB) * CHOL_NB * CHOL_NB;
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int j = j0 + 4 * u;
        Xo[ri + j * CHOL_NB] = X[ri][j];  // column-major, leading dimension 64
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
// trailing update: A22 -= L21 L21^T with L21 the kw columns from k0 (64 or a
// superpanel of 128), on the elements on and below the diagonal of the
// block from t0 = k0 + kw: all lower tiles (XCD-aware banded order), or
// (thin) only the first ncols columns, one tile column
// ---------------------------------------------------------------------------
template <int TS>
struct CholSyrkProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = true;
    // read-modify-write of the tile in 16-byte column segments (the tile is
    // requested before the K loop); rows k0 + kw + r are even for even r, so
    // the segments are aligned
    static constexpr bool EPI_VEC = true;
    typedef typename Vec16<double>::v Vec;
    static constexpr int RPL = 2;
    MatBatch<double> A;
    int k0, kw, m, ncols;  // m = n - k0 - kw trailing rows
    int tiles, thin;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        t.batch = bz;
        int ti, tj;
        if (thin) { ti = bx; tj = 0; }
        else band_lower_tile(xcd_virtual(bx, gridDim.x), tiles, ti, tj);
        t.m0 = ti * TS; t.n0 = tj * TS; t.K = kw;
        return t.m0 < m && t.n0 < ncols;
    }
    __device__ double a(const GemmTile& t, int r, int k) const {
        if (r >= m || k >= kw) return 0.0;
        return A.at(t.batch)[(k0 + kw + r) + (long long)(k0 + k) * A.ld];
    }
    __device__ double b(const GemmTile& t, int k, int c) const {
        if (c >= ncols || k >= kw) return 0.0;
        return A.at(t.batch)[(k0 + kw + c) + (long long)(k0 + k) * A.ld];
    }
    __device__ Vec epi_load(const GemmTile& t, int r, int c) const {
        if (r >= m || c >= ncols || r + RPL <= c) return Vec{};
        return *reinterpret_cast<const Vec*>(A.at(t.batch) + (k0 + kw + r) + (long long)(k0 + kw + c) * A.ld);
    }
    __device__ void epi_store(const GemmTile& t, int r, int c, Vec acc, Vec cin) const {
        if (r >= m || c >= ncols || r + RPL <= c) return;
        double* a = A.at(t.batch) + (k0 + kw + r) + (long long)(k0 + kw + c) * A.ld;
        if (r >= c && r + RPL <= m) {
            *reinterpret_cast<Vec*>(a) = cin - acc;
        } else {
#pragma unroll
            for (int e = 0; e < RPL; e++)
                if (r + e >= c && r + e < m) a[e] = cin[e] - acc[e];
        }
    }
    __device__ void store(const GemmTile&, int, int, double) const {}
};

// ---------------------------------------------------------------------------
// triangular solves; right-hand sides row-major [n][CHOL_NR] per matrix
// ---------------------------------------------------------------------------
// 64 x 64 block of a column-major matrix into LDS, all loads in flight
// together (rows and columns clamped, values outside masked to zero)
__device__ __forceinline__ void chol_stage(double (*S)[CHOL_NB + 1], const double* src, long long ld, int rows,
                                           int cols) {
    constexpr int PER = CHOL_NB * CHOL_NB / 256;
    const int i = threadIdx.x & (CHOL_NB - 1), j0 = threadIdx.x >> 6;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int j = j0 + 4 * u;
        v[u] = src[min(i, rows - 1) + (long long)min(j, cols - 1) * ld];
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int j = j0 + 4 * u;
        S[i][j] = (i < rows && j < cols) ? v[u] : 0.0;
    }
}

// forward step for block kb: y_kb = X_kb r_kb; workgroup 0 stores it, workgroup
// j >= 1 updates the residual of block kb + j: r -= L(kb + j, kb) y_kb
__global__ __launch_bounds__(256) void chol_fwd_kernel(MatBatch<double> A, const double* Linv, long long sLi, int n,
                                                        int kb, double* R, double* Y, long long sR) {
    __shared__ double Xs[CHOL_NB][CHOL_NB + 1];
    __shared__ double Ls[CHOL_NB][CHOL_NB + 1];
    __shared__ double rs[CHOL_NB][CHOL_NR];
    __shared__ double ys[CHOL_NB][CHOL_NR];
    const int b = blockIdx.z, j = blockIdx.x, tid = threadIdx.x;
    const int r0 = kb * CHOL_NB, q0 = (kb + j) * CHOL_NB;
    double* Rb = R + (long long)b * sR;
    const double rv = tid < CHOL_NB * CHOL_NR && r0 + tid / CHOL_NR < n
                          ? Rb[(long long)r0 * CHOL_NR + tid] : 0.0;
    chol_stage(Xs, Linv + (long long)b * sLi + (long long)kb * CHOL_NB * CHOL_NB, CHOL_NB, CHOL_NB, CHOL_NB);
    if (j > 0) chol_stage(Ls, A.at(b) + q0 + (long long)r0 * A.ld, A.ld, min(CHOL_NB, n - q0), min(CHOL_NB, n - r0));
    if (tid < CHOL_NB * CHOL_NR) rs[tid / CHOL_NR][tid % CHOL_NR] = rv;
    __syncthreads();
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid / CHOL_NR, c = tid % CHOL_NR;
        double s = 0.0;
#pragma unroll 8
        for (int l = 0; l <= i; l++) s += Xs[i][l] * rs[l][c];
        ys[i][c] = s;
    }
    __syncthreads();
    if (j == 0) {
        if (tid < CHOL_NB * CHOL_NR && r0 + tid / CHOL_NR < n)
            Y[(long long)b * sR + (long long)r0 * CHOL_NR + tid] = ys[tid / CHOL_NR][tid % CHOL_NR];
        return;
    }
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid / CHOL_NR, c = tid % CHOL_NR;
        double s = 0.0;
#pragma unroll 8
        for (int l = 0; l < CHOL_NB; l++) s += Ls[i][l] * ys[l][c];
        if (q0 + i < n) Rb[(long long)(q0 + i) * CHOL_NR + c] -= s;
    }
}

// backward step for block kb: x_kb = X_kb^T y_kb; workgroup 0 stores it,
// workgroup j >= 1 updates block kb - j: y -= L(kb, kb - j)^T x_kb
__global__ __launch_bounds__(256) void chol_bwd_kernel(MatBatch<double> A, const double* Linv, long long sLi, int n,
                                                        int kb, double* Yr, double* Xo, long long sR) {
    __shared__ double Xs[CHOL_NB][CHOL_NB + 1];
    __shared__ double Ls[CHOL_NB][CHOL_NB + 1];
    __shared__ double rs[CHOL_NB][CHOL_NR];
    __shared__ double xs[CHOL_NB][CHOL_NR];
    const int b = blockIdx.z, j = blockIdx.x, tid = threadIdx.x;
    const int r0 = kb * CHOL_NB, q0 = (kb - j) * CHOL_NB;
    double* Yb = Yr + (long long)b * sR;
    const double rv = tid < CHOL_NB * CHOL_NR && r0 + tid / CHOL_NR < n
                          ? Yb[(long long)r0 * CHOL_NR + tid] : 0.0;
    chol_stage(Xs, Linv + (long long)b * sLi + (long long)kb * CHOL_NB * CHOL_NB, CHOL_NB, CHOL_NB, CHOL_NB);
    // L(kb, kb - j): rows r0.., columns q0.. (below the diagonal)
    if (j > 0) chol_stage(Ls, A.at(b) + r0 + (long long)q0 * A.ld, A.ld, min(CHOL_NB, n - r0), CHOL_NB);
    if (tid < CHOL_NB * CHOL_NR) rs[tid / CHOL_NR][tid % CHOL_NR] = rv;
    __syncthreads();
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid / CHOL_NR, c = tid % CHOL_NR;
        double s = 0.0;
#pragma unroll 8
        for (int l = i; l < CHOL_NB; l++) s += Xs[l][i] * rs[l][c];
        xs[i][c] = s;
    }
    __syncthreads();
    if (j == 0) {
        if (tid < CHOL_NB * CHOL_NR && r0 + tid / CHOL_NR < n)
            Xo[(long long)b * sR + (long long)r0 * CHOL_NR + tid] = xs[tid / CHOL_NR][tid % CHOL_NR];
        return;
    }
    if (tid < CHOL_NB * CHOL_NR) {
        const int i = tid / CHOL_NR, c = tid % CHOL_NR;
        double s = 0.0;
#pragma unroll 8
        for (int l = 0; l < CHOL_NB; l++) s += Ls[l][i] * xs[l][c];
        Yb[(long long)(q0 + i) * CHOL_NR + c] -= s;
    }
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
long long chol_linv_stride(int n) { return (long long)((n + CHOL_NB - 1) / CHOL_NB) * CHOL_NB * CHOL_NB; }

static void chol_syrk(hipStream_t st, MatBatch<double> A, int nbatch, int k0, int kw, int m, bool thin) {
    if (!thin && m >= GEMM_TS128_MIN_ORDER) {
        typedef Gemm128Shape<double> S;
        CholSyrkProb<128> ps;
        ps.A = A; ps.k0 = k0; ps.kw = kw; ps.m = m; ps.ncols = m; ps.thin = 0; ps.tiles = (m + 127) / 128;
        hipLaunchKernelGGL((gemm_mfma_kernel<double, CholSyrkProb<128>, 128, 128, S::BK, S::WM, S::WN>),
                           dim3(ps.tiles * (ps.tiles + 1) / 2, 1, nbatch), dim3(64 * S::WM * S::WN), 0, st, ps);
        return;
    }
    CholSyrkProb<64> ps;
    ps.A = A; ps.k0 = k0; ps.kw = kw; ps.m = m; ps.thin = thin ? 1 : 0;
    ps.ncols = thin ? std::min(m, CHOL_NB) : m;
    ps.tiles = (m + 63) / 64;
    const int grid = thin ? ps.tiles : ps.tiles * (ps.tiles + 1) / 2;
    hipLaunchKernelGGL((gemm_mfma_kernel<double, CholSyrkProb<64>>), dim3(grid, 1, nbatch), dim3(256), 0, st, ps);
}

static void chol_panel(hipStream_t st, MatBatch<double> A, int n, int nbatch, double* Linv, long long sLi, int k0,
                       unsigned* status, int& rows) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(nbatch), dim3(256), 0, st, A, Linv, sLi, n, k0, status);
    rows = n - k0 - CHOL_NB;
    if (rows <= 0) return;
    CholPanelProb pp;
    pp.A = A; pp.Linv = Linv; pp.sLi = sLi; pp.k0 = k0; pp.rows = rows;
    hipLaunchKernelGGL((gemm_mfma_kernel<double, CholPanelProb>), dim3((rows + CHOL_NB - 1) / CHOL_NB, 1, nbatch),
                       dim3(256), 0, st, pp);
}

// Superpanels of 128 columns: the first 64-column panel, its update of the
// second panel's columns only, the second panel, then one trailing update
// with both (K = 128: twice the flops per byte of a 64-deep update).
void chol_factor_launch(hipStream_t st, MatBatch<double> A, int n, int nbatch, double* Linv, unsigned* status) {
    const long long sLi = chol_linv_stride(n);
    for (int k0 = 0; k0 < n; k0 += 2 * CHOL_NB) {
        int rows1, rows2;
        chol_panel(st, A, n, nbatch, Linv, sLi, k0, status, rows1);
        if (rows1 <= 0) break;
        chol_syrk(st, A, nbatch, k0, CHOL_NB, rows1, true);
        chol_panel(st, A, n, nbatch, Linv, sLi, k0 + CHOL_NB, status, rows2);
        if (rows2 <= 0) break;
        chol_syrk(st, A, nbatch, k0, 2 * CHOL_NB, rows2, false);
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
