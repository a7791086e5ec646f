// Back-transformation X = H_0 H_1 ... H_{n-2} Z of the tridiagonal
// eigenvectors Z to the eigenvectors C of Q (eq:diagonalization, paper
// Sec. 2.1).  Reflectors are grouped in blocks of 64 in compact-WY form
// H_b..H_{b+63} = I - V T V^T (T upper triangular) and applied from the last
// block to the first.  Up front, for all blocks at once (independent of X):
//   G = V^T V           split-K over 512-row chunks, partials summed in order
//   T                   from G and tau (forward column recurrence), one WG
//   VT = V T            matrix cores, stored densely per block
// then per pair of blocks h = k+1 (applied first) and k, in one pass over X:
//   Ypart = [V_k V_h]^T X   split-K over 512-row chunks on matrix cores
//   Y = sum Ypart           wide elementwise reduction: P_k (rows 0..63), P_h
//   Y_k = P_k - C_k P_h     C_k = V_k^T VT_h, computed up front for all pairs
//   X -= VT_k Y_k + VT_h P_h  matrix cores (a rank-128 update)
// which is block h's update followed by block k's; a block left over (block
// 0 of an odd count) is applied alone.  Both passes are bound by the X
// traffic, so pairing halves it.
// V is read straight from the reduced matrix with the unit diagonal and the
// zeros above it supplied by the loader.
#include "mbd_internal.h"
#include "gemm_mfma.h"
#include "mbd_kernels.h"

// element (r, i) of the reflector matrix
template <typename T>
__device__ __forceinline__ T hh_v(const T* A, long long ld, int r, int i, int nref) {
    if (i >= nref || r <= i) return T(0);
    if (r == i + 1) return T(1);
    return A[r + (long long)i * ld];
}

// Gpart[split] = V(rows of chunk)^T V(rows of chunk), 64 x 64
template <typename T>
struct VtvProb {
    static constexpr bool A_M_CONTIG = false;
    static constexpr bool B_N_CONTIG = false;
    MatBatch<T> A; const int* ns; T* Gpart; long long sG; int nsplit;
    // grid: x = reflector block, y = row chunk, z = matrix; t.k = x*nsplit + y
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        t.batch = bz;
        t.e0 = ns[bz];  // order, read once
        const int n = ns[bz];
        const int nref = n - 1;
        const int b0 = bx * 64;
        if (b0 >= nref) return false;
        const int m = n - b0 - 1;          // rows b0+1 .. n-1
        const int r0 = by * ORMTR_CHUNK;
        if (r0 >= m) return false;
        t.m0 = 0; t.n0 = 0;
        t.K = min(ORMTR_CHUNK, m - r0);
        t.o = b0 + 1 + r0;
        t.k = bx * nsplit + by;
        return true;
    }
    __device__ T a(const GemmTile& t, int jj, int kk) const {
        if (kk >= t.K) return T(0);
        const int b0 = (t.k / nsplit) * 64;
        return hh_v(A.at(t.batch), A.ld, t.o + kk, b0 + jj, t.e0 - 1);
    }
    __device__ T b(const GemmTile& t, int kk, int jj) const { return a(t, jj, kk); }
    __device__ void store(const GemmTile& t, int m, int nn, T v) const {
        Gpart[(long long)t.batch * sG + (long long)t.k * 4096 + m + nn * 64] = v;
    }
};

// T factor of every block (one workgroup each): T(j,j) = tau_j,
// T(0:j, j) = -tau_j T(0:j,0:j) G(0:j, j), G = V^T V summed over row chunks
template <typename T>
__global__ __launch_bounds__(256) void ormtr_tfactor_kernel(OrmtrWs<T> w, int nsplit) {
    __shared__ T G[64][65];
    __shared__ T Tm[64][65];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int nref = n - 1;
    const int blk = blockIdx.x;
    const int b0 = blk * 64;
    if (b0 >= nref) return;
    const int m = n - b0 - 1;
    const int ns_used = (m + ORMTR_CHUNK - 1) / ORMTR_CHUNK;
    const T* Gp = w.Gpart + (long long)b * w.sG + (long long)blk * nsplit * 4096;
    for (int idx = threadIdx.x; idx < 4096; idx += 256) {
        // partials in groups of 8 independent loads (split index clamped,
        // value masked) summed in split order
        T s = T(0);
        for (int q0 = 0; q0 < ns_used; q0 += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = Gp[(long long)min(q0 + u, ns_used - 1) * 4096 + idx];
#pragma unroll
            for (int u = 0; u < 8; u++) s += q0 + u < ns_used ? v[u] : T(0);
        }
        G[idx & 63][idx >> 6] = s;
        Tm[idx & 63][idx >> 6] = T(0);
    }
    __syncthreads();
    const T* tau = w.tau + (long long)b * w.sD;
    for (int j = 0; j < 64; j++) {
        const int i = b0 + j;
        const T tj = i < nref ? tau[i] : T(0);
        // z = T(0:j,0:j) G(0:j, j) for rows k < j
        T z = T(0);
        const int k = threadIdx.x;
        if (k < j)
            for (int l = k; l < j; l++) z += Tm[k][l] * G[l][j];
        __syncthreads();
        if (k < j) Tm[k][j] = -tj * z;
        if (k == j) Tm[j][j] = tj;
        __syncthreads();
    }
    T* To = w.Tm + (long long)b * w.sT + (long long)blk * 4096;
    for (int idx = threadIdx.x; idx < 4096; idx += 256) To[idx] = Tm[idx & 63][idx >> 6];
}

// Ypart[split] = V^T X over the rows of the chunk for the NR reflectors from
// b0 (one block, or a pair), NR x n, in 64 x TN tiles (grid x = NR / 64 row
// tiles x column tiles)
template <typename T, int TN, int NR = 64>
struct VtxProb {
    static constexpr bool A_M_CONTIG = false;
    static constexpr bool B_N_CONTIG = false;
    MatBatch<T> A; MatBatch<T> X; const int* ns; int b0; T* Ypart; long long sYp; int nmax; int tiles_n;
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        t.batch = bz;
        t.e0 = ns[bz];  // order, read once
        const int n = ns[bz];
        if (b0 >= n - 1) return false;
        const int m = n - b0 - 1;
        const int r0 = by * ORMTR_CHUNK;
        if (r0 >= m) return false;
        t.m0 = (bx / tiles_n) * 64;
        t.n0 = (bx % tiles_n) * TN;
        if (t.n0 >= n) return false;
        t.K = min(ORMTR_CHUNK, m - r0);
        t.o = b0 + 1 + r0;
        t.k = by;
        return true;
    }
    __device__ T a(const GemmTile& t, int jj, int kk) const {
        if (kk >= t.K) return T(0);
        return hh_v(A.at(t.batch), A.ld, t.o + kk, b0 + jj, t.e0 - 1);
    }
    __device__ T b(const GemmTile& t, int kk, int c) const {
        if (kk >= t.K || c >= t.e0) return T(0);
        return X.at(t.batch)[(t.o + kk) + (long long)c * X.ld];
    }
    __device__ void store(const GemmTile& t, int jj, int c, T v) const {
        if (c >= t.e0) return;
        Ypart[(long long)t.batch * sYp + (long long)t.k * NR * nmax + jj + (long long)c * NR] = v;
    }
};

// C_k = V_k^T VT_h (64 x 64) for every pair of blocks k, h = k+1 (pair p
// holds k = nblk - 2 - 2p): the sum runs over the rows of VT_h, b0h+1 ..
// n-1, split over 512-row chunks (grid x = pair, y = chunk); the partials
// go to Cpart and are summed in chunk order by ormtr_cpair_sum_kernel.  The
// first chunk is written even when block h lies past the order (zeros).
template <typename T>
struct CpairProb {
    static constexpr bool A_M_CONTIG = false;
    static constexpr bool B_N_CONTIG = false;
    MatBatch<T> A; const int* ns; const T* VT; long long sVT; T* Cpart; long long sCp; int nmax; int nblk; int nsplit;
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        t.batch = bz;
        const int n = ns[bz];
        t.e0 = n;  // order, read once
        const int k = nblk - 2 - 2 * bx;
        if (k < 0) return false;
        const int b0h = 64 * k + 64;
        const int m = max(0, n - b0h - 1);
        const int r0 = by * ORMTR_CHUNK;
        if (by > 0 && r0 >= m) return false;
        t.m0 = 0; t.n0 = 0;
        t.o = b0h + 1 + r0;        // first row of the chunk
        t.K = max(0, min(ORMTR_CHUNK, m - r0));
        t.k = bx * nsplit + by;
        t.e1 = b0h;
        return true;
    }
    __device__ T a(const GemmTile& t, int i, int kk) const {
        if (kk >= t.K) return T(0);
        return hh_v(A.at(t.batch), A.ld, t.o + kk, t.e1 - 64 + i, t.e0 - 1);
    }
    __device__ T b(const GemmTile& t, int kk, int j) const {
        if (kk >= t.K) return T(0);
        return VT[(long long)t.batch * sVT + (long long)(t.e1 / 64) * 64 * nmax + (long long)j * nmax +
                  (t.o - t.e1 - 1 + kk)];
    }
    __device__ void store(const GemmTile& t, int i, int j, T v) const {
        Cpart[(long long)t.batch * sCp + (long long)t.k * 4096 + i + j * 64] = v;
    }
};

// Cp[p] = sum over the row chunks of Cpart[p] (in chunk order), one
// workgroup per pair
template <typename T>
__global__ __launch_bounds__(256) void ormtr_cpair_sum_kernel(OrmtrWs<T> w, int nblk, int nsplit) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int p = blockIdx.x;
    const int b0h = 64 * (nblk - 2 - 2 * p) + 64;
    const int m = max(0, n - b0h - 1);
    const int nsu = max(1, (m + ORMTR_CHUNK - 1) / ORMTR_CHUNK);
    const T* Cq = w.Gpart + (long long)b * w.sG + (long long)p * nsplit * 4096;
    T* Co = w.Cp + (long long)b * w.sC + (long long)p * 4096;
    for (int idx = threadIdx.x; idx < 4096; idx += 256) {
        T s = T(0);
        for (int q = 0; q < nsu; q++) s += Cq[(long long)q * 4096 + idx];
        Co[idx] = s;
    }
}

// VT(block) = V T: rows b0+1 .. n-1 of the block's reflectors times its T
// factor; grid x = 64-row tile, y = block, z = matrix
template <typename T>
struct VtProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = false;
    MatBatch<T> A; const int* ns; const T* Tm; long long sT; T* VT; long long sVT; int nmax;
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        t.batch = bz;
        t.e0 = ns[bz];  // order, read once
        const int n = ns[bz];
        const int b0 = by * 64;
        if (b0 >= n - 1) return false;
        const int m = n - b0 - 1;
        t.m0 = bx * GEMM_BM;
        t.n0 = 0;
        t.K = 64;
        t.o = b0;
        t.k = m;
        return t.m0 < m;
    }
    __device__ T a(const GemmTile& t, int mm, int kk) const {
        if (mm >= t.k) return T(0);
        return hh_v(A.at(t.batch), A.ld, t.o + 1 + mm, t.o + kk, t.e0 - 1);
    }
    __device__ T b(const GemmTile& t, int kk, int jj) const {
        return Tm[(long long)t.batch * sT + (long long)(t.o / 64) * 4096 + kk + jj * 64];
    }
    __device__ void store(const GemmTile& t, int mm, int jj, T v) const {
        if (mm >= t.k) return;
        VT[(long long)t.batch * sVT + (long long)(t.o / 64) * 64 * nmax + (long long)jj * nmax + mm] = v;
    }
};

// Y(:, c) = sum over the row chunks of Ypart(:, c), NR rows per column
template <typename T>
__global__ __launch_bounds__(256) void ormtr_ysum_kernel(OrmtrWs<T> w, int b0, int NR) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    if (b0 >= n - 1) return;
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;  // jj + NR c
    if (idx >= (long long)NR * n) return;
    const int m = n - b0 - 1;
    const int nsu = (m + ORMTR_CHUNK - 1) / ORMTR_CHUNK;
    const T* Yp = w.Ypart + (long long)b * w.sYp + idx;
    T s = T(0);
    for (int q0 = 0; q0 < nsu; q0 += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = Yp[(long long)min(q0 + u, nsu - 1) * NR * w.nmax];
#pragma unroll
        for (int u = 0; u < 8; u++) s += q0 + u < nsu ? v[u] : T(0);
    }
    w.Y[(long long)b * w.sY + idx] = s;
}

// Y_k = P_k - C_k P_h for pair p (blocks k = b0k / 64 and k + 1): Y holds
// P_k in rows 0..63 and P_h in rows 64..127 of each column; ORMTR_FIX_COLS
// columns per workgroup, each staging C_k (64 columns per workgroup left
// most compute units idle on one large matrix: 94 workgroups at order 6000)
#define ORMTR_FIX_COLS 16
template <typename T>
__global__ __launch_bounds__(256) void ormtr_pair_fix_kernel(OrmtrWs<T> w, int b0k, int p) {
    constexpr int CW = ORMTR_FIX_COLS;
    __shared__ T C[64][65];
    __shared__ T Ph[CW][65];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    if (b0k >= n - 1) return;
    const int c0 = blockIdx.x * CW;
    if (c0 >= n) return;
    const T* Cg = w.Cp + (long long)b * w.sC + (long long)p * 4096;
    T* Y = w.Y + (long long)b * w.sY;
    for (int idx = threadIdx.x; idx < 4096; idx += 256) C[idx & 63][idx >> 6] = Cg[idx];
    for (int idx = threadIdx.x; idx < 64 * CW; idx += 256) {
        const int i = idx & 63, q = idx >> 6;
        Ph[q][i] = c0 + q < n ? Y[64 + i + (long long)(c0 + q) * 128] : T(0);
    }
    __syncthreads();
    const int i = threadIdx.x & 63;
    for (int q = threadIdx.x >> 6; q < CW; q += 4) {
        const int c = c0 + q;
        if (c >= n) break;
        T s = T(0);
#pragma unroll 8
        for (int j = 0; j < 64; j++) s += C[i][j] * Ph[q][j];
        Y[i + (long long)c * 128] -= s;
    }
}

// X(b0+1:n, :) -= VT Y, in TS x TS output tiles.  Tile rows are absolute
// rows of X counted from b0 (a multiple of 64), so that with the 64-padded
// leading dimension every 16-byte column segment is aligned; row b0 itself
// is outside the update (its VT row is zero) and is never written.  The
// epilogue reads X before the K loop and writes it back in 16-byte segments.
// With NR = 128 the K dimension spans the pair: columns kk < 64 are VT_k
// (rows from b0 + 1), kk >= 64 VT_h (rows from b0 + 65); both blocks' VT are
// adjacent in the VT buffer, and Y holds Y_k over P_h.
template <typename T, int TS, int NR = 64>
struct VyProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = false;
    static constexpr bool EPI_VEC = true;
    typedef typename Vec16<T>::v Vec;
    static constexpr int RPL = 16 / (int)sizeof(T);
    MatBatch<T> X; const int* ns; int b0; const T* VT; long long sVT; int nmax; const T* Y; long long sY; int tiles_n;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        t.batch = bz;
        t.e0 = ns[bz];  // order, read once
        const int n = ns[bz];
        if (b0 >= n - 1) return false;
        t.m0 = b0 + (bx / tiles_n) * TS;
        t.n0 = (bx % tiles_n) * TS;
        t.K = NR;
        return t.m0 < n && t.n0 < n;
    }
    __device__ T a(const GemmTile& t, int r, int jj) const {
        const int r0 = jj < 64 ? b0 : b0 + 64;  // the reflector block's first row b0 (+1 below)
        if (r <= r0 || r >= t.e0) return T(0);
        return VT[(long long)t.batch * sVT + (long long)(b0 / 64) * 64 * nmax + (long long)jj * nmax + (r - r0 - 1)];
    }
    __device__ T b(const GemmTile& t, int jj, int c) const {
        if (c >= t.e0) return T(0);
        return Y[(long long)t.batch * sY + jj + (long long)c * NR];
    }
    __device__ Vec epi_load(const GemmTile& t, int r, int c) const {
        const int n = t.e0;
        if (r >= n || c >= n) return Vec{};
        // r + RPL - 1 < ld: the run stays inside the padded column
        return *reinterpret_cast<const Vec*>(X.at(t.batch) + r + (long long)c * X.ld);
    }
    __device__ void epi_store(const GemmTile& t, int r, int c, Vec acc, Vec cin) const {
        const int n = t.e0;
        if (r >= n || c >= n) return;
        T* x = X.at(t.batch) + r + (long long)c * X.ld;
        if (r > b0 && r + RPL <= n) {
            *reinterpret_cast<Vec*>(x) = cin - acc;
        } else {
#pragma unroll
            for (int e = 0; e < RPL; e++)
                if (r + e > b0 && r + e < n) x[e] = cin[e] - acc[e];
        }
    }
    __device__ void store(const GemmTile&, int, int, T) const {}
};

template <typename T>
void ormtr_launch(const OrmtrWs<T>& w, int nbatch, int nmax, hipStream_t st) {
    const int nref = nmax - 1;
    if (nref <= 0) return;
    const int nblk = (nref + 63) / 64;
    const int tiles = (nmax + 63) / 64;
    const int nsplit = (nmax + ORMTR_CHUNK - 1) / ORMTR_CHUNK;
    // Gram matrices and T factors of all blocks up front (independent)
    VtvProb<T> pg;
    pg.A = w.A; pg.ns = w.ns; pg.Gpart = w.Gpart; pg.sG = w.sG; pg.nsplit = nsplit;
    hipLaunchKernelGGL((gemm_mfma_kernel<T, VtvProb<T>>), dim3(nblk, nsplit, nbatch), dim3(256), 0, st, pg);
    hipLaunchKernelGGL(ormtr_tfactor_kernel<T>, dim3(nblk, 1, nbatch), dim3(256), 0, st, w, nsplit);
    VtProb<T> pv;
    pv.A = w.A; pv.ns = w.ns; pv.Tm = w.Tm; pv.sT = w.sT; pv.VT = w.VT; pv.sVT = w.sVT; pv.nmax = w.nmax;
    hipLaunchKernelGGL((gemm_mfma_kernel<T, VtProb<T>>), dim3(tiles, nblk, nbatch), dim3(256), 0, st, pv);
    const int npair = nblk / 2;
    if (npair > 0) {
        // the Gram partials are consumed by the T factors: their buffer
        // takes the C_k partials
        CpairProb<T> pc;
        pc.A = w.A; pc.ns = w.ns; pc.VT = w.VT; pc.sVT = w.sVT; pc.Cpart = w.Gpart; pc.sCp = w.sG;
        pc.nmax = w.nmax; pc.nblk = nblk; pc.nsplit = nsplit;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, CpairProb<T>>), dim3(npair, nsplit, nbatch), dim3(256), 0, st, pc);
        hipLaunchKernelGGL(ormtr_cpair_sum_kernel<T>, dim3(npair, 1, nbatch), dim3(256), 0, st, w, nblk, nsplit);
    }
    // pairs (k, k+1) from the last block down, then block 0 alone if left
    // (64 x 128 tiles measured slower for V^T X: 53 vs 47 us per block at
    // n = 6000; 32-deep K slabs too, 48.5 vs 45.5 us; 128 x 128 tiles for the
    // K = 64 update, 94 vs 83 us per block)
    int blk = nblk - 1;
    for (; blk >= 1; blk -= 2) {
        const int b0 = (blk - 1) * 64;  // block k of the pair
        const int p = (nblk - 1 - blk) / 2;
        VtxProb<T, 64, 128> px;
        px.A = w.A; px.X = w.X; px.ns = w.ns; px.b0 = b0; px.Ypart = w.Ypart; px.sYp = w.sYp; px.nmax = w.nmax;
        px.tiles_n = tiles;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, VtxProb<T, 64, 128>>), dim3(2 * tiles, nsplit, nbatch), dim3(256), 0,
                           st, px);
        hipLaunchKernelGGL(ormtr_ysum_kernel<T>, dim3((128 * nmax + 255) / 256, 1, nbatch), dim3(256), 0, st, w, b0,
                           128);
        hipLaunchKernelGGL(ormtr_pair_fix_kernel<T>, dim3((nmax + ORMTR_FIX_COLS - 1) / ORMTR_FIX_COLS, 1, nbatch),
                           dim3(256), 0, st, w, b0, p);
        VyProb<T, 64, 128> py;
        py.X = w.X; py.ns = w.ns; py.b0 = b0; py.VT = w.VT; py.sVT = w.sVT; py.nmax = w.nmax; py.Y = w.Y; py.sY = w.sY;
        py.tiles_n = tiles;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, VyProb<T, 64, 128>>), dim3(tiles * tiles, 1, nbatch), dim3(256), 0, st,
                           py);
    }
    if (blk == 0) {
        VtxProb<T, 64> px;
        px.A = w.A; px.X = w.X; px.ns = w.ns; px.b0 = 0; px.Ypart = w.Ypart; px.sYp = w.sYp; px.nmax = w.nmax;
        px.tiles_n = tiles;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, VtxProb<T, 64>>), dim3(tiles, nsplit, nbatch), dim3(256), 0, st, px);
        hipLaunchKernelGGL(ormtr_ysum_kernel<T>, dim3((64 * nmax + 255) / 256, 1, nbatch), dim3(256), 0, st, w, 0, 64);
        VyProb<T, 64> py;
        py.X = w.X; py.ns = w.ns; py.b0 = 0; py.VT = w.VT; py.sVT = w.sVT; py.nmax = w.nmax; py.Y = w.Y; py.sY = w.sY;
        py.tiles_n = tiles;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, VyProb<T, 64>>), dim3(tiles * tiles, 1, nbatch), dim3(256), 0, st, py);
    }
}

template void ormtr_launch<double>(const OrmtrWs<double>&, int, int, hipStream_t);
template void ormtr_launch<float>(const OrmtrWs<float>&, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// generic batched GEMM entry used by the refinement and gradient stages
// ---------------------------------------------------------------------------
template <typename T, bool TA, bool TB, int TS>
static void gemm_gen_launch_ts(hipStream_t st, const int* ns, int nmax, int nbatch, const T* A, int lda,
                               long long sA, const T* B, int ldb, long long sB, T* C, int ldc, long long sC,
                               T alpha, T beta, bool lower_only, const int* skip, const T* Cin, int ldcin,
                               long long sCin, const GemmSecond<T>* second) {
    GemmGeneral<T, TA, TB, TS> p;
    p.A = A; p.lda = lda; p.sA = sA; p.B = B; p.ldb = ldb; p.sB = sB; p.C = C; p.ldc = ldc; p.sC = sC;
    p.Cin = Cin; p.ldcin = ldcin; p.sCin = sCin;
    int nz = nbatch;
    if (second) {
        p.B2 = second->B; p.ldb2 = second->ldb; p.sB2 = second->sB;
        p.C2 = second->C; p.ldc2 = second->ldc; p.sC2 = second->sC;
        nz = 2 * nbatch;
    }
    p.ns = ns; p.M = p.N = p.K = nmax; p.alpha = alpha; p.beta = beta;
    p.lower_only = lower_only ? 1 : 0;
    p.skip = skip;
    const int t = (nmax + TS - 1) / TS;
    p.tiles_n = t;
    const int grid = lower_only ? t * (t + 1) / 2 : t * t;
    if constexpr (TS == 128) {
        typedef Gemm128Shape<T> S;
        hipLaunchKernelGGL((gemm_mfma_kernel<T, GemmGeneral<T, TA, TB, TS>, TS, TS, S::BK, S::WM, S::WN>),
                           dim3(grid, 1, nz), dim3(64 * S::WM * S::WN), 0, st, p);
    } else {
        hipLaunchKernelGGL((gemm_mfma_kernel<T, GemmGeneral<T, TA, TB, TS>, TS, TS>), dim3(grid, 1, nz),
                           dim3(256), 0, st, p);
    }
}

thread_local int g_gemm_tile = 0;

// 128x128 tiles for large matrices; batches of small ones keep 64x64 (less
// padding waste at the ragged edges); the autotuner's choice when set
template <typename T, bool TA, bool TB>
static void gemm_gen_launch(hipStream_t st, const int* ns, int nmax, int nbatch, const T* A, int lda,
                            long long sA, const T* B, int ldb, long long sB, T* C, int ldc, long long sC,
                            T alpha, T beta, bool lower_only, const int* skip, const T* Cin, int ldcin,
                            long long sCin, const GemmSecond<T>* second = nullptr) {
    if (g_gemm_tile == 128 || (g_gemm_tile == 0 && nmax >= GEMM_TS128_MIN_ORDER))
        gemm_gen_launch_ts<T, TA, TB, 128>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta,
                                           lower_only, skip, Cin, ldcin, sCin, second);
    else
        gemm_gen_launch_ts<T, TA, TB, 64>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta,
                                          lower_only, skip, Cin, ldcin, sCin, second);
}

template <typename T>
void gemm_batched(hipStream_t st, bool ta, bool tb, const int* ns, int nmax, int nbatch, const T* A,
                  int lda, long long sA, const T* B, int ldb, long long sB, T* C, int ldc, long long sC,
                  T alpha, T beta, bool lower_only, const int* skip, const T* Cin, int ldcin, long long sCin) {
    if (!ta && !tb) gemm_gen_launch<T, false, false>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, Cin, ldcin, sCin);
    else if (ta && !tb) gemm_gen_launch<T, true, false>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, Cin, ldcin, sCin);
    else if (!ta && tb) gemm_gen_launch<T, false, true>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, Cin, ldcin, sCin);
    else gemm_gen_launch<T, true, true>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, Cin, ldcin, sCin);
}

// C = alpha op(A) op(B) + beta C and C2 = alpha op(A) op(B2) + beta C2 in one
// launch (grid.z = 2 nbatch, at most 65535)
template <typename T>
void gemm_batched_pair(hipStream_t st, bool ta, bool tb, const int* ns, int nmax, int nbatch, const T* A, int lda,
                       long long sA, const T* B, int ldb, long long sB, T* C, int ldc, long long sC,
                       const GemmSecond<T>& second, T alpha, T beta, bool lower_only, const int* skip) {
    if (2 * (long long)nbatch > 65535) {
        gemm_batched<T>(st, ta, tb, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only,
                        skip);
        gemm_batched<T>(st, ta, tb, ns, nmax, nbatch, A, lda, sA, second.B, second.ldb, second.sB, second.C,
                        second.ldc, second.sC, alpha, beta, lower_only, skip);
        return;
    }
    const GemmSecond<T>* s2 = &second;
    if (!ta && !tb) gemm_gen_launch<T, false, false>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, nullptr, 0, 0, s2);
    else if (ta && !tb) gemm_gen_launch<T, true, false>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, nullptr, 0, 0, s2);
    else if (!ta && tb) gemm_gen_launch<T, false, true>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, nullptr, 0, 0, s2);
    else gemm_gen_launch<T, true, true>(st, ns, nmax, nbatch, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, lower_only, skip, nullptr, 0, 0, s2);
}
template void gemm_batched_pair<double>(hipStream_t, bool, bool, const int*, int, int, const double*, int, long long,
                                        const double*, int, long long, double*, int, long long,
                                        const GemmSecond<double>&, double, double, bool, const int*);

template void gemm_batched<double>(hipStream_t, bool, bool, const int*, int, int, const double*, int, long long,
                                   const double*, int, long long, double*, int, long long, double, double, bool,
                                   const int*, const double*, int, long long);
template void gemm_batched<float>(hipStream_t, bool, bool, const int*, int, int, const float*, int, long long,
                                   const float*, int, long long, float*, int, long long, float, float, bool,
                                   const int*, const float*, int, long long);
