// Tiled matrix-core (MFMA) GEMM core shared by every dense contraction of the
// MBD path: the symmetric rank-2k trailing update of the Householder
// reduction, the compact-WY back-transform, the divide-and-conquer merges,
// Q^{-1/2} = X diag(lam^{-1/2}) X^T and the Ogita-Aishima refinement products.
//
// A workgroup of WM x WN wavefronts computes a BM x BN tile of C (default 64x64
// with 2x2 wavefronts), each wavefront owning a block of the 16x16x4 MFMA
// (v_mfma_f64_16x16x4f64 or v_mfma_f32_16x16x4f32, FP32 accumulation for
// FP32).  K is staged through LDS in slabs of BK with register prefetch of the
// next slab.  The problem object P supplies the tile map, element loaders and
// the epilogue, so masked Householder vectors, index-mapped eigenvector
// columns, batch strides and triangle-only tile sets need no copies.
//
// A problem may also define EPI_VEC = true for a read-modify-write epilogue
// on 16-byte column segments: its C tile is requested before the K loop
// through
//   Vec16<T>::v epi_load(const GemmTile&, int m, int n)   rows m .. m+RPL-1 of column n
// and, once the accumulators have been transposed through LDS so that every
// thread holds RPL = 16/sizeof(T) consecutive rows of one column, written by
//   void epi_store(const GemmTile&, int m, int n, Vec16<T>::v acc, Vec16<T>::v cin)
// (m, n in the problem's tile coordinates; m is a multiple of RPL).
#pragma once
#include <type_traits>
#include "mbd_internal.h"

template <typename T> struct mfma4;
template <> struct mfma4<double> { typedef double v __attribute__((ext_vector_type(4))); };
template <> struct mfma4<float> { typedef float v __attribute__((ext_vector_type(4))); };

// Row of the 16x16 result held by (lane, register r); the column is lane & 15.
// Measured on gfx950: the f32 form packs 4 consecutive rows per lane group,
// the f64 form interleaves them with stride 4.
template <typename T> struct mfma_rows;
template <> struct mfma_rows<double> {
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct mfma_rows<float> {
    static __device__ __forceinline__ int row(int lane, int r) { return ((lane >> 4) << 2) + r; }
};

__device__ __forceinline__ mfma4<double>::v mfma16x16x4(double a, double b, mfma4<double>::v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mfma4<float>::v mfma16x16x4(float a, float b, mfma4<float>::v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

#define GEMM_BM 64
#define GEMM_BN 64
#define GEMM_BK 16
#define GEMM_PAD 4

template <class P, class = void> struct gemm_epi_vec : std::false_type {};
template <class P>
struct gemm_epi_vec<P, std::void_t<decltype(P::EPI_VEC)>> : std::integral_constant<bool, P::EPI_VEC> {};

template <class P, class = void> struct gemm_k_uniform : std::false_type {};
template <class P>
struct gemm_k_uniform<P, std::void_t<decltype(P::K_UNIFORM)>> : std::integral_constant<bool, P::K_UNIFORM> {};

// Tile descriptor returned by P::tile()
struct GemmTile {
    int batch, m0, n0, K;
    int o, k;    // problem-specific offsets (e.g. merge origin and order)
    int e0, e1;  // further problem-specific values
};

// BM x BN tile per workgroup of WM x WN wavefronts, each owning a
// (BM/WM) x (BN/WN) block of 16x16 MFMA tiles; K staged in LDS slabs of BK.
template <typename T, class P, int BM = GEMM_BM, int BN = GEMM_BN, int BK = GEMM_BK, int WM = 2, int WN = 2>
__global__ __launch_bounds__(64 * WM * WN) void gemm_mfma_kernel(P p) {
    constexpr int NT = 64 * WM * WN;
    static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "wave tiles are multiples of 16");
    constexpr int MI = BM / WM / 16, NJ = BN / WN / 16;   // 16x16 blocks per wave in m and n
    constexpr int LA = BK * BM / NT, LB = BK * BN / NT;
    static_assert(LA * NT == BK * BM && LB * NT == BK * BN, "slab loads divide evenly");
    constexpr bool EV = gemm_epi_vec<P>::value;
    constexpr int RPL = 16 / (int)sizeof(T);
    constexpr int ELD = BM + RPL;  // column stride of the transposed C tile
    constexpr int STAGE = 2 * BK * (BM + GEMM_PAD) + 2 * BK * (BN + GEMM_PAD);
    constexpr int LDSN = EV && BN * ELD > STAGE ? BN * ELD : STAGE;
    // K slabs of A and B; with EV the same space later holds the C tile
    __shared__ __align__(16) T lds[LDSN];
    T(*As)[BK][BM + GEMM_PAD] = reinterpret_cast<T(*)[BK][BM + GEMM_PAD]>(lds);
    T(*Bs)[BK][BN + GEMM_PAD] = reinterpret_cast<T(*)[BK][BN + GEMM_PAD]>(lds + 2 * BK * (BM + GEMM_PAD));
    GemmTile t;
    if (!p.tile(blockIdx.x, blockIdx.y, blockIdx.z, t)) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    typedef typename Vec16<T>::v VT;
    constexpr int CPC = BM / RPL;                // vectors per tile column
    constexpr int NV = EV ? BM * BN / (NT * RPL) : 1;  // vectors per thread
    static_assert(!EV || NV * NT * RPL == BM * BN, "the C tile divides into 16-byte vectors");
    VT cin[NV];
    if constexpr (EV) {
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int idx = tid + v * NT;
            cin[v] = p.epi_load(t, t.m0 + (idx % CPC) * RPL, t.n0 + idx / CPC);
        }
    }

    typename mfma4<T>::v acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) acc[i][j] = typename mfma4<T>::v{0, 0, 0, 0};

    T ra[LA], rb[LB];
    // along a contiguous dimension of 64 or more, a wavefront's 64 lanes share
    // one k; a problem whose loader gathers through a k-indexed table marks it
    // wave-uniform (K_UNIFORM), so the gather goes through the scalar unit
    // (for plain operands the scalar address arithmetic measured slower)
    constexpr bool KU = gemm_k_uniform<P>::value;
    auto a_index = [&](int ii, int& m, int& k) {
        if (P::A_M_CONTIG) {
            m = tid % BM;
            k = tid / BM + (NT / BM) * ii;
            if constexpr (KU && BM % 64 == 0) k = __builtin_amdgcn_readfirstlane(k);
        } else { k = tid % BK; m = tid / BK + (NT / BK) * ii; }
    };
    auto b_index = [&](int ii, int& nn, int& k) {
        if (P::B_N_CONTIG) {
            nn = tid % BN;
            k = tid / BN + (NT / BN) * ii;
            if constexpr (KU && BN % 64 == 0) k = __builtin_amdgcn_readfirstlane(k);
        } else { k = tid % BK; nn = tid / BK + (NT / BK) * ii; }
    };
    auto gload = [&](int k0) {
#pragma unroll
        for (int ii = 0; ii < LA; ii++) {
            int m, k;
            a_index(ii, m, k);
            ra[ii] = p.a(t, t.m0 + m, k0 + k);
        }
#pragma unroll
        for (int ii = 0; ii < LB; ii++) {
            int nn, k;
            b_index(ii, nn, k);
            rb[ii] = p.b(t, k0 + k, t.n0 + nn);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int ii = 0; ii < LA; ii++) {
            int m, k;
            a_index(ii, m, k);
            As[buf][k][m] = ra[ii];
        }
#pragma unroll
        for (int ii = 0; ii < LB; ii++) {
            int nn, k;
            b_index(ii, nn, k);
            Bs[buf][k][nn] = rb[ii];
        }
    };

    const int nk = (t.K + BK - 1) / BK;
    if (nk > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < nk; kt++) {
            const int buf = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                T af[MI], bf[NJ];
#pragma unroll
                for (int i = 0; i < MI; i++) af[i] = As[buf][kk + (lane >> 4)][wm * (BM / WM) + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < NJ; j++) bf[j] = Bs[buf][kk + (lane >> 4)][wn * (BN / WN) + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < MI; i++)
#pragma unroll
                    for (int j = 0; j < NJ; j++) acc[i][j] = mfma16x16x4(af[i], bf[j], acc[i][j]);
            }
            if (kt + 1 < nk) sstore(buf ^ 1);
            __syncthreads();
        }
    }
    if constexpr (EV) {
        // the K loop ended on a barrier, so the staging space is free: write
        // the accumulators column-major, then read them back as 16-byte runs
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                const int col = wn * (BN / WN) + j * 16 + (lane & 15);
                if constexpr (sizeof(T) == 4) {
                    // FP32 layout: the lane's 4 values are consecutive rows
                    const int row = wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
                    *reinterpret_cast<VT*>(&lds[col * ELD + row]) = acc[i][j];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; r++)
                        lds[col * ELD + wm * (BM / WM) + i * 16 + mfma_rows<T>::row(lane, r)] = acc[i][j][r];
                }
            }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int idx = tid + v * NT;
            const int m = (idx % CPC) * RPL, c = idx / CPC;
            p.epi_store(t, t.m0 + m, t.n0 + c, *reinterpret_cast<const VT*>(&lds[c * ELD + m]), cin[v]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
            for (int j = 0; j < NJ; j++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    int row = t.m0 + wm * (BM / WM) + i * 16 + mfma_rows<T>::row(lane, r);
                    int col = t.n0 + wn * (BN / WN) + j * 16 + (lane & 15);
                    p.store(t, row, col, acc[i][j][r]);
                }
    }
}

// Split-FP16 variant for FP32 problems: C = op(A) op(B) through three FP16
// MFMA products.  Each operand value y, first multiplied by the problem's
// power of two (a_scale(t, m) for A's row m, b_scale(t, n) for B's column n,
// chosen so that |y| < 2^15), is split as y = yh + yl with yh = fp16(y) and
// yl = fp16(y - yh); the product is taken as Ah Bh + Ah Bl + Al Bh with FP32
// accumulation (v_mfma_f32_16x16x32_f16).  The parts keep about 22 of FP32's
// 24 bits and the dropped Al Bl term is of the same order, so the result
// matches an FP32 product to within its own accumulation error.  p.store
// receives the scaled accumulator and undoes the scaling.
//
// B is read by p.b4(t, k, n): the values at k .. k+3 of column n (k a
// multiple of 4), from a clamped address; p.b_keep(t, k, n) says which of
// them count.  The masking happens when the slab is written to LDS, after
// the previous slab's MFMAs, so the loads stay in flight meanwhile.
//
// TS x TS tiles, 2 x 2 wavefronts; thread (r, kq) stages row m0 + r of A and
// column n0 + r of B over KPT consecutive k of each 32-deep slab, as 16-byte
// rows of k-contiguous FP16 values in LDS (double buffered), so that each
// MFMA fragment (lane l: rows l % 16, k = 8 (l / 16) .. + 7) is one LDS read.
typedef _Float16 gemm_half8 __attribute__((ext_vector_type(8)));
typedef float gemm_f32x4 __attribute__((ext_vector_type(4)));

template <class P, int TS>
__global__ __launch_bounds__(256) void gemm_f16x3_kernel(P p) {
    constexpr int BK = 32;
    constexpr int WT = TS / 2;
    constexpr int MI = WT / 16, NJ = WT / 16;
    constexpr int LDK = BK + 8;         // halfs per LDS row: 80 bytes, 16-byte aligned
    constexpr int KPT = BK * TS / 256;  // k values per thread and operand in a slab
    static_assert(KPT % 8 == 0 && TS * (BK / KPT) == 256, "whole 16-byte LDS row pieces per thread");
    constexpr bool KU = gemm_k_uniform<P>::value;
    __shared__ __align__(16) _Float16 lds[2][4][TS * LDK];  // [buffer][Ah, Al, Bh, Bl]
    GemmTile t;
    if (!p.tile(blockIdx.x, blockIdx.y, blockIdx.z, t)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int rr = tid % TS, kq = (tid / TS) * KPT;  // kq is wave-uniform
    const int mr = t.m0 + rr, nc = t.n0 + rr;
    const float as = p.a_scale(t, mr), bs = p.b_scale(t, nc);
    float xa[KPT], fa[KPT];
    auto gload = [&](int k0) {
#pragma unroll
        for (int e = 0; e < KPT; e++) {
            int k = k0 + kq + e;
            if constexpr (KU) k = __builtin_amdgcn_readfirstlane(k);
            xa[e] = p.a(t, mr, k);
        }
#pragma unroll
        for (int e = 0; e < KPT; e += 4) {
            const gemm_f32x4 v = p.b4(t, k0 + kq + e, nc);
            fa[e] = v[0]; fa[e + 1] = v[1]; fa[e + 2] = v[2]; fa[e + 3] = v[3];
        }
    };
    auto sstore = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < KPT / 8; q++) {
            gemm_half8 ah, al, bh, bl;
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const float x = xa[8 * q + e] * as;
                const float y = p.b_keep(t, k0 + kq + 8 * q + e, nc) ? fa[8 * q + e] * bs : 0.0f;
                const _Float16 h = (_Float16)x, g = (_Float16)y;
                ah[e] = h; al[e] = (_Float16)(x - (float)h);
                bh[e] = g; bl[e] = (_Float16)(y - (float)g);
            }
            const int off = rr * LDK + kq + 8 * q;
            *reinterpret_cast<gemm_half8*>(&lds[buf][0][off]) = ah;
            *reinterpret_cast<gemm_half8*>(&lds[buf][1][off]) = al;
            *reinterpret_cast<gemm_half8*>(&lds[buf][2][off]) = bh;
            *reinterpret_cast<gemm_half8*>(&lds[buf][3][off]) = bl;
        }
    };
    gemm_f32x4 acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) acc[i][j] = gemm_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int fo = (lane & 15) * LDK + 8 * (lane >> 4);
    const int nk = (t.K + BK - 1) / BK;
    if (nk > 0) {
        gload(0);
        sstore(0, 0);
        __syncthreads();
        for (int kt = 0; kt < nk; kt++) {
            const int buf = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * BK);
            gemm_half8 ah[MI], al[MI], bh[NJ], bl[NJ];
#pragma unroll
            for (int i = 0; i < MI; i++) {
                const int r = (wm * WT + 16 * i) * LDK + fo;
                ah[i] = *reinterpret_cast<const gemm_half8*>(&lds[buf][0][r]);
                al[i] = *reinterpret_cast<const gemm_half8*>(&lds[buf][1][r]);
            }
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                const int r = (wn * WT + 16 * j) * LDK + fo;
                bh[j] = *reinterpret_cast<const gemm_half8*>(&lds[buf][2][r]);
                bl[j] = *reinterpret_cast<const gemm_half8*>(&lds[buf][3][r]);
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
    }
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                p.store(t, t.m0 + wm * WT + 16 * i + 4 * (lane >> 4) + r, t.n0 + wn * WT + 16 * j + (lane & 15),
                        acc[i][j][r]);
}

// Launch shape of the 128 x 128 tile per type, measured on gfx950 at order
// 6000: FP64 with 2 x 4 wavefronts and 8-deep K slabs (58 vs 50 TFLOP/s for
// 64 x 64 tiles), FP32 with 4 x 4 wavefronts and 16-deep slabs (99 vs 88).
// Large problems take these tiles: twice the flops per byte staged from L2.
#define GEMM_TS128_MIN_ORDER 2048
template <typename T> struct Gemm128Shape;
template <> struct Gemm128Shape<double> { static constexpr int BK = 8, WM = 2, WN = 4; };
template <> struct Gemm128Shape<float> { static constexpr int BK = 16, WM = 4, WN = 4; };

// Lower-triangle tile enumeration: linear index -> (ti, tj) with ti >= tj.
__device__ __forceinline__ void lower_tile(int lin, int& ti, int& tj) {
    int r = (int)((sqrtf(8.0f * (float)lin + 1.0f) - 1.0f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= lin) r++;
    while (r * (r + 1) / 2 > lin) r--;
    ti = r;
    tj = lin - r * (r + 1) / 2;
}

// XCD-aware tile order.  The 8 XCDs of the chip take workgroups round robin
// (workgroup bx runs on XCD bx mod 8) and each has its own L2, so workgroup
// bx = x + 8k is given the k-th tile of a contiguous share x of a banded
// order: bands of GEMM_BAND tile rows walked column by column.  The tiles an
// XCD runs at once then share A panels (same band) and B panels (same
// column) in its L2.  Any grid size works: the map is a bijection.
#define GEMM_NXCD 8
#define GEMM_BAND 8
__device__ __forceinline__ int xcd_virtual(int bx, int G) {
    const int x = bx % GEMM_NXCD, k = bx / GEMM_NXCD;
    const int q = G / GEMM_NXCD, r = G % GEMM_NXCD;
    return x * q + min(x, r) + k;
}
// full tm x tn grid
__device__ __forceinline__ void band_tile(int v, int tm, int tn, int& ti, int& tj) {
    const int band = v / (GEMM_BAND * tn);
    const int idx = v - band * GEMM_BAND * tn;
    const int rows = min(GEMM_BAND, tm - band * GEMM_BAND);
    ti = band * GEMM_BAND + idx % rows;
    tj = idx / rows;
}
// lower triangle (ti >= tj) of a t x t grid: band b holds rows r0 = b BAND ..
// r0 + rows - 1, first the r0 x rows rectangle left of the diagonal block,
// column by column, then the diagonal block's lower triangle, column by column
__device__ __forceinline__ void band_lower_tile(int v, int t, int& ti, int& tj) {
    int r0 = 0, rows = min(GEMM_BAND, t);
    for (;;) {
        const int cnt = r0 * rows + rows * (rows + 1) / 2;
        if (v < cnt || r0 + rows >= t) break;
        v -= cnt;
        r0 += rows;
        rows = min(GEMM_BAND, t - r0);
    }
    if (v < r0 * rows) {
        ti = r0 + v % rows;
        tj = v / rows;
        return;
    }
    v -= r0 * rows;
    int c = 0;
    while (c < rows - 1 && v >= rows - c) { v -= rows - c; c++; }
    tj = r0 + c;
    ti = r0 + c + v;
}

// General batched C = alpha op(A) op(B) + beta C over matrices of order ns[b]
// (M, N, K derived from ns through the m/n/k multipliers and offsets), in
// TS x TS output tiles.
template <typename T, bool TA, bool TB, int TS = GEMM_BM>
struct GemmGeneral {
    static constexpr bool A_M_CONTIG = !TA;
    static constexpr bool B_N_CONTIG = TB;
    const T* A; int lda; long long sA;
    const T* B; int ldb; long long sB;
    T* C; int ldc; long long sC;
    const T* Cin; int ldcin; long long sCin;  // beta term read from here (nullptr: from C)
    const int* ns;       // per-matrix order, or nullptr => fixed M,N,K
    int M, N, K;         // used when ns == nullptr
    T alpha, beta;
    int lower_only;      // only tiles (and elements) with row >= col
    int tiles_n;         // tiles along N (grid.x = tiles_m * tiles_n, or lower count)
    const int* skip;     // optional per-matrix flag: nonzero skips the matrix
    // Optional second product with the same A, orders and scaling (B2 set:
    // grid.z = 2 nbatch, odd z computes C2 = alpha op(A) op(B2) + beta C2).
    // Two products in one launch leave fewer partly filled rounds of tiles.
    const T* B2 = nullptr; int ldb2 = 0; long long sB2 = 0;
    T* C2 = nullptr; int ldc2 = 0; long long sC2 = 0;
    // the orders travel in the tile (t.o = M, t.k = N, t.K = K), read once;
    // t.e1 selects the product
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        const int b = B2 ? (bz >> 1) : bz;
        t.batch = b;
        t.e1 = B2 ? (bz & 1) : 0;
        if (skip && skip[b]) return false;
        const int Mb = ns ? ns[b] : M, Nb = ns ? ns[b] : N, Kb = ns ? ns[b] : K;
        int ti, tj;
        const int v = xcd_virtual(bx, gridDim.x);
        if (lower_only) band_lower_tile(v, tiles_n, ti, tj);
        else band_tile(v, tiles_n, tiles_n, ti, tj);
        t.m0 = ti * TS; t.n0 = tj * TS; t.K = Kb;
        t.o = Mb; t.k = Nb;
        return t.m0 < Mb && t.n0 < Nb;
    }
    __device__ T a(const GemmTile& t, int m, int k) const {
        if (m >= t.o || k >= t.K) return T(0);
        const T* Ab = A + (long long)t.batch * sA;
        return TA ? Ab[k + (long long)m * lda] : Ab[m + (long long)k * lda];
    }
    __device__ T b(const GemmTile& t, int k, int n) const {
        if (n >= t.k || k >= t.K) return T(0);
        const T* Bb = t.e1 ? B2 + (long long)t.batch * sB2 : B + (long long)t.batch * sB;
        const int ld = t.e1 ? ldb2 : ldb;
        return TB ? Bb[n + (long long)k * ld] : Bb[k + (long long)n * ld];
    }
    __device__ void store(const GemmTile& t, int m, int n, T v) const {
        if (m >= t.o || n >= t.k) return;
        if (lower_only && m < n) return;
        T* Cb = t.e1 ? C2 + (long long)t.batch * sC2 + m + (long long)n * ldc2
                     : C + (long long)t.batch * sC + m + (long long)n * ldc;
        if (beta == T(0)) { *Cb = alpha * v; return; }
        const T cin = Cin ? Cin[(long long)t.batch * sCin + m + (long long)n * ldcin] : *Cb;
        *Cb = alpha * v + beta * cin;
    }
};
