// Blocked Householder reduction of a real symmetric matrix to tridiagonal form
// (lower storage), the first stage of the diagonalisation Q = C Lambda C^T of
// eq:diagonalization (paper Sec. 2.1; Sec. 3.1 names the CPU libraries this
// replaces).
//
// Per panel of NBP columns, per column i (reflector H_i = I - tau v v^T with
// v(i+1) = 1 annihilating A(i+2:n, i)):
//   SYMV phase    one pass over the not-yet-updated lower trailing matrix
//                 A(i+1:n, i+1:n) in 64x64 tiles, each element read once and
//                 used for both y_R += A_RC v_C and y_C += A_RC^T v_R; also
//                 the panel products p = W^T v, s = V^T v and v^T A v, all
//                 added into per-column accumulators with float atomics.
//                 This is the bandwidth-bound BLAS-2 half of the reduction.
//   finish phase  per 64-row block: read the accumulated y, form
//                 w = tau (A v - V p - W s) - (tau/2)(w^T v) v, and apply the
//                 panel to the next column so its reflector can be built
//                 without another pass.
// After the panel: A(t0:n, t0:n) -= V W^T + W V^T on matrix cores (the BLAS-3
// half).  The accumulation order of the atomics varies, so results agree
// between runs to rounding, not bitwise.
//
// While the trailing matrix is large each phase is one launch per column.
// Below a trailing order (FP32: 4000) one launch per column does both: each
// workgroup finishes the previous column on the rows it touches, then runs
// this column's SYMV (the fused path below); the panel's last column gets a
// finish launch of its own.  A dependent launch costs about 2.8 us on gfx950
// even when empty, so the fused path saves that per column where its
// redundant row work is cheap; for large trailing orders that row work (about
// as many bytes as the tiles) costs more, and in FP64 its registers leave one
// wavefront per SIMD.  A cooperative kernel with a grid-wide barrier after
// each phase and a single launch that chained the phases through
// device-scope counters were both measured slower (a grid barrier or a
// release fence per workgroup costs more than a dependent launch).  Every
// work item carries a batch index, so one launch sequence serves a single
// large matrix and batches of uneven matrices alike.
#include <algorithm>
#include <cstdlib>
#include <string>

#include "gemm_mfma.h"
#include "mbd_internal.h"
#include "mbd_kernels.h"


// occupancy target of the SYMV kernel (waves per SIMD): the largest at which
// the compiler keeps the tile loop free of register spills
template <typename T> struct SymvWaves;
template <> struct SymvWaves<float> { static constexpr int value = 4; };
template <> struct SymvWaves<double> { static constexpr int value = 2; };

template <typename T>
struct Refl {
    T beta, tau, scale;
};

template <typename T>
__device__ __forceinline__ T refl_v(const T* col, int r, int s, int n, T scale) {
    if (r < s || r >= n) return T(0);
    return r == s ? T(1) : col[r] * scale;
}

// Reflector scalars from the updated column held in colbuf (LAPACK dlarfg
// convention: beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta).  The
// squared norm of x = col(i+2:n) was accumulated (atomically, by the phase
// that produced the column) into slot i % SYTRD_SLOTS of normacc; the column
// itself is in colbuf slot i & 1.
template <typename T>
__device__ __forceinline__ Refl<T> refl_scalars(const SytrdWs<T>& w, int b, int i, int n) {
    const T xn2 = w.normacc[(long long)b * SYTRD_SLOTS + i % SYTRD_SLOTS];
    const T alpha = w.colbuf[(long long)b * 2 * w.sC + (i & 1) * w.sC + i + 1];
    Refl<T> r;
    if (xn2 == T(0)) {
        r.tau = T(0); r.beta = alpha; r.scale = T(0);
    } else {
        const T nrm = sqrt(alpha * alpha + xn2);
        r.beta = alpha >= T(0) ? -nrm : nrm;
        r.tau = (r.beta - alpha) / r.beta;
        r.scale = T(1) / (alpha - r.beta);
    }
    return r;
}

// Work items of a launch are dispatched strip by strip (grid x = matrix +
// nbatch * item, y = strip), so in a batch the longest strips of every
// matrix (the first) start first rather than those of the last matrices
// last.
//
// Tiles per work item of the SYMV phase: the fewest that keep the launch
// within `target` workgroups.  Strip c (c = 1 .. nbt tiles long) splits into
// ceil(c / Kt) work items, nbt = q Kt + r strips in all, so a launch has
//   nbatch (Kt q (q + 1) / 2 + r (q + 1))
// workgroups; with the target at the number of workgroups the device holds
// at once the launch runs in a single round (a second, nearly empty round
// would cost another full memory latency).
#define SYTRD_KTMAX 16
__host__ __device__ __forceinline__ long long sytrd_items(int nbt, int nbatch, int kt) {
    const long long q = nbt / kt, r = nbt % kt;
    return ((long long)kt * q * (q + 1) / 2 + r * (q + 1)) * nbatch;
}
__host__ __device__ __forceinline__ int sytrd_kt(int nbt, int nbatch, int target) {
    for (int kt = 1; kt < SYTRD_KTMAX; kt++)
        if (sytrd_items(nbt, nbatch, kt) <= target) return kt;
    return SYTRD_KTMAX;
}

// The last columns of a matrix are reduced by one workgroup with the trailing
// block packed in LDS (sytrd_tail_kernel): M0 columns at most, the largest
// order whose packed lower triangle and two vectors fit in 160 KB.  The
// panel path stops at a panel boundary, tail_start, so that the trailing
// block it leaves has had every panel update applied.
template <typename T> struct SytrdTail;
template <> struct SytrdTail<float> { static constexpr int M0 = 256; };
template <> struct SytrdTail<double> { static constexpr int M0 = 192; };
template <typename T>
__host__ __device__ __forceinline__ int sytrd_tail_start(int n) {
    constexpr int M0 = SytrdTail<T>::M0;
    return n <= M0 ? 0 : (n - M0 + SYTRD_NBP - 1) / SYTRD_NBP * SYTRD_NBP;
}

// Accumulators of column i live in slot i % SYTRD_SLOTS.  To keep atomic
// contention low they are spread over copies: y and the panel products over
// SYTRD_YC copies chosen by column strip, v^T A v over SYTRD_VC copies chosen
// by workgroup; the finish phase adds the copies.
#define SYTRD_YC SYTRD_YCOPIES
#define SYTRD_VC SYTRD_VCOPIES
template <typename T>
__device__ __forceinline__ T* yacc_of(const SytrdWs<T>& w, int b, int i, int copy) {
    return w.yacc + (long long)b * w.sY + ((i % SYTRD_SLOTS) * SYTRD_YC + copy) * (long long)w.nmax;
}
template <typename T>
__device__ __forceinline__ T* sacc_of(const SytrdWs<T>& w, int b, int i, int copy) {
    return w.sacc + (long long)b * w.sS + ((i % SYTRD_SLOTS) * SYTRD_YC + copy) * (2 * SYTRD_NBP);
}
template <typename T>
__device__ __forceinline__ T* vacc_of(const SytrdWs<T>& w, int b, int i) {
    return w.vacc + (long long)b * (SYTRD_SLOTS * SYTRD_VC) + (i % SYTRD_SLOTS) * SYTRD_VC;
}

template <typename T>
__global__ __launch_bounds__(256) void sytrd_init_kernel(SytrdWs<T> w) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int R = blockIdx.x;
    const int nbk = (n + 63) >> 6;
    if (R >= nbk) return;
    const T* A = w.A.at(b);
    T* col = w.colbuf + (long long)b * 2 * w.sC;
    // every slot of the accumulators starts at zero
    for (int t = threadIdx.x; t < SYTRD_SLOTS * SYTRD_YC * 64; t += 256) {
        const int r = R * 64 + (t & 63);
        if (r < n) w.yacc[(long long)b * w.sY + (t >> 6) * (long long)w.nmax + r] = T(0);
    }
    if (R == 0) {
        for (int t = threadIdx.x; t < SYTRD_SLOTS * SYTRD_YC * 2 * SYTRD_NBP; t += 256) w.sacc[(long long)b * w.sS + t] = T(0);
        for (int t = threadIdx.x; t < SYTRD_SLOTS * SYTRD_VC; t += 256)
            w.vacc[(long long)b * (SYTRD_SLOTS * SYTRD_VC) + t] = T(0);
    }
    if (n == 1) {
        if (threadIdx.x == 0) w.d[(long long)b * w.sD] = A[0];
        return;
    }
    if (threadIdx.x >= 64) return;
    const int r = R * 64 + threadIdx.x;
    T x = r < n ? A[r] : T(0);
    if (r < n) col[r] = x;
    T q = (r >= 2 && r < n) ? x * x : T(0);
    q = wave_sum(q);
    if (threadIdx.x == 0) unsafeAtomicAdd(&w.normacc[(long long)b * SYTRD_SLOTS + 0], q);
}

// both norm slots to zero before the first column
template <typename T>
__global__ void sytrd_zero_norm_kernel(SytrdWs<T> w, int nbatch) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < SYTRD_SLOTS * nbatch) w.normacc[t] = T(0);
}

// ---------------------------------------------------------------------------
// SYMV work item: tiles R in [C + q Kt, C + (q+1) Kt) of column strip C.
// Wavefront wv streams the 16 columns c0 = 64 C + 16 wv ... c0 + 15.  Each
// lane loads 16 bytes of one column segment (RPL consecutive rows: 4 floats
// or 2 doubles), so one load instruction covers RPL columns x 64 rows and a
// tile takes 16 / RPL loads per lane.  The column buffer entries of the
// tile's rows come with the same batch of loads, and the next tile is
// requested before the current one is reduced, unconditionally (a tile past
// the chunk reads zeros through the out-of-range offset): the in-order load
// counter then never waits for more than the tile in use.  Row sums, column
// sums, the panel products and v^T A v are added into the column's
// accumulators with hardware float atomics, so the finish phase reads one
// value per row.
// ---------------------------------------------------------------------------
template <typename T, int NBP>
__device__ void symv_item(const SytrdWs<T>& w, int b, int n, int i, int j, int Kt, int C, int q,
                          const Refl<T>* rf_in) {
    constexpr int RPL = 16 / (int)sizeof(T);  // rows per lane per load
    constexpr int LPC = 64 / RPL;             // lanes per column segment
    constexpr int NI = 16 / RPL;              // loads per lane per tile
    typedef typename Vec16<T>::v VT;
    __shared__ T rpart[SYTRD_KTMAX][4][64];  // per-tile, per-wave row partials
    __shared__ T vrow[SYTRD_KTMAX][64];      // reflector entries of the tile rows
    __shared__ T red[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane / LPC, rq = lane % LPC;
    const int s = i + 1;
    const int b0 = s >> 6;
    const int nbk = (n + 63) >> 6;
    T* A = w.A.at(b);
    const long long ld = w.A.ld;
    const T* col = w.colbuf + (long long)b * 2 * w.sC + (i & 1) * w.sC;
    T* Vp = w.Vp + (long long)b * w.sP;
    T* Wp = w.Wp + (long long)b * w.sP;
    T* yacc = yacc_of(w, b, i, C % SYTRD_YC);
    const int ldp = w.ldp;
    const int Rb = C + q * Kt;
    const int Re = min(Rb + Kt, nbk);
    const int c0 = C * 64 + wv * 16;

    // the column buffer is padded to 64 nbk rows; the wave's strip holds
    // ncols columns of the matrix
    const __amdgpu_buffer_rsrc_t csrc = make_rsrc(col, (unsigned)(nbk * 64 * (int)sizeof(T)));
    const int ncols = max(0, min(16, n - c0));
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(A + (long long)c0 * ld, (unsigned)(ncols * ld * (long long)sizeof(T)));
    // reflector scalars and this lane's column entries are requested first,
    // so waiting for them never waits for a tile
    const Refl<T> rf = rf_in ? *rf_in : refl_scalars(w, b, i, n);
    unsigned coff[NI];
    bool cok[NI];
    T craw[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) {
        const int c = c0 + RPL * k + g;
        cok[k] = c >= s && c < n;
        coff[k] = (unsigned)((RPL * k + g) * ld * (long long)sizeof(T));
        craw[k] = buf_load<T>(csrc, cok[k] ? (unsigned)(c * (int)sizeof(T)) : OOB_OFFSET);
    }
    VT buf[NI + 1];  // tile column segments and the column buffer rows
    auto issue = [&](int R) {
        // past the chunk every offset lands at or beyond OOB_OFFSET
        const unsigned roff = R < Re ? (unsigned)((R * 64 + RPL * rq) * (int)sizeof(T)) : OOB_OFFSET;
#pragma unroll
        for (int k = 0; k < NI; k++) buf[k] = buf_load16<T>(rsrc, cok[k] ? coff[k] + roff : OOB_OFFSET);
        buf[NI] = buf_load16<T>(csrc, roff);
    };
    // the first work item of a strip also handles the rows of block C: it
    // stores v there (panel column j and matrix column i) and forms the panel
    // products W^T v and V^T v over those rows; its loads are unconditional
    // (rows clamped, results masked) and requested before the tile's
    const int rq0 = C * 64 + lane;
    const int rq0c = rq0 < n ? rq0 : n - 1;
    static_assert(NBP == 32, "eight panel columns per wave");
    T cq = T(0), di = T(0), pwl[8], pvl[8];
    if (q == 0) {
        cq = col[rq0c];
        if (C == b0) di = col[i];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int k = wv + 4 * t;
            pwl[t] = Wp[rq0c + (long long)k * ldp];
            pvl[t] = Vp[rq0c + (long long)k * ldp];
        }
    }
    issue(Rb);

    if (q == 0) {
        const bool rv = rq0 >= s && rq0 < n;
        const T vq = rv ? (rq0 == s ? T(1) : cq * rf.scale) : T(0);
        if (wv == 0 && rq0 < n) {
            Vp[rq0 + (long long)j * ldp] = vq;
            if (rq0 >= s) A[rq0 + (long long)i * ld] = vq;
        }
        // the 16 sums of a wave (columns k = wv + 4 t of W and of V) come out
        // of one multi-value butterfly, lane 4 u holding sum u
        T* sacc = sacc_of(w, b, i, C % SYTRD_YC);
        T pr[16];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const bool ok = rv && wv + 4 * t < j;
            pr[t] = ok ? pwl[t] * vq : T(0);
            pr[8 + t] = ok ? pvl[t] * vq : T(0);
        }
        const T ps = wave_sum16(pr);
        const int u = lane >> 2, k = wv + 4 * (u & 7);
        if ((lane & 3) == 0 && k < j) unsafeAtomicAdd(&sacc[(u >> 3) * NBP + k], ps);
    }

    T vc[NI], cacc[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) {
        const int c = c0 + RPL * k + g;
        vc[k] = cok[k] ? (c == s ? T(1) : craw[k] * rf.scale) : T(0);
        cacc[k] = T(0);
    }
    for (int R = Rb; R < Re; R++) {
        const int r0 = R * 64 + RPL * rq;
        T vr[RPL], rs[RPL];
#pragma unroll
        for (int e = 0; e < RPL; e++) {
            const int r = r0 + e;
            vr[e] = (r < s || r >= n) ? T(0) : (r == s ? T(1) : buf[NI][e] * rf.scale);
            rs[e] = T(0);
        }
#pragma unroll
        for (int k = 0; k < NI; k++) {
            const int c = c0 + RPL * k + g;
#pragma unroll
            for (int e = 0; e < RPL; e++) {
                const int r = r0 + e;
                // rows past n (padding) and, on the diagonal tile, above the
                // diagonal are not part of the lower trailing matrix
                const T x = (r < n && (R > C || r >= c)) ? buf[k][e] : T(0);
                rs[e] += x * vc[k];
                cacc[k] += (R > C || r != c) ? x * vr[e] : T(0);
            }
        }
        issue(R + 1);
        // row sums over the RPL column groups of the wave (lane bits 5, 4
        // for floats, bit 5 for doubles): lane (rq, g) ends with row RPL rq + g
        T rsum;
        if constexpr (RPL == 4) {
            rsum = pair_sum_b4(pair_sum_b5(rs[0], rs[2]), pair_sum_b5(rs[1], rs[3]));
        } else {
            rsum = pair_sum_b5(rs[0], rs[1]);
        }
        rpart[R - Rb][wv][RPL * rq + g] = rsum;
        if (wv == 0 && g == 0) {
#pragma unroll
            for (int e = 0; e < RPL; e++) vrow[R - Rb][RPL * rq + e] = vr[e];
        }
    }
    // column sums over the LPC row groups (lane bits below 6 - log2 RPL): lane
    // l ends with the sum of column index k = (l >> 2) mod NI of group g
    T vav = T(0);
#pragma unroll
    for (int k = 0; k < NI; k++) vav += vc[k] * cacc[k];
    T csum;
    if constexpr (NI == 4) {
        csum = quad_sum(pair_sum_b2(pair_sum_b3(cacc[0], cacc[2]), pair_sum_b3(cacc[1], cacc[3])));
    } else {
        const T u0 = pair_sum_b4(cacc[0], cacc[4]), u1 = pair_sum_b4(cacc[1], cacc[5]);
        const T u2 = pair_sum_b4(cacc[2], cacc[6]), u3 = pair_sum_b4(cacc[3], cacc[7]);
        csum = quad_sum(pair_sum_b2(pair_sum_b3(u0, u2), pair_sum_b3(u1, u3)));
    }
    {
        const int c = c0 + RPL * ((lane >> 2) % NI) + g;
        if ((lane & 3) == 0 && c >= s && c < n) unsafeAtomicAdd(&yacc[c], csum);
    }
    __syncthreads();
    for (int t = wv; t < Re - Rb; t += 4) {
        const T y = (rpart[t][0][lane] + rpart[t][1][lane]) + (rpart[t][2][lane] + rpart[t][3][lane]);
        const int r = (Rb + t) * 64 + lane;
        if (r >= s && r < n) {
            unsafeAtomicAdd(&yacc[r], y);
            vav += vrow[t][lane] * y;
        }
    }
    vav = block_sum256(vav, red);
    if (tid == 0) {
        unsafeAtomicAdd(vacc_of(w, b, i) + (C * 7 + q) % SYTRD_VC, vav);
        if (q == 0 && C == b0) {
            w.d[(long long)b * w.sD + i] = di;
            w.e[(long long)b * w.sD + i] = rf.beta;
            w.tau[(long long)b * w.sD + i] = rf.tau;
        }
    }
}

// ---------------------------------------------------------------------------
// finish work item: 64-row block R.  Reads y = A v, the panel products and
// v^T A v from the column's accumulators, forms w, applies the panel to the
// next column, and clears the other parity slot for the next column.
// ---------------------------------------------------------------------------
template <typename T, int NBP>
__device__ void finish_item(const SytrdWs<T>& w, int b, int n, int i, int j, int R) {
    static_assert(SYTRD_VC == 256, "four v^T A v copies per lane of wavefront 0");
    static_assert(2 * NBP <= 64, "panel products are reduced by one wavefront");
    static_assert(NBP % 4 == 0, "panel columns are split over 4 wavefronts");
    __shared__ T sps[2 * NBP];
    __shared__ T rr[3][4][64];
    const int s = i + 1;
    const int b0 = s >> 6;
    const int tid = threadIdx.x, lane = tid & 63, part = tid >> 6;
    const T* Vp = w.Vp + (long long)b * w.sP;
    T* Wp = w.Wp + (long long)b * w.sP;
    const int ldp = w.ldp;
    const T* A = w.A.at(b);
    const long long ld = w.A.ld;
    const int r = R * 64 + lane;
    const bool rv = (r >= s && r < n);

    // ---- independent loads, all unconditional (rows clamped into the
    // matrix, panel columns k >= j masked afterwards) so that they form one
    // round trip instead of a chain of branch-guarded load/wait pairs
    const int rc = r < n ? r : n - 1;
    const T tau = w.tau[(long long)b * w.sD + i];
    // wavefront 0 forms w and the next column: only it needs the panel
    // products, y at row r, v(r) and the column of A (a wave-uniform branch)
    const bool w0 = __builtin_amdgcn_readfirstlane(tid >> 6) == 0;
    T spc[SYTRD_YC], yrc[SYTRD_YC];
    T vr_l = T(0), acol_l = T(0), vq[4];
    if (w0) {
#pragma unroll
        for (int c = 0; c < SYTRD_YC; c++) {
            spc[c] = sacc_of(w, b, i, c)[tid & (2 * NBP - 1)];
            yrc[c] = yacc_of(w, b, i, c)[rc];
        }
#pragma unroll
        for (int c = 0; c < 4; c++) vq[c] = vacc_of(w, b, i)[lane + 64 * c];
        vr_l = Vp[rc + (long long)j * ldp];
        acol_l = A[rc + (long long)s * ld];
    } else {
#pragma unroll
        for (int c = 0; c < SYTRD_YC; c++) {
            spc[c] = T(0);
            yrc[c] = T(0);
        }
#pragma unroll
        for (int c = 0; c < 4; c++) vq[c] = T(0);
    }
    // the wave-uniform values at row s (the accumulator copies and the
    // wave's panel entries) come from one load, a value per lane, and are
    // broadcast from their lanes afterwards
    static_assert(SYTRD_YC + 2 * (NBP / 4) <= 64, "row-s values fit in a wavefront");
    T srow;
    {
        const int l = lane;
        const T* src;
        if (l < SYTRD_YC) src = yacc_of(w, b, i, l) + s;
        else if (l < SYTRD_YC + NBP / 4) src = Vp + s + (long long)(part + 4 * (l - SYTRD_YC)) * ldp;
        else if (l < SYTRD_YC + NBP / 2) src = Wp + s + (long long)(part + 4 * (l - SYTRD_YC - NBP / 4)) * ldp;
        else src = yacc_of(w, b, i, 0) + s;
        srow = *src;
    }
    T vr_k[NBP / 4], wr_k[NBP / 4];
#pragma unroll
    for (int t = 0; t < NBP / 4; t++) {
        const int k = part + 4 * t;
        vr_k[t] = Vp[rc + (long long)k * ldp];
        wr_k[t] = Wp[rc + (long long)k * ldp];
    }
    T sp = T(0), yr = T(0), ysv = T(0);
#pragma unroll
    for (int c = 0; c < SYTRD_YC; c++) {
        sp += spc[c];
        yr += yrc[c];
        ysv += lane_value(srow, c);
    }
    T vs_k[NBP / 4], ws_k[NBP / 4];
#pragma unroll
    for (int t = 0; t < NBP / 4; t++) {
        vs_k[t] = lane_value(srow, SYTRD_YC + t);
        ws_k[t] = lane_value(srow, SYTRD_YC + NBP / 4 + t);
    }
    if (!(tid < 2 * NBP && (tid % NBP) < j)) sp = T(0);
    if (!rv) yr = T(0);
#pragma unroll
    for (int t = 0; t < NBP / 4; t++) {
        const bool ok = part + 4 * t < j;
        vr_k[t] = (ok && rv) ? vr_k[t] : T(0);
        wr_k[t] = (ok && rv) ? wr_k[t] : T(0);
        vs_k[t] = ok ? vs_k[t] : T(0);
        ws_k[t] = ok ? ws_k[t] : T(0);
    }
    const T vr = rv ? vr_l : T(0);
    const T acol = rv ? acol_l : T(0);
    if (tid < 2 * NBP) sps[tid] = sp;
    // v^T A v is needed by wavefront 0 only (w at row r and at row s)
    const T vAv = wave_sum((vq[0] + vq[1]) + (vq[2] + vq[3]));
    __syncthreads();

    // clear the next column's slot for column i + 1 (its SYMV runs after
    // this kernel): rows of block R, and the scalars once per matrix
    for (int c = part; c < SYTRD_YC; c += 4)
        if (R * 64 + lane < n) yacc_of(w, b, i + 1, c)[R * 64 + lane] = T(0);
    if (R == b0) {
        for (int t = tid; t < SYTRD_YC * 2 * NBP; t += 256) sacc_of(w, b, i + 1, 0)[t] = T(0);
        vacc_of(w, b, i + 1)[tid] = T(0);
    }

    T pts = T(0);
    for (int k = 0; k < j; k++) pts += sps[k] * sps[NBP + k];
    const T wtv = tau * (vAv - T(2) * pts);
    // corr = V p + W s at row r and at row s, split over the wavefronts
    T cr = T(0), csp = T(0);
#pragma unroll
    for (int t = 0; t < NBP / 4; t++) {
        const int k = part + 4 * t;
        if (k < j) {
            cr += vr_k[t] * sps[k] + wr_k[t] * sps[NBP + k];
            csp += vs_k[t] * sps[k] + ws_k[t] * sps[NBP + k];
        }
    }
    rr[0][part][lane] = cr;
    rr[1][part][lane] = csp;
    __syncthreads();
    cr = (rr[0][0][lane] + rr[0][1][lane]) + (rr[0][2][lane] + rr[0][3][lane]);
    csp = (rr[1][0][0] + rr[1][1][0]) + (rr[1][2][0] + rr[1][3][0]);
    const T wr = rv ? tau * (yr - cr) - T(0.5) * tau * wtv * vr : T(0);
    if (part == 0 && r < n) Wp[r + (long long)j * ldp] = wr;
    const T ws = tau * (ysv - csp) - T(0.5) * tau * wtv;
    // apply the panel (columns 0..j) to column s, rows of block R
    T u = T(0);
    if (rv) {
#pragma unroll
        for (int t = 0; t < NBP / 4; t++) {
            const int k = part + 4 * t;
            if (k < j) u += vr_k[t] * ws_k[t] + wr_k[t] * vs_k[t];
        }
        if (part == 0) u += vr * ws + wr;
    }
    rr[2][part][lane] = u;
    __syncthreads();
    if (part == 0) {
        u = (rr[2][0][lane] + rr[2][1][lane]) + (rr[2][2][lane] + rr[2][3][lane]);
        T cval = T(0);
        if (rv) {
            cval = acol - u;
            w.colbuf[(long long)b * 2 * w.sC + (s & 1) * w.sC + r] = cval;
            if (s == n - 1) w.d[(long long)b * w.sD + n - 1] = cval;
        }
        T q2 = (r >= s + 2 && r < n) ? cval * cval : T(0);
        q2 = wave_sum(q2);
        if (lane == 0) unsafeAtomicAdd(&w.normacc[(long long)b * SYTRD_SLOTS + s % SYTRD_SLOTS], q2);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// tail: unblocked reduction of the trailing block A(k0:n, k0:n), m = n - k0
// <= M0, one workgroup of 1024 threads per matrix: thread tid of quarter q =
// tid / 256 works on one row r and on the columns c = q (mod 4), so that
// each SIMD holds four waves (the quarter's four wavefronts take the four
// 64-row blocks, in an order rotated by q).  The lower triangle is held packed by columns in
// LDS (column c holds rows c .. m-1).  Per column i, s = i + 1, with the
// panel path's reflector convention (beta = -sign(alpha) ||x||, tau =
// (beta - alpha) / beta, v(s) = 1, v(r) = x(r) / (alpha - beta)) for x =
// A(s:m-1, i), alpha = x(s):
//   1. y' = A x' over the trailing block for x' = x with x'(s) = 0, which
//      needs no reflector scalars, and with it the partial sums of x^T x
//      (r > s), x'^T A x' and x'^T A e_s;                        barrier
//   2. every thread forms beta, tau and scale = 1/(alpha - beta) from the
//      same sums; A v = scale y' + A e_s, v^T A v = scale^2 x'^T A x' +
//      2 scale x'^T A e_s + A(s,s), y = tau A v, w = y - (tau/2)(y^T v) v;
//                                                                 barrier
//   3. the rank-2 update A -= v w^T + w v^T of the lower triangle; barrier.
// Three barriers per column (none when tau = 0).  d, e, tau and the
// reflectors (stored in A below the diagonal) are written as the panel path
// writes them.
// ---------------------------------------------------------------------------
#define SYTRD_TAIL_THREADS 1024

template <typename T>
__global__ __launch_bounds__(SYTRD_TAIL_THREADS) void sytrd_tail_kernel(SytrdWs<T> w) {
    constexpr int M0 = SytrdTail<T>::M0;
    constexpr int Q = SYTRD_TAIL_THREADS / 256;
    constexpr int NW = SYTRD_TAIL_THREADS / 64;
    static_assert(M0 <= 256, "one row per thread of a quarter");
    __shared__ T L[M0 * (M0 + 1) / 2];
    __shared__ T vv[M0], ww[M0];
    __shared__ T yp[Q - 1][M0];   // SYMV partials of quarters 1 .. Q-1 (quarter 0 keeps its own)
    __shared__ T red[2][3][NW];   // per-wave partial sums, by column parity
    const int b = blockIdx.x;
    const int n = w.ns[b];
    const int k0 = sytrd_tail_start<T>(n);
    const int m = n - k0;
    if (m <= 0) return;
    T* A = w.A.at(b) + k0 + (long long)k0 * w.A.ld;
    const long long ld = w.A.ld;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
    // row of this thread: the four wavefronts of quarter q take the 64-row
    // blocks rotated by q, so that each SIMD (wavefront k of a workgroup
    // runs on SIMD k mod 4) holds one wavefront of every row block and the
    // triangular update (row r: about r/4 columns per quarter) is spread
    // evenly over the SIMDs
    const int r = ((((int)threadIdx.x >> 6) + q) & 3) * 64 + (int)(threadIdx.x & 63);
    const int wv = threadIdx.x >> 6;
    const bool rv = r < m;
    // start of packed column c
    auto cs = [m](int c) { return c * m - c * (c - 1) / 2; };

    // load the lower triangle, quarter q taking columns c = q (mod 4), 8
    // columns per round with the loads issued together from clamped (always
    // valid) addresses and the values masked afterwards
    constexpr int U = 8;
    for (int c0 = q; c0 < m; c0 += Q * U) {
        T t[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int c = min(c0 + Q * u, m - 1);
            const int rr = min(max(r, c), m - 1);
            t[u] = A[rr + (long long)c * ld];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int c = c0 + Q * u;
            if (c < m && rv && r >= c) L[cs(c) + r - c] = t[u];
        }
    }
    __syncthreads();

    const int csr = rv ? cs(r) : 0;
    T* d = w.d + (long long)b * w.sD + k0;
    T* e = w.e + (long long)b * w.sD + k0;
    T* tau_o = w.tau + (long long)b * w.sD + k0;
    for (int i = 0; i + 1 < m; i++) {
        const int s = i + 1, ci = cs(i), css = cs(s);
        const bool row = rv && r >= s;       // rows of the trailing block
        const T xr = (rv && r > s) ? L[ci + r - i] : T(0);   // x'(r)
        // 1. y'(r) partial over c = s + q, s + q + Q, ... (c > s: x'(s) = 0),
        // A(r, c) from column c while c <= r, then from column r; four
        // columns per step with their loads issued together
        T ys = T(0);
        if (row) {
            int c = s + q + (q == 0 ? Q : 0), csc = cs(c);
            const T* xc = L + ci - i;   // x'(c) = xc[c]
            T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
            for (; c + 3 * Q <= r; c += 4 * Q) {
                // cs(c + Q) - cs(c) = Q m - Q c - Q (Q - 1) / 2, falling by Q^2 per step
                const int d0 = Q * m - Q * c - Q * (Q - 1) / 2, d1 = d0 - Q * Q, d2 = d1 - Q * Q;
                const int a0 = csc + r - c, a1 = a0 + d0 - Q, a2 = a1 + d1 - Q, a3 = a2 + d2 - Q;
                s0 += L[a0] * xc[c];
                s1 += L[a1] * xc[c + Q];
                s2 += L[a2] * xc[c + 2 * Q];
                s3 += L[a3] * xc[c + 3 * Q];
                csc += 4 * d0 - 6 * Q * Q;
            }
            for (; c <= r; c += Q) {
                s0 += L[csc + r - c] * xc[c];
                csc += Q * m - Q * c - Q * (Q - 1) / 2;
            }
            for (; c + 3 * Q < m; c += 4 * Q) {
                const int a0 = csr + c - r;
                s0 += L[a0] * xc[c];
                s1 += L[a0 + Q] * xc[c + Q];
                s2 += L[a0 + 2 * Q] * xc[c + 2 * Q];
                s3 += L[a0 + 3 * Q] * xc[c + 3 * Q];
            }
            for (; c < m; c += Q) s0 += L[csr + c - r] * xc[c];
            ys = (s0 + s1) + (s2 + s3);
        }
        const T ars = row ? L[css + r - s] : T(0);   // A(r, s)
        {
            const T p0 = wave_sum(q == 0 ? xr * xr : T(0));
            const T p1 = wave_sum(xr * ys);
            const T p2 = wave_sum(q == 0 ? xr * ars : T(0));
            if ((threadIdx.x & 63) == 0) {
                red[i & 1][0][wv] = p0;
                red[i & 1][1][wv] = p1;
                red[i & 1][2][wv] = p2;
            }
        }
        if (q > 0 && rv) yp[q - 1][r] = ys;
        __syncthreads();
        // 2. reflector and w from the sums (the same order in every thread)
        T xn2 = T(0), xax = T(0), xae = T(0);
#pragma unroll
        for (int k = 0; k < NW; k++) {
            xn2 += red[i & 1][0][k];
            xax += red[i & 1][1][k];
            xae += red[i & 1][2][k];
        }
        const T alpha = L[ci + 1];
        T beta, tau, scale;
        if (xn2 == T(0)) {
            tau = T(0); beta = alpha; scale = T(0);
        } else {
            const T nrm = sqrt(alpha * alpha + xn2);
            beta = alpha >= T(0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scale = T(1) / (alpha - beta);
        }
        if (q == 0) {
            const T vr = (r == s) ? T(1) : xr * scale;
            if (row) A[r + (long long)i * ld] = vr;
            if (r == 0) {
                d[i] = L[ci];
                e[i] = beta;
                tau_o[i] = tau;
            }
            if (tau != T(0) && row) {
                const T yr = tau * (scale * (((ys + yp[0][r]) + yp[1][r]) + yp[2][r]) + ars);
                const T vav = scale * scale * xax + T(2) * scale * xae + L[css];
                const T ytv = tau * vav;
                vv[r] = vr;
                ww[r] = yr - T(0.5) * tau * ytv * vr;
            }
        }
        if (tau != T(0)) {
            __syncthreads();
            // 3. A(r, c) -= v(r) w(c) + w(r) v(c), c = s + q, ... <= r; four
            // columns per step, all loads before the stores
            if (row) {
                const T vr = vv[r], wr = ww[r];
                int c = s + q, csc = cs(c);
                for (; c + 3 * Q <= r; c += 4 * Q) {
                    const int d0 = Q * m - Q * c - Q * (Q - 1) / 2, d1 = d0 - Q * Q, d2 = d1 - Q * Q;
                    const int a0 = csc + r - c, a1 = a0 + d0 - Q, a2 = a1 + d1 - Q, a3 = a2 + d2 - Q;
                    const T t0 = L[a0], t1 = L[a1], t2 = L[a2], t3 = L[a3];
                    L[a0] = t0 - (vr * ww[c] + wr * vv[c]);
                    L[a1] = t1 - (vr * ww[c + Q] + wr * vv[c + Q]);
                    L[a2] = t2 - (vr * ww[c + 2 * Q] + wr * vv[c + 2 * Q]);
                    L[a3] = t3 - (vr * ww[c + 3 * Q] + wr * vv[c + 3 * Q]);
                    csc += 4 * d0 - 6 * Q * Q;
                }
                for (; c <= r; c += Q) {
                    L[csc + r - c] -= vr * ww[c] + wr * vv[c];
                    csc += Q * m - Q * c - Q * (Q - 1) / 2;
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) d[m - 1] = L[cs(m - 1)];
}

// ===========================================================================
// One workgroup per matrix, for batches of matrices of order at most
// SYTRD_WG_NMAX (by default FP64 only: SytrdWgMinBatch below).
//
// The per-column launches step every matrix of a batch through the columns
// of the largest in lockstep, each launch a dependent round trip.  Here one
// workgroup reduces a whole matrix, its barriers taking the place of
// launches; per column i (s = i + 1, J its panel column):
//   1. the thread of row r forms the column updated by the panel so far,
//      u(r) = A(r,i) - sum_k [V(r,k) W(i,k) + W(r,k) V(i,k)], into LDS;
//   2. the SYMV y' = A x of x = u on rows s+1.. (x(s) = 0) over the stored
//      trailing matrix, in the tiles of the multi-workgroup kernel with
//      WgDepth tiles in flight per wavefront, row and column sums added into
//      LDS; with it x^T x, x^T A x and the panel products W^T x, V^T x;
//   3. beta from ||x||, then A v = scale y' + A e_s, the panel corrections
//      and w = tau y - (tau^2/2)(y^T v) v, with y^T v formed from the
//      scalars of step 2 (no further reduction).
// Every thread forms w(s), which the next column's update needs, itself;
// the LDS column and y alternate between two buffers, so a column takes two
// barriers.  After each panel of SYTRD_NBP columns the rank-2 NBP update of
// the trailing matrix runs on the matrix cores.  Workgroups take the
// matrices largest first.  The last columns are left to the LDS tail
// kernel, as in the other path.
// ===========================================================================
#define SYTRD_WG_NMAX 1024
#define SYTRD_WG_WAVES 8
// SYMV tiles in flight per wavefront.  In FP64 two, with the panel loops of
// steps 1-3 unrolled twice (two iterations' loads in flight), fit in 249
// registers without spills; three tiles without unrolling measured 7% slower
// on 960 matrices of order 384, and every variant that spilled (unrolled four
// times, a four-wave occupancy target) or ran fewer waves per workgroup
// slower still.
template <typename T> struct WgDepth;
template <> struct WgDepth<float> { static constexpr int value = 6; };
template <> struct WgDepth<double> { static constexpr int value = 2; };

// order: the matrices by decreasing order (counting sort over the orders
// 0..SYTRD_WG_NMAX in one workgroup; the order among equal sizes is that of
// the atomics)
__global__ __launch_bounds__(1024) void sytrd_wg_order_kernel(const int* ns, int nbatch, int* order) {
    constexpr int NB = SYTRD_WG_NMAX + 1;
    __shared__ int cnt[NB];
    __shared__ int wsum[16];
    const int tid = threadIdx.x;
    for (int k = tid; k < NB; k += 1024) cnt[k] = 0;
    __syncthreads();
    for (int b = tid; b < nbatch; b += 1024) atomicAdd(&cnt[SYTRD_WG_NMAX - min(ns[b], SYTRD_WG_NMAX)], 1);
    __syncthreads();
    // exclusive prefix sum of the bin counts: two bins per thread (NB <= 2048)
    static_assert(NB <= 2048, "two bins per thread");
    const int k0 = 2 * tid;
    const int c0 = k0 < NB ? cnt[k0] : 0, c1 = k0 + 1 < NB ? cnt[k0 + 1] : 0;
    int v = c0 + c1;
    const int lane = tid & 63, wv = tid >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    int base = 0;
    for (int q = 0; q < wv; q++) base += wsum[q];
    const int excl = base + v - (c0 + c1);
    __syncthreads();
    if (k0 < NB) cnt[k0] = excl;
    if (k0 + 1 < NB) cnt[k0 + 1] = excl + c0;
    __syncthreads();
    for (int b = tid; b < nbatch; b += 1024) order[atomicAdd(&cnt[SYTRD_WG_NMAX - min(ns[b], SYTRD_WG_NMAX)], 1)] = b;
}

// A(t0:n, t0:n) -= V W^T + W V^T on the lower triangle, K = 2 NBP, on the
// matrix cores: each wavefront takes block rows of 16 HR rows (longest
// first), loads their operand rows [V W] once and sweeps the block columns
// of 16 HC columns at and left of the diagonal.
template <typename T, int NW>
__device__ void wg_syr2k(T* A, long long ld, const T* Vp, const T* Wp, int ldp, int n, int t0) {
    constexpr int NBP = SYTRD_NBP;
    constexpr int KS = 2 * NBP / 4;  // k steps of four
    constexpr int HR = sizeof(T) == 4 ? 2 : 1;
    constexpr int HC = sizeof(T) == 4 ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nbr = (n - t0 + 16 * HR - 1) / (16 * HR);
    for (int jj = wv; jj < nbr; jj += NW) {
        const int rb = t0 + 16 * HR * (nbr - 1 - jj);
        T af[HR][KS];
#pragma unroll
        for (int h = 0; h < HR; h++) {
            const int r = min(rb + 16 * h + (lane & 15), n - 1);
#pragma unroll
            for (int st = 0; st < KS; st++) {
                const int k = 4 * st + (lane >> 4);
                af[h][st] = k < NBP ? Vp[r + (long long)k * ldp] : Wp[r + (long long)(k - NBP) * ldp];
            }
        }
        for (int cc = t0; cc < rb + 16 * HR; cc += 16 * HC) {
            T bf[HC][KS];
#pragma unroll
            for (int h = 0; h < HC; h++) {
                const int c = min(cc + 16 * h + (lane & 15), n - 1);
#pragma unroll
                for (int st = 0; st < KS; st++) {
                    const int k = 4 * st + (lane >> 4);
                    bf[h][st] = k < NBP ? Wp[c + (long long)k * ldp] : Vp[c + (long long)(k - NBP) * ldp];
                }
            }
            typename mfma4<T>::v acc[HR][HC];
#pragma unroll
            for (int hr = 0; hr < HR; hr++)
#pragma unroll
                for (int hc = 0; hc < HC; hc++) acc[hr][hc] = typename mfma4<T>::v{0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < KS; st++)
#pragma unroll
                for (int hr = 0; hr < HR; hr++)
#pragma unroll
                    for (int hc = 0; hc < HC; hc++) acc[hr][hc] = mfma16x16x4(af[hr][st], bf[hc][st], acc[hr][hc]);
#pragma unroll
            for (int hr = 0; hr < HR; hr++)
#pragma unroll
                for (int hc = 0; hc < HC; hc++)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int r = rb + 16 * hr + mfma_rows<T>::row(lane, q);
                        const int c = cc + 16 * hc + (lane & 15);
                        if (r < n && c < n && r >= c) A[r + (long long)c * ld] -= acc[hr][hc][q];
                    }
        }
    }
}

template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void sytrd_wg_kernel(SytrdWs<T> w) {
    constexpr int NT = 64 * NW;
    constexpr int NBP = SYTRD_NBP;
    constexpr int RPT = (SYTRD_WG_NMAX + NT - 1) / NT;  // rows per thread
    constexpr int RPL = 16 / (int)sizeof(T);
    constexpr int LPC = 64 / RPL;
    constexpr int NI = 16 / RPL;
    constexpr int D = WgDepth<T>::value;
    typedef typename Vec16<T>::v VT;
    static_assert(NBP == 32 && NW % 4 == 0, "layout");
    __shared__ T ucb[2][SYTRD_WG_NMAX];  // updated column, by column parity
    __shared__ T yyb[2][SYTRD_WG_NMAX];  // y' = A x, by column parity
    __shared__ T dots[2 * NBP + 1];      // W^T x, V^T x, x^T x
    __shared__ T xaxw[NW];               // x^T A x per wavefront

    const int b = w.order[blockIdx.x];
    const int n = w.ns[b];
    const int kend = sytrd_tail_start<T>(n);
    if (kend <= 0) return;
    T* A = w.A.at(b);
    const long long ld = w.A.ld;
    T* Vp = w.Vp + (long long)b * w.sP;
    T* Wp = w.Wp + (long long)b * w.sP;
    const int ldp = w.ldp;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane / LPC, rq = lane % LPC;
    const int nbk = (n + 63) >> 6;
    unsigned coff[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) coff[k] = (unsigned)((RPL * k + g) * ld * (long long)sizeof(T));

    for (int k0 = 0; k0 < kend; k0 += NBP) {
        T ws_prev = T(0);  // w(s) of the previous column (its s is this column's i)
        for (int J = 0; J < NBP; J++) {
            const int i = k0 + J, s = i + 1, cb = i & 1;
            T* uc = ucb[cb];
            T* yy = yyb[cb];
            // ---- 1. column i updated by the panel's previous columns
#pragma unroll
            for (int t = 0; t < RPT; t++) {
                const int r = tid + t * NT;
                if (r >= i && r < n) {
                    T u = A[r + (long long)i * ld];
#pragma unroll 2
                    for (int k = 0; k + 1 < J; k++)
                        u -= Vp[r + (long long)k * ldp] * Wp[i + (long long)k * ldp] +
                             Wp[r + (long long)k * ldp] * Vp[i + (long long)k * ldp];
                    if (J > 0) u -= Vp[r + (long long)(J - 1) * ldp] * ws_prev + Wp[r + (long long)(J - 1) * ldp];
                    uc[r] = u;
                    yy[r] = T(0);
                }
            }
            __syncthreads();

            // ---- 2. panel products and norm of x, then the SYMV
            for (int q = wv; q <= 2 * J; q += NW) {
                const T* col = q < J ? Wp + (long long)q * ldp : Vp + (long long)(q - J) * ldp;
                T acc = T(0);
#pragma unroll 2
                for (int r = s + 1 + lane; r < n; r += 64) {
                    const T x = uc[r];
                    acc += (q == 2 * J ? x : col[r]) * x;
                }
                acc = wave_sum(acc);
                if (lane == 0) dots[q] = acc;
            }
            {
                const int b0 = s >> 6;
                const int P = 4 * (nbk - b0);  // column pairs: strip b0 + p / 4, sixteen columns 16 (p % 4)
                auto pair_c0 = [&](int p) { return 64 * (b0 + (p >> 2)) + 16 * (p & 3); };
                // this wavefront's pairs, in snake order over rounds of NW
                auto pair_of = [&](int k) { return k * NW + ((k & 1) ? NW - 1 - wv : wv); };
                struct It { int k, p, R; };
                auto seek = [&](It& it) {
                    for (;; it.k++) {
                        it.p = pair_of(it.k);
                        if (it.p >= P) return;
                        const int c0 = pair_c0(it.p);
                        if (c0 < n && c0 + 16 > s) break;
                    }
                    it.R = b0 + (it.p >> 2);
                };
                auto next = [&](It& it) {
                    if (it.p >= P) return;
                    if (++it.R < nbk) return;
                    it.k++;
                    seek(it);
                };
                auto issue = [&](VT (&bf)[NI], const It& it) {
                    if (it.p >= P) return;
                    const int c0 = pair_c0(it.p);
                    const int ncols = min(16, n - c0);
                    const __amdgpu_buffer_rsrc_t rs =
                        make_rsrc(A + (long long)c0 * ld, (unsigned)(ncols * ld * (long long)sizeof(T)));
                    const unsigned roff = (unsigned)((it.R * 64 + RPL * rq) * (int)sizeof(T));
#pragma unroll
                    for (int k = 0; k < NI; k++) {
                        const int c = c0 + RPL * k + g;
                        bf[k] = buf_load16<T>(rs, (c >= s && c < n) ? coff[k] + roff : OOB_OFFSET);
                    }
                };
                T vc[NI], cacc[NI];
                T xax = T(0);
                int cur = -1, pc0 = 0, pC = 0;
                auto start_pair = [&](const It& it) {
                    cur = it.p;
                    pc0 = pair_c0(it.p);
                    pC = b0 + (it.p >> 2);
#pragma unroll
                    for (int k = 0; k < NI; k++) {
                        const int c = pc0 + RPL * k + g;
                        vc[k] = (c > s && c < n) ? uc[c] : T(0);
                        cacc[k] = T(0);
                    }
                };
                auto flush_pair = [&]() {
#pragma unroll
                    for (int k = 0; k < NI; k++) xax += vc[k] * cacc[k];
                    T csum;
                    if constexpr (NI == 4) {
                        csum = quad_sum(pair_sum_b2(pair_sum_b3(cacc[0], cacc[2]), pair_sum_b3(cacc[1], cacc[3])));
                    } else {
                        const T u0 = pair_sum_b4(cacc[0], cacc[4]), u1 = pair_sum_b4(cacc[1], cacc[5]);
                        const T u2 = pair_sum_b4(cacc[2], cacc[6]), u3 = pair_sum_b4(cacc[3], cacc[7]);
                        csum = quad_sum(pair_sum_b2(pair_sum_b3(u0, u2), pair_sum_b3(u1, u3)));
                    }
                    const int c = pc0 + RPL * ((lane >> 2) % NI) + g;
                    if ((lane & 3) == 0 && c >= s && c < n)
                        __hip_atomic_fetch_add(&yy[c], csum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                };
                auto process = [&](const VT (&bf)[NI], int R) {
                    const int r0 = R * 64 + RPL * rq;
                    T vr[RPL], rs[RPL];
#pragma unroll
                    for (int e = 0; e < RPL; e++) {
                        const int r = r0 + e;
                        vr[e] = (r > s && r < n) ? uc[r] : T(0);
                        rs[e] = T(0);
                    }
#pragma unroll
                    for (int k = 0; k < NI; k++) {
                        const int c = pc0 + RPL * k + g;
#pragma unroll
                        for (int e = 0; e < RPL; e++) {
                            const int r = r0 + e;
                            const T xa = (r < n && (R > pC || r >= c)) ? bf[k][e] : T(0);
                            rs[e] += xa * vc[k];
                            cacc[k] += (R > pC || r != c) ? xa * vr[e] : T(0);
                        }
                    }
#pragma unroll
                    for (int e = 0; e < RPL; e++) xax += vr[e] * rs[e];
                    T rsum;
                    if constexpr (RPL == 4) {
                        rsum = pair_sum_b4(pair_sum_b5(rs[0], rs[2]), pair_sum_b5(rs[1], rs[3]));
                    } else {
                        rsum = pair_sum_b5(rs[0], rs[1]);
                    }
                    const int row = R * 64 + RPL * rq + g;
                    if (row >= s && row < n)
                        __hip_atomic_fetch_add(&yy[row], rsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                };
                It ip{0, 0, 0}, iq{0, 0, 0};
                seek(ip);
                seek(iq);
                VT buf[D][NI];
#pragma unroll
                for (int d = 0; d < D; d++) {
                    issue(buf[d], ip);
                    next(ip);
                }
                while (iq.p < P) {
#pragma unroll
                    for (int d = 0; d < D; d++) {
                        if (iq.p >= P) break;
                        if (iq.p != cur) {
                            if (cur >= 0) flush_pair();
                            start_pair(iq);
                        }
                        process(buf[d], iq.R);
                        issue(buf[d], ip);
                        next(ip);
                        next(iq);
                    }
                }
                if (cur >= 0) flush_pair();
                xax = wave_sum(xax);
                if (lane == 0) xaxw[wv] = xax;
            }
            __syncthreads();

            // ---- 3. reflector, y = A v with the panel corrections, w
            const T xn2 = dots[2 * J];
            const T alpha = uc[s];
            T beta, tau, scale;
            if (xn2 == T(0)) {
                tau = T(0); beta = alpha; scale = T(0);
            } else {
                const T nrm = sqrt(alpha * alpha + xn2);
                beta = alpha >= T(0) ? -nrm : nrm;
                tau = (beta - alpha) / beta;
                scale = T(1) / (alpha - beta);
            }
            T xax = T(0);
#pragma unroll
            for (int q = 0; q < NW; q++) xax += xaxw[q];
            const T ys = yy[s];
            const T Ass = A[s + (long long)s * ld];
            T corr[RPT], pq = T(0), corr_s = T(0);
#pragma unroll
            for (int t = 0; t < RPT; t++) corr[t] = T(0);
#pragma unroll 2
            for (int k = 0; k < J; k++) {
                const T Wsk = Wp[s + (long long)k * ldp], Vsk = Vp[s + (long long)k * ldp];
                const T pk = Wsk + scale * dots[k];      // W(:,k)^T v
                const T qk = Vsk + scale * dots[J + k];  // V(:,k)^T v
                pq += pk * qk;
                corr_s += Vsk * pk + Wsk * qk;
#pragma unroll
                for (int t = 0; t < RPT; t++) {
                    const int r = min(tid + t * NT, n - 1);
                    corr[t] += Vp[r + (long long)k * ldp] * pk + Wp[r + (long long)k * ldp] * qk;
                }
            }
            // v^T A v (A with the panel's updates) = y^T v
            const T vav = scale * scale * xax + T(2) * scale * ys + Ass - T(2) * pq;
            const T half = T(0.5) * tau * tau * vav;
            const T ws = tau * (scale * ys + Ass - corr_s) - half;
#pragma unroll
            for (int t = 0; t < RPT; t++) {
                const int r = tid + t * NT;
                if (r >= s && r < n) {
                    const T v = r == s ? T(1) : scale * uc[r];
                    const T wr = r == s ? ws : tau * (scale * yy[r] + A[r + (long long)s * ld] - corr[t]) - half * v;
                    Vp[r + (long long)J * ldp] = v;
                    Wp[r + (long long)J * ldp] = wr;
                    A[r + (long long)i * ld] = v;
                }
            }
            if (tid == 0) {
                w.d[(long long)b * w.sD + i] = uc[i];
                w.e[(long long)b * w.sD + i] = beta;
                w.tau[(long long)b * w.sD + i] = tau;
            }
            ws_prev = ws;
        }
        // ---- panel update of the trailing matrix
        __syncthreads();
        wg_syr2k<T, NW>(A, ld, Vp, Wp, ldp, n, k0 + NBP);
        __syncthreads();
    }
}

// ===========================================================================
// Fused per-column path: one launch per column.
//
// The launch for column i first finishes column c = i - 1 (what the separate
// finish phase does), in every workgroup for the rows that workgroup touches,
// then runs the SYMV of column i on the unscaled updated column
// x = A(i+1:n, i).  The reflector v = (x - beta e_1) / (alpha - beta) needs
// the norm of x, which is only complete when this launch has ended; every
// product the SYMV forms is linear in v, so the launch accumulates A x,
// W^T x, V^T x and x^T A x, and the next launch turns them into the products
// with v once beta is known:
//   A v     = (A x - beta A e_1) / (alpha - beta)
//   W^T v   = (W^T x - beta W(i+1, :)^T) / (alpha - beta)
//   v^T A v = (x^T A x - 2 beta (A x)_1 + beta^2 A_11) / (alpha - beta)^2
// (A the lower trailing matrix as stored, before this panel's update).  The
// last column of a panel is finished by a launch of its own: the panel
// update needs its w before the next column's SYMV.  Accumulators rotate
// over three slots (a launch reads the previous column's slot, adds into its
// own and clears the next one), the column buffer over two.
// ===========================================================================
template <typename T>
__device__ __forceinline__ T* yacc_s(const SytrdWs<T>& w, int b, int slot, int copy) {
    return w.yacc + (long long)b * w.sY + (slot * SYTRD_YC + copy) * (long long)w.nmax;
}
template <typename T>
__device__ __forceinline__ T* sacc_s(const SytrdWs<T>& w, int b, int slot, int copy) {
    return w.sacc + (long long)b * w.sS + (slot * SYTRD_YC + copy) * (2 * SYTRD_NBP);
}
template <typename T>
__device__ __forceinline__ T* vacc_s(const SytrdWs<T>& w, int b, int slot) {
    return w.vacc + (long long)b * (SYTRD_SLOTS * SYTRD_VC) + slot * SYTRD_VC;
}
template <typename T>
__device__ __forceinline__ T* norm_s(const SytrdWs<T>& w, int b, int slot) {
    return w.normacc + (long long)b * SYTRD_SLOTS + slot;
}
template <typename T>
__device__ __forceinline__ T* col_s(const SytrdWs<T>& w, int b, int slot2) {
    return w.colbuf + (long long)b * 2 * w.sC + slot2 * w.sC;
}

// Scalars of the finished column c, held by every wavefront.
template <typename T>
struct FinScal {
    T beta, tau, scale, wtv, ws, us, dprev;
    bool zero;  // x(2:) == 0: H = I, v = e_1
};

// Row r of the finish of column c: the inputs, requested together.
template <typename T>
struct FinRow {
    T uc, ar, yc[SYTRD_YC], vk[SYTRD_NBP], wk[SYTRD_NBP];
};

// c: finished column (s = c + 1 its reflector's first row), J: its panel
// column.  Rows are clamped into the matrix; the panel columns k >= J (not
// yet written in this panel) are requested at an out-of-range offset, which
// reads zero without a memory access.
template <typename T>
__device__ __forceinline__ void fin_load(const SytrdWs<T>& w, int b, int n, int c, int J, int r, FinRow<T>& f) {
    const int s = c + 1, sl = c % SYTRD_SLOTS;
    const int rc = r < n ? r : n - 1;
    f.uc = col_s(w, b, c & 1)[rc];
    f.ar = w.A.at(b)[rc + (long long)s * w.A.ld];
#pragma unroll
    for (int cp = 0; cp < SYTRD_YC; cp++) f.yc[cp] = yacc_s(w, b, sl, cp)[rc];
    const unsigned pbytes = (unsigned)(w.sP * (long long)sizeof(T));
    const __amdgpu_buffer_rsrc_t vs = make_rsrc(w.Vp + (long long)b * w.sP, pbytes);
    const __amdgpu_buffer_rsrc_t ws = make_rsrc(w.Wp + (long long)b * w.sP, pbytes);
#pragma unroll
    for (int k = 0; k < SYTRD_NBP; k++) {
        const unsigned off = k < J ? (unsigned)((rc + (long long)k * w.ldp) * sizeof(T)) : OOB_OFFSET;
        f.vk[k] = buf_load<T>(vs, off);
        f.wk[k] = buf_load<T>(ws, off);
    }
}

// Column scalars of the finished column c from the accumulators of its SYMV
// (reflector: LAPACK dlarfg convention, beta = -sign(alpha) ||x||,
// tau = (beta - alpha) / beta), then the panel products with v, v^T A v,
// w^T v, and w and the updated next column at row s.  Each wavefront forms
// them on its own (no barrier); coef (wavefront-private LDS) receives
// p_k = W(:,k)^T v, s_k = V(:,k)^T v, W(s,k), V(s,k), zero for k >= J.
template <typename T>
__device__ __forceinline__ FinScal<T> fin_scalars(const SytrdWs<T>& w, int b, int c, int J, T (*coef)[4]) {
    constexpr int NBP = SYTRD_NBP;
    static_assert(SYTRD_VC == 256 && SYTRD_YC == 4 && 2 * NBP == 64, "accumulator layout");
    const int lane = threadIdx.x & 63;
    const int s = c + 1, sl = c % SYTRD_SLOTS;
    const T* A = w.A.at(b);
    const long long ld = w.A.ld;
    const int k = lane & (NBP - 1);
    T sW[SYTRD_YC], sV[SYTRD_YC], va[4];
#pragma unroll
    for (int cp = 0; cp < SYTRD_YC; cp++) {
        sW[cp] = sacc_s(w, b, sl, cp)[k];
        sV[cp] = sacc_s(w, b, sl, cp)[NBP + k];
    }
#pragma unroll
    for (int t = 0; t < 4; t++) va[t] = vacc_s(w, b, sl)[lane + 64 * t];
    const unsigned pbytes = (unsigned)(w.sP * (long long)sizeof(T));
    const unsigned off = lane < J ? (unsigned)((s + (long long)lane * w.ldp) * sizeof(T)) : OOB_OFFSET;
    const T Vs = buf_load<T>(make_rsrc(w.Vp + (long long)b * w.sP, pbytes), off);
    const T Ws = buf_load<T>(make_rsrc(w.Wp + (long long)b * w.sP, pbytes), off);
    const T yq = yacc_s(w, b, sl, lane & (SYTRD_YC - 1))[s];
    const T xn2 = *norm_s(w, b, sl);
    const T alpha = col_s(w, b, c & 1)[s];
    const T dprev = col_s(w, b, c & 1)[c];
    const T Ass = A[s + (long long)s * ld];

    const T xAx = wave_sum((va[0] + va[1]) + (va[2] + va[3]));
    const T yxs = (lane_value(yq, 0) + lane_value(yq, 1)) + (lane_value(yq, 2) + lane_value(yq, 3));
    FinScal<T> f;
    f.zero = xn2 == T(0);
    if (f.zero) {
        f.tau = T(0); f.beta = alpha; f.scale = T(0);
    } else {
        const T nrm = sqrt(alpha * alpha + xn2);
        f.beta = alpha >= T(0) ? -nrm : nrm;
        f.tau = (f.beta - alpha) / f.beta;
        f.scale = T(1) / (alpha - f.beta);
    }
    const bool kv = lane < J;
    const T Wx = (sW[0] + sW[1]) + (sW[2] + sW[3]);
    const T Vx = (sV[0] + sV[1]) + (sV[2] + sV[3]);
    const T pk = kv ? f.scale * (Wx - f.beta * Ws) : T(0);
    const T sk = kv ? f.scale * (Vx - f.beta * Vs) : T(0);
    const T pts = wave_sum(pk * sk);
    const T corr = wave_sum(Vs * pk + Ws * sk);
    const T vw = wave_sum(Vs * Ws);
    const T vAv = f.scale * f.scale * ((xAx - T(2) * f.beta * yxs) + f.beta * f.beta * Ass);
    f.wtv = f.tau * (vAv - T(2) * pts);
    f.ws = f.tau * (f.scale * (yxs - f.beta * Ass) - corr) - T(0.5) * f.tau * f.wtv;
    f.us = Ass - T(2) * vw - T(2) * f.ws;
    f.dprev = dprev;
    if (lane < NBP) {
        coef[lane][0] = pk;
        coef[lane][1] = sk;
        coef[lane][2] = Ws;
        coef[lane][3] = Vs;
    }
    return f;
}

// v and w of the finished column at row r, and the next column (s) updated
// by the whole panel so far at row r:
//   w(r) = tau (A v - V p - W s)(r) - (tau/2) (w^T v) v(r)
//   u(r) = A(r, s) - sum_k [V(r,k) W(s,k) + W(r,k) V(s,k)]      (k <= J, V(s, J) = 1)
// with A v, the panel products and v^T A v from those of x (above).
template <typename T>
__device__ __forceinline__ void fin_row(const FinScal<T>& fs, const T (*coef)[4], const FinRow<T>& f, int r, int s,
                                        int n, T& v, T& wr, T& u) {
    const bool rv = r >= s && r < n;
    T corr = T(0), ucor = T(0);
#pragma unroll
    for (int k = 0; k < SYTRD_NBP; k++) {
        corr += f.vk[k] * coef[k][0] + f.wk[k] * coef[k][1];
        ucor += f.vk[k] * coef[k][2] + f.wk[k] * coef[k][3];
    }
    const T yx = (f.yc[0] + f.yc[1]) + (f.yc[2] + f.yc[3]);
    T vr = r == s ? T(1) : (fs.zero ? T(0) : fs.scale * f.uc);
    vr = rv ? vr : T(0);
    const T yv = fs.scale * (yx - fs.beta * f.ar);
    wr = rv ? fs.tau * (yv - corr) - T(0.5) * fs.tau * fs.wtv * vr : T(0);
    u = f.ar - ucor - vr * fs.ws - wr;
    v = vr;
}

// The updated next column at row r as fin_row computes it, with the panel
// rows read eight columns at a time (for rows beyond the first block of a
// wave, where no latency is to be hidden and registers are short).
template <typename T>
__device__ __forceinline__ T fin_row_stream(const SytrdWs<T>& w, const FinScal<T>& fs, const T (*coef)[4], int b, int n,
                                            int c, int J, int r) {
    const int s = c + 1, sl = c % SYTRD_SLOTS;
    const int rc = r < n ? r : n - 1;
    const T uc = col_s(w, b, c & 1)[rc];
    const T ar = w.A.at(b)[rc + (long long)s * w.A.ld];
    T yc[SYTRD_YC];
#pragma unroll
    for (int cp = 0; cp < SYTRD_YC; cp++) yc[cp] = yacc_s(w, b, sl, cp)[rc];
    const T* Vp = w.Vp + (long long)b * w.sP + rc;
    const T* Wp = w.Wp + (long long)b * w.sP + rc;
    T corr = T(0), ucor = T(0);
#pragma unroll 1
    for (int k0 = 0; k0 < J; k0 += 8) {
        T vk[8], wk[8];
#pragma unroll
        for (int t = 0; t < 8; t++) {
            const int k = k0 + t < J ? k0 + t : J - 1;
            const T a = Vp[(long long)k * w.ldp], bb = Wp[(long long)k * w.ldp];
            vk[t] = k0 + t < J ? a : T(0);
            wk[t] = k0 + t < J ? bb : T(0);
        }
#pragma unroll
        for (int t = 0; t < 8; t++) {
            corr += vk[t] * coef[k0 + t][0] + wk[t] * coef[k0 + t][1];
            ucor += vk[t] * coef[k0 + t][2] + wk[t] * coef[k0 + t][3];
        }
    }
    const bool rv = r >= s && r < n;
    const T yx = (yc[0] + yc[1]) + (yc[2] + yc[3]);
    T vr = r == s ? T(1) : (fs.zero ? T(0) : fs.scale * uc);
    vr = rv ? vr : T(0);
    const T yv = fs.scale * (yx - fs.beta * ar);
    const T wr = rv ? fs.tau * (yv - corr) - T(0.5) * fs.tau * fs.wtv * vr : T(0);
    return ar - ucor - vr * fs.ws - wr;
}

// ---------------------------------------------------------------------------
// Column work item: finishes column i - 1 on the item's rows (j > 0), then
// the SYMV of column i over tiles R in [C + q Kt, C + (q+1) Kt) of strip C,
// as symv_item but with x in LDS.  Items q == 0 also store what the finish
// produces on the rows of block C (v, w into the panel, v into the matrix,
// the next column and its norm) and clear the next slot there.
// ---------------------------------------------------------------------------
template <typename T, int NBP>
__device__ void col_item(const SytrdWs<T>& w, int b, int n, int i, int j, int Kt, int C, int q) {
    constexpr int RPL = 16 / (int)sizeof(T);
    constexpr int LPC = 64 / RPL;
    constexpr int NI = 16 / RPL;
    typedef typename Vec16<T>::v VT;
    static_assert(NBP == SYTRD_NBP && NBP == 32, "panel products in four groups of sixteen");
    __shared__ T rpart[SYTRD_KTMAX][4][64];
    __shared__ T ubuf[SYTRD_KTMAX + 1][64];  // x on the rows of the item's blocks
    __shared__ T coefw[4][SYTRD_NBP][4];     // per-wavefront column coefficients
    __shared__ T red[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane / LPC, rq = lane % LPC;
    const int t1 = i + 1;  // first row of the trailing block
    const int b0 = t1 >> 6;
    const int nbk = (n + 63) >> 6;
    T* A = w.A.at(b);
    const long long ld = w.A.ld;
    const int ldp = w.ldp;
    const int Rb = C + q * Kt;
    const int Re = min(Rb + Kt, nbk);
    const int c0 = C * 64 + wv * 16;
    // the item's row blocks: C first, then the tile rows (q == 0: they start at C)
    const int nblk = (q == 0 ? 0 : 1) + (Re - Rb);
    auto blk = [&](int m) { return q == 0 ? C + m : (m == 0 ? C : Rb + m - 1); };
    auto slot_of = [&](int R) { return q == 0 ? R - C : 1 + R - Rb; };

    // the first tile is requested before anything else
    const int ncols = max(0, min(16, n - c0));
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(A + (long long)c0 * ld, (unsigned)(ncols * ld * (long long)sizeof(T)));
    unsigned coff[NI];
    bool cok[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) {
        const int c = c0 + RPL * k + g;
        cok[k] = c >= t1 && c < n;
        coff[k] = (unsigned)((RPL * k + g) * ld * (long long)sizeof(T));
    }
    VT buf[NI];
    auto issue = [&](int R) {
        const unsigned roff = R < Re ? (unsigned)((R * 64 + RPL * rq) * (int)sizeof(T)) : OOB_OFFSET;
#pragma unroll
        for (int k = 0; k < NI; k++) buf[k] = buf_load16<T>(rsrc, cok[k] ? coff[k] + roff : OOB_OFFSET);
    };
    issue(Rb);

    const bool fin = j > 0;
    const int cf = i - 1, J = j - 1;
    const int sln = (i + 1) % SYTRD_SLOTS, slc = i % SYTRD_SLOTS;
    FinScal<T> fs{};
    if (fin && wv < nblk) {
        // the first block of each wave: its row data is requested with the
        // tile, the column scalars formed while it arrives
        FinRow<T> fr;
        const int r = blk(wv) * 64 + lane;
        fin_load(w, b, n, cf, J, r, fr);
        fs = fin_scalars(w, b, cf, J, coefw[wv]);
        {
            T v, wr, u;
            fin_row(fs, coefw[wv], fr, r, i, n, v, wr, u);
            const T x = (r >= t1 && r < n) ? u : T(0);
            ubuf[wv][lane] = x;
            if (wv == 0 && q == 0) {
                // block C: what the finish produces, stored once
                T* Vp = w.Vp + (long long)b * w.sP;
                T* Wp = w.Wp + (long long)b * w.sP;
                if (r < n) {
                    Vp[r + (long long)J * ldp] = v;
                    Wp[r + (long long)J * ldp] = wr;
                    if (r >= i) {
                        A[r + (long long)cf * ld] = v;
                        col_s(w, b, i & 1)[r] = u;
                    }
                }
                T q2 = (r >= i + 2 && r < n) ? u * u : T(0);
                q2 = wave_sum(q2);
                if (lane == 0) unsafeAtomicAdd(norm_s(w, b, slc), q2);
                // panel products of column i over the rows of block C:
                // W(:,k)^T x and V(:,k)^T x for k <= J (column J is w, v)
                T* sacc = sacc_s(w, b, slc, C % SYTRD_YC);
#pragma unroll
                for (int grp = 0; grp < 4; grp++) {
                    const int kb = (grp & 1) * 16;
                    if (kb <= J) {
                        T pr[16];
#pragma unroll
                        for (int t = 0; t < 16; t++) {
                            const int k = kb + t;
                            const T pv = grp < 2 ? (k == J ? wr : fr.wk[k]) : (k == J ? v : fr.vk[k]);
                            pr[t] = pv * x;
                        }
                        const T ps = wave_sum16(pr);
                        const int k = kb + (lane >> 2);
                        if ((lane & 3) == 0 && k <= J) unsafeAtomicAdd(&sacc[(grp >> 1) * NBP + k], ps);
                    }
                }
            }
        }
        // further blocks (long strips): one at a time, streaming the panel
        for (int m = wv + 4; m < nblk; m += 4) {
            const int r2 = blk(m) * 64 + lane;
            ubuf[m][lane] = (r2 >= t1 && r2 < n) ? fin_row_stream(w, fs, coefw[wv], b, n, cf, J, r2) : T(0);
        }
    } else if (!fin) {
        for (int m = wv; m < nblk; m += 4) {
            const int r = blk(m) * 64 + lane;
            const T uu = col_s(w, b, i & 1)[r < n ? r : n - 1];
            ubuf[m][lane] = (r >= t1 && r < n) ? uu : T(0);
        }
    }
    if (q == 0) {
        // clear the next column's slot on the rows of block C
        const int r = C * 64 + lane;
        if (r < n) yacc_s(w, b, sln, wv)[r] = T(0);
        if (C == b0) {
            sacc_s(w, b, sln, wv)[lane] = T(0);
            vacc_s(w, b, sln)[tid] = T(0);
            if (tid == 0) *norm_s(w, b, sln) = T(0);
            if (fin && tid == 0) {
                // row i when it lies above block b0, and the finished column's outputs
                if (i < b0 * 64) {
                    w.Vp[(long long)b * w.sP + i + (long long)J * ldp] = T(1);
                    w.Wp[(long long)b * w.sP + i + (long long)J * ldp] = fs.ws;
                    A[i + (long long)cf * ld] = T(1);
                    col_s(w, b, i & 1)[i] = fs.us;
                }
                w.d[(long long)b * w.sD + cf] = fs.dprev;
                w.e[(long long)b * w.sD + cf] = fs.beta;
                w.tau[(long long)b * w.sD + cf] = fs.tau;
            }
        }
    }
    __syncthreads();

    // SYMV of column i with x
    T vc[NI], cacc[NI];
#pragma unroll
    for (int k = 0; k < NI; k++) {
        vc[k] = ubuf[0][wv * 16 + RPL * k + g];
        cacc[k] = T(0);
    }
    T* yacc = yacc_s(w, b, slc, C % SYTRD_YC);
    for (int R = Rb; R < Re; R++) {
        const int r0 = R * 64 + RPL * rq;
        const int sl = slot_of(R);
        T vr[RPL], rs[RPL];
#pragma unroll
        for (int e = 0; e < RPL; e++) {
            vr[e] = ubuf[sl][RPL * rq + e];
            rs[e] = T(0);
        }
#pragma unroll
        for (int k = 0; k < NI; k++) {
            const int c = c0 + RPL * k + g;
#pragma unroll
            for (int e = 0; e < RPL; e++) {
                const int r = r0 + e;
                const T xa = (r < n && (R > C || r >= c)) ? buf[k][e] : T(0);
                rs[e] += xa * vc[k];
                cacc[k] += (R > C || r != c) ? xa * vr[e] : T(0);
            }
        }
        issue(R + 1);
        T rsum;
        if constexpr (RPL == 4) {
            rsum = pair_sum_b4(pair_sum_b5(rs[0], rs[2]), pair_sum_b5(rs[1], rs[3]));
        } else {
            rsum = pair_sum_b5(rs[0], rs[1]);
        }
        rpart[R - Rb][wv][RPL * rq + g] = rsum;
    }
    T vav = T(0);
#pragma unroll
    for (int k = 0; k < NI; k++) vav += vc[k] * cacc[k];
    T csum;
    if constexpr (NI == 4) {
        csum = quad_sum(pair_sum_b2(pair_sum_b3(cacc[0], cacc[2]), pair_sum_b3(cacc[1], cacc[3])));
    } else {
        const T u0_ = pair_sum_b4(cacc[0], cacc[4]), u1 = pair_sum_b4(cacc[1], cacc[5]);
        const T u2 = pair_sum_b4(cacc[2], cacc[6]), u3 = pair_sum_b4(cacc[3], cacc[7]);
        csum = quad_sum(pair_sum_b2(pair_sum_b3(u0_, u2), pair_sum_b3(u1, u3)));
    }
    {
        const int c = c0 + RPL * ((lane >> 2) % NI) + g;
        if ((lane & 3) == 0 && c >= t1 && c < n) unsafeAtomicAdd(&yacc[c], csum);
    }
    __syncthreads();
    for (int t = wv; t < Re - Rb; t += 4) {
        const T y = (rpart[t][0][lane] + rpart[t][1][lane]) + (rpart[t][2][lane] + rpart[t][3][lane]);
        const int r = (Rb + t) * 64 + lane;
        if (r >= t1 && r < n) {
            unsafeAtomicAdd(&yacc[r], y);
            vav += ubuf[slot_of(Rb + t)][lane] * y;
        }
    }
    vav = block_sum256(vav, red);
    if (tid == 0) unsafeAtomicAdd(vacc_s(w, b, slc) + (C * 7 + q) % SYTRD_VC, vav);
}

// Trailing orders at and below which the fused path is used (measured on
// the N=2000 cluster reduction: above it the redundant row work of the
// fused launch costs more than the finish launch it saves; in FP64 the
// fused launch's registers leave one wavefront per SIMD).
#define SYTRD_FUSED_KT 3
// Batches of at least this many matrices, all of order <= SYTRD_WG_NMAX,
// take the one-workgroup-per-matrix path (0: never).  One workgroup streams
// its matrix far below the device's bandwidth, so the path needs a batch
// that fills the 256 compute units.  Measured on 512 molecules of orders
// 30..900: FP64 54 ms against 66 ms per reduction for the per-column
// launches, FP32 37 ms against 34 ms (FP32 keeps the per-column launches);
// on 64 matrices of order 384 (a periodic cell's q-points) FP64 4.5 ms
// against about 3 ms.
template <typename T> struct SytrdWgMinBatch;
template <> struct SytrdWgMinBatch<float> { static constexpr int value = 0; };
template <> struct SytrdWgMinBatch<double> { static constexpr int value = 256; };
template <typename T> struct SytrdFused;
template <> struct SytrdFused<float> { static constexpr int max_order = 4000; };
template <> struct SytrdFused<double> { static constexpr int max_order = 0; };
// occupancy target of the fused kernel (waves per SIMD): in FP32 three is the
// most without spills (168 registers; a target of four spills 45)
template <typename T> struct ColWaves;
template <> struct ColWaves<float> { static constexpr int value = 3; };
template <> struct ColWaves<double> { static constexpr int value = 1; };
template <typename T, int NBP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ColWaves<T>::value)))
void sytrd_col_kernel(SytrdWs<T> w, int i, int j, int Kt, int nbatch) {
    const int b = blockIdx.x % nbatch;
    const int n = w.ns[b];
    if (i > n - 2 || i >= sytrd_tail_start<T>(n)) return;
    const int b0 = (i + 1) >> 6;
    const int nbk = (n + 63) >> 6;
    const int C = b0 + blockIdx.y;
    const int q = blockIdx.x / nbatch;
    if (C >= nbk || q >= (nbk - C + Kt - 1) / Kt) return;
    col_item<T, NBP>(w, b, n, i, j, Kt, C, q);
}

// Finish of the last column c of a panel (panel column J), one workgroup per
// 64-row block from the block of s = c + 1: stores v, w, the reflector, the
// updated column s and its norm, and the column's d, e, tau.
template <typename T, int NBP>
__global__ __launch_bounds__(64) void sytrd_pfinish_kernel(SytrdWs<T> w, int c, int J) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    if (c > n - 2 || c >= sytrd_tail_start<T>(n)) return;
    const int s = c + 1;
    const int nbk = (n + 63) >> 6;
    const int R = (s >> 6) + blockIdx.x;
    if (R >= nbk) return;
    __shared__ T coef[SYTRD_NBP][4];
    const int lane = threadIdx.x;
    const int r = R * 64 + lane;
    FinRow<T> fr;
    fin_load(w, b, n, c, J, r, fr);
    const FinScal<T> fs = fin_scalars(w, b, c, J, coef);
    T v, wr, u;
    fin_row(fs, coef, fr, r, s, n, v, wr, u);
    T* A = w.A.at(b);
    if (r < n) {
        w.Vp[(long long)b * w.sP + r + (long long)J * w.ldp] = v;
        w.Wp[(long long)b * w.sP + r + (long long)J * w.ldp] = wr;
        if (r >= s) {
            A[r + (long long)c * w.A.ld] = v;
            col_s(w, b, s & 1)[r] = u;
        }
    }
    T q2 = (r >= s + 2 && r < n) ? u * u : T(0);
    q2 = wave_sum(q2);
    if (lane == 0) unsafeAtomicAdd(norm_s(w, b, s % SYTRD_SLOTS), q2);
    if (R == (s >> 6) && lane == 0) {
        w.d[(long long)b * w.sD + c] = fs.dprev;
        w.e[(long long)b * w.sD + c] = fs.beta;
        w.tau[(long long)b * w.sD + c] = fs.tau;
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename T, int NBP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SymvWaves<T>::value)))
void sytrd_symv_kernel(SytrdWs<T> w, int i, int j, int Kt, int nbatch) {
    const int b = blockIdx.x % nbatch;
    const int n = w.ns[b];
    if (i > n - 2 || i >= sytrd_tail_start<T>(n)) return;
    const int b0 = (i + 1) >> 6;
    const int nbk = (n + 63) >> 6;
    const int C = b0 + blockIdx.y;
    const int q = blockIdx.x / nbatch;
    // the norm slot of column i + 1 is filled by this column's finish phase
    if (q == 0 && blockIdx.y == 0 && threadIdx.x == 0) w.normacc[(long long)b * SYTRD_SLOTS + (i + 1) % SYTRD_SLOTS] = T(0);
    if (C >= nbk || q >= (nbk - C + Kt - 1) / Kt) return;
    symv_item<T, NBP>(w, b, n, i, j, Kt, C, q, nullptr);
}

template <typename T, int NBP>
__global__ __launch_bounds__(256) void sytrd_finish_kernel(SytrdWs<T> w, int i, int j) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    if (i > n - 2 || i >= sytrd_tail_start<T>(n)) return;
    const int b0 = (i + 1) >> 6;
    const int nbk = (n + 63) >> 6;
    const int R = b0 + blockIdx.x;
    if (R >= nbk) return;
    finish_item<T, NBP>(w, b, n, i, j, R);
}

// Trailing update A(t0:n, t0:n) -= V W^T + W V^T, lower TS x TS tiles only.
// t0 is a multiple of the panel width and the leading dimension a multiple of
// 64, so the epilogue reads A before the K loop and writes it back in aligned
// 16-byte column segments (elements above the diagonal left untouched).
template <typename T, int NBP, int TS>
struct Syr2kProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = true;
    static constexpr bool EPI_VEC = true;
    typedef typename Vec16<T>::v Vec;
    static constexpr int RPL = 16 / (int)sizeof(T);
    static_assert(NBP % RPL == 0, "panel starts align to 16-byte segments");
    MatBatch<T> A;
    const int* ns;
    const T* Vp; const T* Wp; int ldp; long long sP;
    int t0;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        t.batch = bz;
        t.e0 = ns[bz];  // order, read once
        const int mb = ns[bz] - t0;
        if (mb <= 0 || t0 - NBP >= sytrd_tail_start<T>(ns[bz])) return false;
        int ti, tj;
        lower_tile(bx, ti, tj);
        t.m0 = ti * TS; t.n0 = tj * TS; t.K = 2 * NBP;
        return t.m0 < mb;
    }
    __device__ T a(const GemmTile& t, int m, int k) const {
        const int r = t0 + m;
        if (r >= t.e0) return T(0);
        const long long o = (long long)t.batch * sP + r;
        return k < NBP ? Vp[o + (long long)k * ldp] : Wp[o + (long long)(k - NBP) * ldp];
    }
    __device__ T b(const GemmTile& t, int k, int nn) const {
        const int c = t0 + nn;
        if (c >= t.e0) return T(0);
        const long long o = (long long)t.batch * sP + c;
        return k < NBP ? Wp[o + (long long)k * ldp] : Vp[o + (long long)(k - NBP) * ldp];
    }
    __device__ Vec epi_load(const GemmTile& t, int m, int nn) const {
        const int r = t0 + m, c = t0 + nn, nb_ = t.e0;
        if (r >= nb_ || c >= nb_ || r + RPL <= c) return Vec{};
        return *reinterpret_cast<const Vec*>(A.at(t.batch) + r + (long long)c * A.ld);
    }
    __device__ void epi_store(const GemmTile& t, int m, int nn, Vec acc, Vec cin) const {
        const int r = t0 + m, c = t0 + nn, nb_ = t.e0;
        if (r >= nb_ || c >= nb_ || r + RPL <= c) return;
        T* a = A.at(t.batch) + r + (long long)c * A.ld;
        if (r >= c && r + RPL <= nb_) {
            *reinterpret_cast<Vec*>(a) = cin - acc;
        } else {
#pragma unroll
            for (int e = 0; e < RPL; e++)
                if (r + e >= c && r + e < nb_) a[e] = cin[e] - acc[e];
        }
    }
    __device__ void store(const GemmTile&, int, int, T) const {}
};

template <typename T>
void sytrd_launch(const SytrdWs<T>& w, int nbatch, int nmax, hipStream_t st, const int* ns_host,
                  LaunchProfiler* prof) {
    constexpr int NBP = SYTRD_NBP;
    const bool timing = prof && prof->enabled && prof->launches && ns_host;
    const int nbk_max = w.nbk_max;
    // panels whose trailing order is at most fused_max run one launch per
    // column (the fused path); larger ones the SYMV and finish launches
    static const int env_max = [] {
        const char* e = std::getenv("MBD_SYTRD_FUSED_MAXN");
        return e ? std::atoi(e) : -1;
    }();
    const int fused_max = env_max >= 0 ? env_max : SytrdFused<T>::max_order;
    // batches of small matrices: one workgroup per matrix
    static const int env_wg = [] {
        const char* e = std::getenv("MBD_SYTRD_WG_MIN_BATCH");
        return e ? std::atoi(e) : -1;
    }();
    const int wg_min = env_wg >= 0 ? env_wg : SytrdWgMinBatch<T>::value;
    if (wg_min > 0 && nbatch >= wg_min && nmax <= SYTRD_WG_NMAX) {
        if (sytrd_tail_start<T>(nmax) > 0) {
            hipLaunchKernelGGL(sytrd_wg_order_kernel, dim3(1), dim3(1024), 0, st, w.ns, nbatch, w.order);
            auto k = sytrd_wg_kernel<T, SYTRD_WG_WAVES>;
            if (timing) {
                double bb = 0;
                for (int b = 0; b < nbatch; b++) {
                    const int kt = sytrd_tail_start<T>(ns_host[b]);
                    for (int i = 0; i < kt; i++) {
                        const double m = ns_host[b] - i - 1;
                        bb += m * (m + 1) * 0.5 * sizeof(T);
                    }
                }
                hipEvent_t e0, e1;
                prof->pair(&e0, &e1, 10, bb);
                hipExtLaunchKernelGGL(k, dim3(nbatch), dim3(64 * SYTRD_WG_WAVES), 0, st, e0, e1, 0, w);
            } else {
                hipLaunchKernelGGL(k, dim3(nbatch), dim3(64 * SYTRD_WG_WAVES), 0, st, w);
            }
        }
        hipLaunchKernelGGL(sytrd_tail_kernel<T>, dim3(nbatch), dim3(SYTRD_TAIL_THREADS), 0, st, w);
        return;
    }
    hipLaunchKernelGGL(sytrd_zero_norm_kernel<T>, dim3((SYTRD_SLOTS * nbatch + 255) / 256), dim3(256), 0, st, w, nbatch);
    hipLaunchKernelGGL(sytrd_init_kernel<T>, dim3(nbk_max, 1, nbatch), dim3(256), 0, st, w);
    // panels up to the tail of the largest matrix (smaller ones drop out of
    // the per-column kernels at their own tail start)
    const int kend = sytrd_tail_start<T>(nmax);
    for (int k0 = 0; k0 < kend && k0 + 2 <= nmax; k0 += NBP) {
        const int k1 = std::min(k0 + NBP, nmax - 1);
        // fused only where work items can be short (at most SYTRD_FUSED_KT
        // tiles at the default target, so at most four row blocks to finish
        // per item, one per wavefront): in batches of small matrices an item
        // spans a whole strip.  The choice depends on the sizes only, not on
        // the tuned targets; inside a fused panel the item length is capped.
        const bool fused = nmax - k0 - 1 <= fused_max &&
                           sytrd_kt(nbk_max - ((k0 + 1) >> 6), nbatch, 1536) <= SYTRD_FUSED_KT;
        {
            for (int i = k0; i < k1; i++) {
                const int j = i - k0;
                const int b0 = (i + 1) >> 6;
                const int nbt = nbk_max - b0;
                // trailing sizes in the upper quarter stream many tiles per
                // workgroup already; below it fewer, longer work items measured
                // faster, so each range has its own tuned target
                const int tgt = 4 * nbt >= 3 * nbk_max ? w.chunk_target : w.chunk_target_lo;
                const int Kt0 = sytrd_kt(nbt, nbatch, tgt > 0 ? tgt : 1536);
                const int Kt = fused ? std::min(Kt0, SYTRD_FUSED_KT) : Kt0;
                const int gx = (nbt + Kt - 1) / Kt;
                auto kern = fused ? sytrd_col_kernel<T, NBP> : sytrd_symv_kernel<T, NBP>;
                if (timing) {
                    double bb = 0;
                    for (int b = 0; b < nbatch; b++) {
                        const double m = ns_host[b] - i - 1;
                        if (m > 0) bb += m * (m + 1) * 0.5 * sizeof(T);
                    }
                    hipEvent_t e0, e1;
                    prof->pair(&e0, &e1, fused ? 8 : 0, bb);
                    hipExtLaunchKernelGGL(kern, dim3(gx * nbatch, nbt), dim3(256), 0, st, e0, e1, 0, w, i, j, Kt, nbatch);
                } else {
                    hipLaunchKernelGGL(kern, dim3(gx * nbatch, nbt), dim3(256), 0, st, w, i, j, Kt, nbatch);
                }
                if (!fused)
                    hipLaunchKernelGGL((sytrd_finish_kernel<T, NBP>), dim3(nbt, 1, nbatch), dim3(256), 0, st, w, i, j);
            }
            if (fused && k1 > k0) {
                // the panel's last column is finished before the panel update
                const int c = k1 - 1;
                hipLaunchKernelGGL((sytrd_pfinish_kernel<T, NBP>), dim3(nbk_max - ((c + 1) >> 6), 1, nbatch), dim3(64),
                                   0, st, w, c, c - k0);
            }
        }
        const int t0 = k0 + NBP;
        if (k1 == k0 + NBP && t0 + 1 < nmax) {
            // K = 2 NBP is only 4 slabs deep: a 128 x 128 tile's prologue and
            // epilogue outweighed its lower L2 traffic (measured 7.5 vs 6.2 ms
            // FP32, 9.3 vs 7.5 ms FP64 per N=2000 reduction), so 64 x 64 tiles
            const int tm = (nmax - t0 + 63) / 64;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (timing) {
                double flops = 0;
                for (int b = 0; b < nbatch; b++) {
                    const double m = ns_host[b] - t0;
                    if (m > 0) flops += 2.0 * (2 * NBP) * m * (m + 1) * 0.5;
                }
                prof->pair(&e0, &e1, 1, flops);
            }
            Syr2kProb<T, NBP, 64> p;
            p.A = w.A; p.ns = w.ns; p.Vp = w.Vp; p.Wp = w.Wp; p.ldp = w.ldp; p.sP = w.sP; p.t0 = t0;
            auto k = gemm_mfma_kernel<T, Syr2kProb<T, NBP, 64>>;
            const dim3 grid(tm * (tm + 1) / 2, 1, nbatch), block(256);
            if (timing) hipExtLaunchKernelGGL(k, grid, block, 0, st, e0, e1, 0, p);
            else hipLaunchKernelGGL(k, grid, block, 0, st, p);
        }
    }
    hipLaunchKernelGGL(sytrd_tail_kernel<T>, dim3(nbatch), dim3(SYTRD_TAIL_THREADS), 0, st, w);
}

template void sytrd_launch<double>(const SytrdWs<double>&, int, int, hipStream_t, const int*, LaunchProfiler*);
template void sytrd_launch<float>(const SytrdWs<float>&, int, int, hipStream_t, const int*, LaunchProfiler*);
