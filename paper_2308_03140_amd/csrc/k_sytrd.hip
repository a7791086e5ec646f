// Blocked Householder reduction of a real symmetric matrix to tridiagonal form
// (lower storage), the first stage of the diagonalisation Q = C Lambda C^T of
// eq:diagonalization (paper Sec. 2.1; Sec. 3.1 names the CPU libraries this
// replaces).
//
// Per panel of NBP columns, per column i (reflector H_i = I - tau v v^T with
// v(i+1) = 1 annihilating A(i+2:n, i)):
//   sytrd_symv   one pass over the not-yet-updated lower trailing matrix
//                A(i+1:n, i+1:n), 64x64 tiles, each element read once and used
//                for both y_R += A_RC v_C and y_C += A_RC^T v_R; also the panel
//                products p = W^T v, s = V^T v and the scalar v^T A v.  This
//                is the bandwidth-bound BLAS-2 half of the reduction.
//   sytrd_finish reduces the tile partials per 64-row block, forms
//                w = tau (A v - V p - W s) - (tau/2)(w^T v) v, and already
//                applies the panel to the next column (so the next reflector
//                can be built without another pass).
// After the panel: A(t0:n, t0:n) -= V W^T + W V^T on matrix cores
// (the BLAS-3 half).  All partial sums go through fixed-order reductions, so
// results are bitwise reproducible.  Every kernel takes a batch index
// (blockIdx.z) and the order of its own matrix, so one launch sequence
// serves a single large matrix and batches of uneven matrices alike.
#include "mbd_internal.h"
#include "gemm_mfma.h"
#include "mbd_kernels.h"

template <typename T>
__device__ __forceinline__ T refl_v(const T* col, int r, int s, int n, T scale) {
    if (r < s || r >= n) return T(0);
    return r == s ? T(1) : col[r] * scale;
}

// Reflector scalars from the updated column held in colbuf (LAPACK dlarfg
// convention: beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta).
template <typename T>
__device__ __forceinline__ void refl_scalars(const SytrdWs<T>& w, int b, int i, int n, T& beta,
                                             T& tau, T& scale) {
    const T* col = w.colbuf + (long long)b * w.sC;
    const T* np_ = w.normpart + (long long)b * w.sNP;
    const int nbk = (n + 63) >> 6;
    T xn2 = T(0);
    for (int R = (i >> 6); R < nbk; R++) xn2 += np_[R];
    const T alpha = col[i + 1];
    if (xn2 == T(0)) {
        tau = T(0); beta = alpha; scale = T(0);
    } else {
        T nrm = sqrt(alpha * alpha + xn2);
        beta = alpha >= T(0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = T(1) / (alpha - beta);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void sytrd_init_kernel(SytrdWs<T> w) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int R = blockIdx.x;
    const int nbk = (n + 63) >> 6;
    if (R >= nbk) return;
    const T* A = w.A.at(b);
    T* col = w.colbuf + (long long)b * w.sC;
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
    if (threadIdx.x == 0) w.normpart[(long long)b * w.sNP + R] = q;
}

template <typename T, int NBP>
__global__ __launch_bounds__(256) void sytrd_symv_kernel(SytrdWs<T> w, int i, int j, int Kt) {
    __shared__ T tb[64][65];
    __shared__ T rrow[4][64];
    __shared__ T red[4];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int slot = blockIdx.y * gridDim.x + blockIdx.x;
    T* PV = w.PV + (long long)b * w.sPV;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (i > n - 2) { if (tid == 0) PV[slot] = T(0); return; }
    const int s = i + 1;
    const int b0 = s >> 6;
    const int nbk = (n + 63) >> 6;
    const int C = b0 + blockIdx.y;
    const int q = blockIdx.x;
    if (C >= nbk) { if (tid == 0) PV[slot] = T(0); return; }
    const int nch = (nbk - C + Kt - 1) / Kt;
    if (q >= nch) { if (tid == 0) PV[slot] = T(0); return; }

    T* A = w.A.at(b);
    const int ld = w.A.ld;
    const T* col = w.colbuf + (long long)b * w.sC;
    T beta, tau, scale;
    refl_scalars(w, b, i, n, beta, tau, scale);

    T* Vp = w.Vp + (long long)b * w.sP;
    T* Wp = w.Wp + (long long)b * w.sP;
    const int ldp = w.ldp;

    if (q == 0) {
        // store v for the rows of block C (panel column j and the matrix column i)
        if (tid < 64) {
            const int r = C * 64 + tid;
            if (r < n) {
                T vr = refl_v(col, r, s, n, scale);
                Vp[r + (long long)j * ldp] = vr;
                if (r >= s) A[r + (long long)i * ld] = vr;
            }
        }
        if (C == b0 && tid == 0) {
            w.d[(long long)b * w.sD + i] = col[i];
            w.e[(long long)b * w.sD + i] = beta;
            w.tau[(long long)b * w.sD + i] = tau;
        }
        // panel products over the rows of block C
        T* PS = w.PS + (long long)b * w.sPS + (long long)C * (2 * NBP);
        const int r = C * 64 + lane;
        const bool rv = (r >= s && r < n);
        const T vr = rv ? refl_v(col, r, s, n, scale) : T(0);
        for (int k = wv; k < j; k += 4) {
            T pw = rv ? Wp[r + (long long)k * ldp] * vr : T(0);
            T pv = rv ? Vp[r + (long long)k * ldp] * vr : T(0);
            pw = wave_sum(pw);
            pv = wave_sum(pv);
            if (lane == 0) { PS[k] = pw; PS[NBP + k] = pv; }
        }
    }

    // column strip values
    T vc[16];
#pragma unroll
    for (int k = 0; k < 16; k++) vc[k] = refl_v(col, C * 64 + wv * 16 + k, s, n, scale);
    T cacc[16];
#pragma unroll
    for (int k = 0; k < 16; k++) cacc[k] = T(0);
    T vav = T(0);

    const int Rb = C + q * Kt;
    const int Re = min(Rb + Kt, nbk);
    const int c0 = C * 64 + wv * 16;
    T a[16], an[16];
    auto load_tile = [&](int R, T* dst) {
        const int r = R * 64 + lane;
        const bool rok = (r < n) && (r >= s);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const int c = c0 + k;
            const bool ok = rok && (c < n) && (c >= s) && (R > C || r >= c);
            dst[k] = ok ? A[r + (long long)c * ld] : T(0);
        }
    };
    load_tile(Rb, a);
    for (int R = Rb; R < Re; R++) {
        if (R + 1 < Re) load_tile(R + 1, an);
        const int r = R * 64 + lane;
        const T vr = refl_v(col, r, s, n, scale);
        T rs = T(0);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            rs += a[k] * vc[k];
            const bool offd = (R > C) || (r != c0 + k);
            cacc[k] += offd ? a[k] * vr : T(0);
        }
        rrow[wv][lane] = rs;
        __syncthreads();
        if (wv == 0) {
            T y = (rrow[0][lane] + rrow[1][lane]) + (rrow[2][lane] + rrow[3][lane]);
            w.P1[(long long)b * w.sP1 + ((long long)C * w.nbk_max + R) * 64 + lane] = y;
            vav += vr * y;
        }
        __syncthreads();
        if (R + 1 < Re) {
#pragma unroll
            for (int k = 0; k < 16; k++) a[k] = an[k];
        }
    }
    // column sums of the strip: transpose through LDS
#pragma unroll
    for (int k = 0; k < 16; k++) tb[wv * 16 + k][lane] = cacc[k];
    __syncthreads();
    {
        const int cc = tid & 63, part = tid >> 6;
        T ps = T(0);
#pragma unroll
        for (int l = 0; l < 16; l++) ps += tb[cc][part * 16 + l];
        rrow[part][cc] = ps;
    }
    __syncthreads();
    if (tid < 64) {
        T cs = (rrow[0][tid] + rrow[1][tid]) + (rrow[2][tid] + rrow[3][tid]);
        w.P2[(long long)b * w.sP2 + ((long long)C * w.maxchunk + q) * 64 + tid] = cs;
        vav += refl_v(col, C * 64 + tid, s, n, scale) * cs;
    }
    vav = block_sum256(vav, red);
    if (tid == 0) PV[slot] = vav;
}

template <typename T, int NBP>
__global__ __launch_bounds__(256) void sytrd_finish_kernel(SytrdWs<T> w, int i, int j, int Kt,
                                                           int nslots) {
    static_assert(2 * NBP <= 64, "panel products are reduced by one wavefront");
    __shared__ T sps[2 * NBP];
    __shared__ T rrow[4][64];
    __shared__ T red[4];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    if (i > n - 2) return;
    const int s = i + 1;
    const int b0 = s >> 6;
    const int nbk = (n + 63) >> 6;
    const int R = b0 + blockIdx.x;
    if (R >= nbk) return;
    const int tid = threadIdx.x, lane = tid & 63, part = tid >> 6;
    const T tau = w.tau[(long long)b * w.sD + i];
    const T* PV = w.PV + (long long)b * w.sPV;
    const T* PS = w.PS + (long long)b * w.sPS;
    const T* P1 = w.P1 + (long long)b * w.sP1;
    const T* P2 = w.P2 + (long long)b * w.sP2;
    T* Vp = w.Vp + (long long)b * w.sP;
    T* Wp = w.Wp + (long long)b * w.sP;
    const int ldp = w.ldp;
    T* A = w.A.at(b);
    const int ld = w.A.ld;

    // v^T A v
    T acc = T(0);
    for (int sl = tid; sl < nslots; sl += 256) acc += PV[sl];
    const T vAv = block_sum256(acc, red);
    // p = W^T v (k < NBP), s = V^T v (NBP + k)
    {
        T x = T(0);
        if (lane < 2 * NBP && (lane % NBP) < j)
            for (int Cb = b0 + part; Cb < nbk; Cb += 4) x += PS[(long long)Cb * (2 * NBP) + lane];
        rrow[part][lane] = x;
        __syncthreads();
        if (tid < 2 * NBP) sps[tid] = (rrow[0][tid] + rrow[1][tid]) + (rrow[2][tid] + rrow[3][tid]);
        __syncthreads();
    }
    T pts = T(0);
    for (int k = 0; k < j; k++) pts += sps[k] * sps[NBP + k];
    const T wtv = tau * (vAv - T(2) * pts);

    // y for the rows of block R
    const int nchR = (nbk - R + Kt - 1) / Kt;
    const int nitems = (R - b0 + 1) + nchR;
    T y = T(0);
    for (int it = part; it < nitems; it += 4) {
        if (it <= R - b0) {
            const int Cb = b0 + it;
            y += P1[((long long)Cb * w.nbk_max + R) * 64 + lane];
        } else {
            const int qq = it - (R - b0 + 1);
            y += P2[((long long)R * w.maxchunk + qq) * 64 + lane];
        }
    }
    __syncthreads();
    rrow[part][lane] = y;
    __syncthreads();
    y = (rrow[0][lane] + rrow[1][lane]) + (rrow[2][lane] + rrow[3][lane]);
    __syncthreads();
    const int r = R * 64 + lane;
    const bool rv = (r >= s && r < n);
    // corr = V p + W s over the previous panel columns
    T cr = T(0);
    if (rv)
        for (int k = part; k < j; k += 4)
            cr += Vp[r + (long long)k * ldp] * sps[k] + Wp[r + (long long)k * ldp] * sps[NBP + k];
    rrow[part][lane] = cr;
    __syncthreads();
    cr = (rrow[0][lane] + rrow[1][lane]) + (rrow[2][lane] + rrow[3][lane]);
    __syncthreads();
    const T vr = rv ? Vp[r + (long long)j * ldp] : T(0);
    const T wr = rv ? tau * (y - cr) - T(0.5) * tau * wtv * vr : T(0);
    if (part == 0 && r < n) Wp[r + (long long)j * ldp] = wr;

    // w(s), needed by every block for the update of column s
    T ws;
    {
        const int ls = s - b0 * 64;
        T ys = P1[((long long)b0 * w.nbk_max + b0) * 64 + ls];
        const int nch0 = (nbk - b0 + Kt - 1) / Kt;
        for (int qq = 0; qq < nch0; qq++) ys += P2[((long long)b0 * w.maxchunk + qq) * 64 + ls];
        T cs = T(0);
        for (int k = 0; k < j; k++)
            cs += Vp[s + (long long)k * ldp] * sps[k] + Wp[s + (long long)k * ldp] * sps[NBP + k];
        ws = tau * (ys - cs) - T(0.5) * tau * wtv;
    }
    // apply the panel (columns 0..j) to column s, rows of block R
    T u = T(0);
    if (rv) {
        for (int k = part; k < j; k += 4)
            u += Vp[r + (long long)k * ldp] * Wp[s + (long long)k * ldp] +
                 Wp[r + (long long)k * ldp] * Vp[s + (long long)k * ldp];
        if (part == 0) u += vr * ws + wr * T(1);
    }
    rrow[part][lane] = u;
    __syncthreads();
    u = (rrow[0][lane] + rrow[1][lane]) + (rrow[2][lane] + rrow[3][lane]);
    if (part == 0) {
        T cval = T(0);
        if (rv) {
            cval = A[r + (long long)s * ld] - u;
            w.colbuf[(long long)b * w.sC + r] = cval;
            if (s == n - 1) w.d[(long long)b * w.sD + n - 1] = cval;
        }
        T q2 = (r >= s + 2 && r < n) ? cval * cval : T(0);
        q2 = wave_sum(q2);
        if (lane == 0) w.normpart[(long long)b * w.sNP + R] = q2;
    }
}

// Trailing update A(t0:n, t0:n) -= V W^T + W V^T, lower tiles only.
template <typename T, int NBP>
struct Syr2kProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = true;
    MatBatch<T> A;
    const int* ns;
    const T* Vp; const T* Wp; int ldp; long long sP;
    int t0;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        t.batch = bz;
        const int mb = ns[bz] - t0;
        if (mb <= 0) return false;
        int ti, tj;
        lower_tile(bx, ti, tj);
        t.m0 = ti * GEMM_BM; t.n0 = tj * GEMM_BN; t.K = 2 * NBP;
        return t.m0 < mb;
    }
    __device__ T a(const GemmTile& t, int m, int k) const {
        const int r = t0 + m;
        if (r >= ns[t.batch]) return T(0);
        const long long o = (long long)t.batch * sP + r;
        return k < NBP ? Vp[o + (long long)k * ldp] : Wp[o + (long long)(k - NBP) * ldp];
    }
    __device__ T b(const GemmTile& t, int k, int nn) const {
        const int c = t0 + nn;
        if (c >= ns[t.batch]) return T(0);
        const long long o = (long long)t.batch * sP + c;
        return k < NBP ? Wp[o + (long long)k * ldp] : Vp[o + (long long)(k - NBP) * ldp];
    }
    __device__ void store(const GemmTile& t, int m, int nn, T v) const {
        const int r = t0 + m, c = t0 + nn, nb_ = ns[t.batch];
        if (r >= nb_ || c >= nb_ || r < c) return;
        A.at(t.batch)[r + (long long)c * A.ld] -= v;
    }
};

template <typename T>
int sytrd_tiles_per_chunk(int nbk_trail, int nbatch) {
    long long tiles = (long long)nbk_trail * (nbk_trail + 1) / 2 * nbatch;
    long long kt = tiles / 1536;
    if (kt < 1) kt = 1;
    if (kt > 8) kt = 8;
    return (int)kt;
}

template <typename T>
void sytrd_launch(const SytrdWs<T>& w, int nbatch, int nmax, hipStream_t st, const int* ns_host,
                  LaunchProfiler* prof) {
    constexpr int NBP = SYTRD_NBP;
    const bool timing = prof && prof->enabled && ns_host;
    const int nbk_max = w.nbk_max;
    hipLaunchKernelGGL(sytrd_init_kernel<T>, dim3(nbk_max, 1, nbatch), dim3(256), 0, st, w);
    int k0 = 0;
    for (int i = 0; i + 2 <= nmax; i++) {
        const int j = i - k0;
        const int b0 = (i + 1) >> 6;
        const int nbt = nbk_max - b0;
        const int Kt = sytrd_tiles_per_chunk<T>(nbt, nbatch);
        const int gx = (nbt + Kt - 1) / Kt;
        if (timing) prof->begin(st);
        hipLaunchKernelGGL((sytrd_symv_kernel<T, NBP>), dim3(gx, nbt, nbatch), dim3(256), 0, st, w, i, j,
                           Kt);
        if (timing) {
            // algorithmic traffic: the lower trailing triangle, read once
            double bytes = 0;
            for (int b = 0; b < nbatch; b++) {
                const double m = ns_host[b] - i - 1;
                if (m > 0) bytes += m * (m + 1) * 0.5 * sizeof(T);
            }
            prof->end(st, 0, bytes);
        }
        hipLaunchKernelGGL((sytrd_finish_kernel<T, NBP>), dim3(nbt, 1, nbatch), dim3(256), 0, st, w, i, j,
                           Kt, gx * nbt);
        if (j == NBP - 1 && i + 2 < nmax) {
            const int t0 = k0 + NBP;
            const int tm = (nmax - t0 + 63) / 64;
            Syr2kProb<T, NBP> p;
            p.A = w.A; p.ns = w.ns; p.Vp = w.Vp; p.Wp = w.Wp; p.ldp = w.ldp; p.sP = w.sP; p.t0 = t0;
            if (timing) prof->begin(st);
            hipLaunchKernelGGL((gemm_mfma_kernel<T, Syr2kProb<T, NBP>>), dim3(tm * (tm + 1) / 2, 1, nbatch),
                               dim3(256), 0, st, p);
            if (timing) {
                double flops = 0;
                for (int b = 0; b < nbatch; b++) {
                    const double m = ns_host[b] - t0;
                    if (m > 0) flops += 2.0 * (2 * NBP) * m * (m + 1) * 0.5;
                }
                prof->end(st, 1, flops);
            }
            k0 += NBP;
        }
    }
}

template void sytrd_launch<double>(const SytrdWs<double>&, int, int, hipStream_t, const int*, LaunchProfiler*);
template void sytrd_launch<float>(const SytrdWs<float>&, int, int, hipStream_t, const int*, LaunchProfiler*);
