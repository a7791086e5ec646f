// Symmetric tridiagonal eigensolver: divide and conquer (Cuppen's tearing
// with rank-one merges), eigenvectors by the Loewner-formula recomputation of
// the updating vector (Gu & Eisenstat) so they are orthogonal to working
// precision, deflation of negligible z components and of close pole pairs
// (Givens rotation), and merges multiplied out on matrix cores.  Second
// stage of eq:diagonalization (paper Sec. 2.1).
//
// The tree is fixed bottom-up: leaves are single diagonal entries (every
// off-diagonal torn: d_p - |e_{p-1}| - |e_p|), level L merges neighbouring
// blocks [o, o+2^(L-1)) and [o+2^(L-1), o+2^L).  Each level is a fixed set of
// launches over all merges of all matrices of a batch, so the sequence is
// independent of the data and can be captured once in a HIP graph.
//
// Secular roots: one wavefront per root, a safeguarded Newton iteration in the
// variable mu = lambda - d_origin, where the origin is the pole the root is
// closer to, so differences d_i - lambda are formed without cancellation; the
// sign of the secular function keeps a bracket and a bisection step replaces
// any Newton step that leaves it.
#include <algorithm>

#include "mbd_internal.h"
#include "gemm_mfma.h"
#include "mbd_kernels.h"

struct MergeInfo {
    int o, k1, k;
    __device__ __forceinline__ bool active() const { return k > k1; }
};

__device__ __forceinline__ MergeInfo merge_of(int p, int lev, int n) {
    MergeInfo m;
    const int size = 1 << lev, half = size >> 1;
    m.o = (p >> lev) << lev;
    m.k1 = min(half, n - m.o);
    m.k = min(size, n - m.o);
    return m;
}

template <typename T>
__global__ __launch_bounds__(256) void stedc_init_kernel(StedcWs<T> w) {
    __shared__ double red[4];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const T* d = w.d_in + (long long)b * w.sDin;
    const T* e = w.e_in + (long long)b * w.sDin;
    double mx = 0.0;
    for (int p = threadIdx.x; p < n; p += 256) {
        mx = fmax(mx, fabs((double)d[p]));
        if (p < n - 1) mx = fmax(mx, fabs((double)e[p]));
    }
    mx = block_max256(mx, red);
    if (mx == 0.0) mx = 1.0;
    const double inv = 1.0 / mx;
    double* D = w.D + (long long)b * w.sV;
    double* E = w.E + (long long)b * w.sV;
    for (int p = threadIdx.x; p < n; p += 256) {
        const double el = p > 0 ? fabs((double)e[p - 1]) * inv : 0.0;
        const double er = p < n - 1 ? fabs((double)e[p]) * inv : 0.0;
        D[p] = (double)d[p] * inv - el - er;
        E[p] = p < n - 1 ? (double)e[p] * inv : 0.0;
    }
    if (threadIdx.x == 0) w.scale[b] = mx;
}

// Z0 = I, Z1 = 0 on the n x n block; one workgroup per column (a grid of
// row chunks per column left most workgroups of a batch of small matrices
// with nothing to do)
template <typename T>
__global__ __launch_bounds__(256) void stedc_fill_kernel(StedcWs<T> w) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int c = blockIdx.x;
    if (c >= n) return;
    T* z0 = w.Z0.at(b) + (long long)c * w.Z0.ld;
    T* z1 = w.Z1.at(b) + (long long)c * w.Z1.ld;
    for (int r = threadIdx.x; r < n; r += 256) {
        z0[r] = (r == c) ? T(1) : T(0);
        z1[r] = T(0);
    }
}

// merge inputs: z vector, sorted poles, permutation
template <typename T>
__global__ __launch_bounds__(256) void stedc_setup_kernel(StedcWs<T> w, int lev, int src) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    const MergeInfo m = merge_of(p, lev, n);
    if (!m.active()) return;
    const MatBatch<T>& Zc = src ? w.Z1 : w.Z0;
    const T* Zb = Zc.at(b);
    const long long ld = Zc.ld;
    const double* D = w.D + (long long)b * w.sV;
    const double ee = w.E[(long long)b * w.sV + m.o + m.k1 - 1];
    const double sg = ee >= 0.0 ? 1.0 : -1.0;
    const int lp = p - m.o;
    const double dp = D[p];
    const double inv_sqrt2 = 0.70710678118654752440;
    double zp = lp < m.k1 ? (double)Zb[(m.o + m.k1 - 1) + (long long)p * ld]
                          : sg * (double)Zb[(m.o + m.k1) + (long long)p * ld];
    zp *= inv_sqrt2;
    int rank;
    if (lp < m.k1) {
        // elements of the second half strictly below dp
        int lo = m.o + m.k1, hi = m.o + m.k;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (D[mid] < dp) lo = mid + 1; else hi = mid; }
        rank = lp + (lo - (m.o + m.k1));
    } else {
        int lo = m.o, hi = m.o + m.k1;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (D[mid] <= dp) lo = mid + 1; else hi = mid; }
        rank = (lp - m.k1) + (lo - m.o);
    }
    const long long base = (long long)b * w.sV + m.o;
    w.ds[base + rank] = dp;
    w.zs[base + rank] = zp;
    w.perm[base + rank] = lp;
    if (lp == 0) w.rho[base] = 2.0 * fabs(ee);
}

// sequential deflation scan, one thread per merge
template <typename T>
__global__ __launch_bounds__(64) void stedc_deflate_kernel(StedcWs<T> w, int lev) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int t = blockIdx.x * 64 + threadIdx.x;
    const int o = t << lev;
    if (o >= n) return;
    const MergeInfo m = merge_of(o, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + o;
    double* ds = w.ds + base;
    double* zs = w.zs + base;
    const int* perm = w.perm + base;
    int* ndpos = w.ndpos + base;
    int* dfpos = w.dfpos + base;
    const double rho = w.rho[base];
    double dmax = 0.0, zmax = 0.0;
    for (int j = 0; j < m.k; j++) { dmax = fmax(dmax, fabs(ds[j])); zmax = fmax(zmax, fabs(zs[j])); }
    // deflation at the precision of the eigenvector matrices
    const double tol = 8.0 * (double)num_limits<T>::eps * fmax(dmax, zmax);
    int* sup = w.sup + base;
    int K = 0, ndf = 0, nrot = 0, pj = -1, spj = 0;
    for (int jx = 0; jx < m.k; jx++) {
        if (rho * fabs(zs[jx]) <= tol) { dfpos[ndf++] = jx; continue; }
        const int sjx = perm[jx] < m.k1 ? 1 : 2;
        if (pj < 0) { pj = jx; spj = sjx; continue; }
        double s = zs[pj], c = zs[jx];
        const double tau = sqrt(c * c + s * s);
        const double tt = ds[jx] - ds[pj];
        c /= tau;
        s = -s / tau;
        if (fabs(tt * c * s) <= tol) {
            zs[jx] = tau;
            zs[pj] = 0.0;
            w.rp[base + nrot] = perm[pj];
            w.rq[base + nrot] = perm[jx];
            w.rc[base + nrot] = c;
            w.rs[base + nrot] = s;
            nrot++;
            const double dpj = ds[pj] * c * c + ds[jx] * s * s;
            ds[jx] = ds[pj] * s * s + ds[jx] * c * c;
            ds[pj] = dpj;
            dfpos[ndf++] = pj;
            pj = jx;
            spj |= sjx;  // the survivor carries both columns' rows
        } else {
            sup[K] = spj;
            ndpos[K++] = pj;
            pj = jx;
            spj = sjx;
        }
    }
    if (pj >= 0) { sup[K] = spj; ndpos[K++] = pj; }
    for (int kk = 0; kk < K; kk++) {
        w.dn[base + kk] = ds[ndpos[kk]];
        w.zn[base + kk] = zs[ndpos[kk]];
    }
    w.Kcnt[base] = K;
    w.rotcnt[base] = nrot;
}

// Exclusive prefix sum of one int per thread over a 256-thread block; the
// total comes back through *total.  tmp holds 256 ints of LDS.
__device__ __forceinline__ int block_exscan256(int v, int* tmp, int* total) {
    const int tid = threadIdx.x;
    __syncthreads();
    tmp[tid] = v;
    for (int off = 1; off < 256; off <<= 1) {
        __syncthreads();
        const int x = tid >= off ? tmp[tid - off] : 0;
        __syncthreads();
        tmp[tid] += x;
    }
    __syncthreads();
    *total = tmp[255];
    const int r = tmp[tid] - v;
    __syncthreads();
    return r;
}

// The same deflation for merges of up to DEFL_LDS entries, one workgroup per
// merge, with the poles and the updating vector in LDS and the scan made
// parallel.  The z-deflation flags depend only on the original values; so
// does the rotation test of every adjacent pair of the remaining entries
// unless the pair before it rotated.  Those tests are precomputed in
// parallel; one thread then walks only the candidate pairs and the chains of
// rotations that follow them (re-testing with the rotated values), skipping
// 16 flags per LDS read.  The output positions of the sequential scan
// (deflated entries in scan order, kept entries in list order, rotations in
// order) follow from block prefix sums, so the results are the sequential
// scan's, bit for bit.
#define DEFL_LDS 7168
template <typename T>
__global__ __launch_bounds__(256) void stedc_deflate_lds_kernel(StedcWs<T> w, int lev) {
    static_assert((DEFL_LDS + 255) / 256 <= 32, "one 32-bit z-deflation mask per thread chunk");
    __shared__ double sd[DEFL_LDS], sz[DEFL_LDS];
    __shared__ int sL[DEFL_LDS];
    __shared__ __align__(16) unsigned char cand[DEFL_LDS];
    __shared__ unsigned char rotf[DEFL_LDS];
    __shared__ int tmp[256];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int o = blockIdx.x << lev;
    if (o >= n) return;
    const MergeInfo m = merge_of(o, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + o;
    double* ds = w.ds + base;
    double* zs = w.zs + base;
    const int* perm = w.perm + base;
    int* dfpos = w.dfpos + base;
    const int k = m.k;
    double dmax = 0.0, zmax = 0.0;
    for (int j = tid; j < k; j += 256) {
        const double d = ds[j], z = zs[j];
        sd[j] = d;
        sz[j] = z;
        dmax = fmax(dmax, fabs(d));
        zmax = fmax(zmax, fabs(z));
    }
    dmax = block_max256(dmax, red);
    zmax = block_max256(zmax, red);
    // deflation at the precision of the eigenvector matrices
    const double tol = 8.0 * (double)num_limits<T>::eps * fmax(dmax, zmax);
    const double rho = w.rho[base];

    // z-deflation flags of this thread's contiguous chunk, and the list L of
    // the remaining entries in index order
    const int per = (k + 255) / 256;
    const int j0 = min(k, tid * per), j1 = min(k, j0 + per);
    unsigned zmask = 0;
    int cnt = 0;
    for (int j = j0; j < j1; j++) {
        if (rho * fabs(sz[j]) <= tol) zmask |= 1u << (j - j0);
        else cnt++;
    }
    int K0;
    const int t0 = block_exscan256(cnt, tmp, &K0);
    {
        int t = t0;
        for (int j = j0; j < j1; j++)
            if (!((zmask >> (j - j0)) & 1u)) sL[t++] = j;
    }
    __syncthreads();
    // rotation tests of adjacent list pairs on the original values
    for (int t = tid; t < K0; t += 256) {
        unsigned char c = 0;
        if (t >= 1) {
            const int pj = sL[t - 1], jx = sL[t];
            double sn = sz[pj], cs = sz[jx];
            const double tau = sqrt(cs * cs + sn * sn);
            const double tt = sd[jx] - sd[pj];
            cs /= tau;
            sn = -sn / tau;
            c = fabs(tt * cs * sn) <= tol ? 1 : 0;
        }
        cand[t] = c;
        rotf[t] = 0;
    }
    for (int t = K0 + tid; t < ((K0 + 15) & ~15); t += 256) cand[t] = 0;  // pad to a 16-flag boundary
    __syncthreads();
    if (tid == 0) {
        int nrot = 0;
        bool prev = false;  // the pair before rotated: re-test with its values
        int t = 1;
        while (t < K0) {
            if (!prev) {
                if ((t & 15) == 0) {
                    const uint4 q = *reinterpret_cast<const uint4*>(&cand[t]);
                    if ((q.x | q.y | q.z | q.w) == 0u) { t += 16; continue; }
                }
                if (!cand[t]) { t++; continue; }
            }
            const int pj = sL[t - 1], jx = sL[t];
            double sn = sz[pj], cs = sz[jx];
            const double tau = sqrt(cs * cs + sn * sn);
            const double tt = sd[jx] - sd[pj];
            cs /= tau;
            sn = -sn / tau;
            if (fabs(tt * cs * sn) <= tol) {
                sz[jx] = tau;
                sz[pj] = 0.0;
                w.rp[base + nrot] = perm[pj];
                w.rq[base + nrot] = perm[jx];
                w.rc[base + nrot] = cs;
                w.rs[base + nrot] = sn;
                nrot++;
                const double dpj = sd[pj] * cs * cs + sd[jx] * sn * sn;
                sd[jx] = sd[pj] * sn * sn + sd[jx] * cs * cs;
                sd[pj] = dpj;
                rotf[t] = 1;
                prev = true;
            } else {
                prev = false;
            }
            t++;
        }
        w.rotcnt[base] = nrot;
    }
    __syncthreads();
    // rows carried by the kept entry at list position u: its own half's and
    // those of the entries rotated into it (the chain of rotated pairs ending
    // at u)
    auto chain_support = [&](int u) {
        int sp = perm[sL[u]] < m.k1 ? 1 : 2;
        for (int q = u; q >= 1 && rotf[q]; q--) sp |= perm[sL[q - 1]] < m.k1 ? 1 : 2;
        return sp;
    };
    // output positions: at index j the sequential scan appends j to the
    // deflated list (z-deflated), or the list predecessor L[t-1] of j = L[t]
    // to the deflated list (the pair rotated) or to the kept list (it did not)
    int cdf = 0, cnd = 0;
    {
        int t = t0;
        for (int j = j0; j < j1; j++) {
            if ((zmask >> (j - j0)) & 1u) { cdf++; continue; }
            if (t >= 1) { if (rotf[t]) cdf++; else cnd++; }
            t++;
        }
    }
    int ndf_tot, nnd_tot;
    int odf = block_exscan256(cdf, tmp, &ndf_tot);
    int ond = block_exscan256(cnd, tmp, &nnd_tot);
    {
        int t = t0;
        for (int j = j0; j < j1; j++) {
            if ((zmask >> (j - j0)) & 1u) { dfpos[odf++] = j; continue; }
            if (t >= 1) {
                const int p = sL[t - 1];
                if (rotf[t]) {
                    dfpos[odf++] = p;
                } else {
                    w.ndpos[base + ond] = p;
                    w.dn[base + ond] = sd[p];
                    w.zn[base + ond] = sz[p];
                    w.sup[base + ond] = chain_support(t - 1);
                    ond++;
                }
            }
            t++;
        }
    }
    const int K = K0 > 0 ? nnd_tot + 1 : 0;
    if (tid == 0) {
        if (K0 > 0) {
            const int p = sL[K0 - 1];
            w.ndpos[base + K - 1] = p;
            w.dn[base + K - 1] = sd[p];
            w.zn[base + K - 1] = sz[p];
            w.sup[base + K - 1] = chain_support(K0 - 1);
        }
        w.Kcnt[base] = K;
    }
    for (int j = tid; j < k; j += 256) {
        ds[j] = sd[j];
        zs[j] = sz[j];
    }
}

// per merge, the kept columns whose rows reach the first half (ltop) and the
// second half (lbot), each in kept order; one workgroup per merge
template <typename T>
__global__ __launch_bounds__(256) void stedc_split_kernel(StedcWs<T> w, int lev) {
    __shared__ int tmp[256];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int o = blockIdx.x << lev;
    if (o >= n) return;
    const MergeInfo m = merge_of(o, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + o;
    const int K = w.Kcnt[base];
    const int per = (K + 255) / 256;
    const int q0 = min(K, (int)threadIdx.x * per), q1 = min(K, q0 + per);
    int ct = 0, cb = 0;
    for (int q = q0; q < q1; q++) {
        const int sp = w.sup[base + q];
        ct += sp & 1;
        cb += sp >> 1;
    }
    int nt, nb;
    int ot = block_exscan256(ct, tmp, &nt);
    int ob = block_exscan256(cb, tmp, &nb);
    for (int q = q0; q < q1; q++) {
        const int sp = w.sup[base + q];
        const int col = w.perm[base + w.ndpos[base + q]];
        if (sp & 1) { w.ltop[base + ot] = q; w.ctop[base + ot] = col; ot++; }
        if (sp & 2) { w.lbot[base + ob] = q; w.cbot[base + ob] = col; ob++; }
    }
    if (threadIdx.x == 0) {
        w.ktop[base] = nt;
        w.kbot[base] = nb;
    }
}

// apply the deflation rotations to the eigenvector columns of the merge
template <typename T>
__global__ __launch_bounds__(256) void stedc_rotate_kernel(StedcWs<T> w, int lev, int src) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const MergeInfo m = merge_of(r, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + m.o;
    const int nrot = w.rotcnt[base];
    if (nrot == 0) return;
    const MatBatch<T>& Zc = src ? w.Z1 : w.Z0;
    T* Zb = Zc.at(b);
    const long long ld = Zc.ld;
    for (int q = 0; q < nrot; q++) {
        const long long ca = m.o + w.rp[base + q], cb = m.o + w.rq[base + q];
        const double c = w.rc[base + q], s = w.rs[base + q];
        const double x = Zb[r + ca * ld], y = Zb[r + cb * ld];
        Zb[r + ca * ld] = (T)(c * x + s * y);
        Zb[r + cb * ld] = (T)(c * y - s * x);
    }
}

// secular equation 1 + rho sum z_i^2/(d_i - lambda) = 0, one wavefront per root
template <typename T>
__global__ __launch_bounds__(256) void stedc_secular_kernel(StedcWs<T> w, int lev) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    const MergeInfo m = merge_of(p, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + m.o;
    const int K = w.Kcnt[base];
    const int jx = p - m.o;
    if (jx >= K) return;
    const double* dn = w.dn + base;
    const double* zn = w.zn + base;
    const double rho = w.rho[base];
    int org;
    double lo, hi, x0 = 0.0;
    bool guess = false;
    if (jx < K - 1) {
        const double mid = 0.5 * (dn[jx] + dn[jx + 1]);
        double f = 0.0;
        for (int i = lane; i < K; i += 64) f += zn[i] * zn[i] / (dn[i] - mid);
        const double fs = wave_sum(f);
        f = 1.0 + rho * fs;
        if (f >= 0.0) { org = jx; lo = 0.0; hi = mid - dn[jx]; }
        else { org = jx + 1; lo = mid - dn[jx + 1]; hi = 0.0; }
        // starting point: the root of the two nearest poles' terms with the
        // others frozen at their values at the midpoint, a quadratic in
        // x = lambda - d_org (the bracket and its bisection fallback stay)
        const double za = zn[jx] * zn[jx], zb = zn[jx + 1] * zn[jx + 1];
        const double c = 1.0 + rho * (fs - za / (dn[jx] - mid) - zb / (dn[jx + 1] - mid));
        const double da = dn[jx] - dn[org], db = dn[jx + 1] - dn[org];
        const double B = -(c * (da + db) + rho * (za + zb));
        const double C = c * da * db + rho * (za * db + zb * da);
        const double disc = B * B - 4.0 * c * C;
        if (c != 0.0 && disc >= 0.0) {
            const double q = -0.5 * (B + (B >= 0.0 ? sqrt(disc) : -sqrt(disc)));
            const double r1 = q / c, r2 = q != 0.0 ? C / q : r1;
            if (r1 > lo && r1 < hi) { x0 = r1; guess = true; }
            else if (r2 > lo && r2 < hi) { x0 = r2; guess = true; }
        }
    } else {
        double z2 = 0.0;
        for (int i = lane; i < K; i += 64) z2 += zn[i] * zn[i];
        org = K - 1; lo = 0.0; hi = rho * wave_sum(z2);
    }
    const double dorg = dn[org];
    // safeguarded Newton in mu: f is increasing between the poles, so the sign
    // of f(x) keeps the bracket [lo, hi]; a Newton step leaving it is replaced
    // by bisection.  Stops when |f| is at its rounding level or the bracket
    // is relatively tight (the Loewner step only needs d_i - lambda =
    // (d_i - d_org) - mu to relative accuracy).
    double x = guess ? x0 : 0.5 * (lo + hi);
    for (int it = 0; it < 120; it++) {
        double f = 0.0, fp = 0.0, fa = 0.0;
        for (int i = lane; i < K; i += 64) {
            const double t = 1.0 / ((dn[i] - dorg) - x);
            const double z2 = zn[i] * zn[i];
            f += z2 * t;
            fp += z2 * t * t;
            fa += fabs(z2 * t);
        }
        f = 1.0 + rho * wave_sum(f);
        fp = rho * wave_sum(fp);
        fa = 1.0 + rho * wave_sum(fa);
        if (f < 0.0) lo = x; else hi = x;
        if (fabs(f) <= 4.0 * num_limits<double>::eps * fa) break;
        if (hi - lo <= 4.0 * num_limits<double>::eps * fmax(fabs(lo), fabs(hi))) break;
        double xn = x - f / fp;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (xn == x) break;
        x = xn;
    }
    if (lane == 0) {
        const double mu = x;
        w.org[base + jx] = org;
        w.mu[base + jx] = mu;
        w.lam[base + jx] = dorg + mu;
    }
}

// Loewner formula for the updating vector consistent with the computed roots
// Loewner updating vector zhat_i = sqrt(prod_j (lambda_j - d_i) / (d_j - d_i)
// * (lambda_i - d_i) / rho), signed like z_i; one wavefront per i, the
// factors strided over the lanes and multiplied across the wave.
template <typename T>
__global__ __launch_bounds__(256) void stedc_zhat_kernel(StedcWs<T> w, int lev) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    const MergeInfo m = merge_of(p, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + m.o;
    const int K = w.Kcnt[base];
    const int i = p - m.o;
    if (i >= K) return;
    const double* dn = w.dn + base;
    const double* mu = w.mu + base;
    const int* org = w.org + base;
    const double di = dn[i];
    double prod = 1.0;
    for (int j = lane; j < K; j += 64)
        if (j != i) prod *= ((dn[org[j]] - di) + mu[j]) / (dn[j] - di);
    prod = wave_prod(prod) * (((dn[org[i]] - di) + mu[i]) / w.rho[base]);
    if (lane == 0) {
        const double z = sqrt(fmax(prod, 0.0));
        w.zh[base + i] = w.zn[base + i] >= 0.0 ? z : -z;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void stedc_vectors_kernel(StedcWs<T> w, int lev) {
    __shared__ double red[4];
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int p = blockIdx.x;
    if (p >= n) return;
    const MergeInfo m = merge_of(p, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + m.o;
    const int K = w.Kcnt[base];
    const int jx = p - m.o;
    if (jx >= K) return;
    const double* dn = w.dn + base;
    const double* zh = w.zh + base;
    const double dorg = dn[w.org[base + jx]];
    const double muj = w.mu[base + jx];
    double ss = 0.0;
    for (int i = threadIdx.x; i < K; i += 256) {
        const double u = zh[i] / ((dn[i] - dorg) - muj);
        ss += u * u;
    }
    ss = block_sum256(ss, red);
    const double inv = 1.0 / sqrt(ss);
    T* Ub = w.U.at(b);
    const long long ld = w.U.ld;
    for (int i = threadIdx.x; i < K; i += 256) {
        const double u = zh[i] / ((dn[i] - dorg) - muj);
        Ub[(m.o + i) + (long long)(m.o + jx) * ld] = (T)(u * inv);
    }
}

// final ascending order of the merged spectrum (roots and deflated values)
// position of every eigenvalue of the merge in ascending order (ties by
// index); one wavefront per value, the comparisons strided over the lanes
template <typename T>
__global__ __launch_bounds__(256) void stedc_order_kernel(StedcWs<T> w, int lev) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= n) return;
    const MergeInfo m = merge_of(p, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + m.o;
    const int K = w.Kcnt[base];
    const double* lam = w.lam + base;
    const double* ds = w.ds + base;
    const int* dfpos = w.dfpos + base;
    const int it = p - m.o;
    auto val = [&](int q) -> double { return q < K ? lam[q] : ds[dfpos[q - K]]; };
    const double v = val(it);
    int cnt = 0;
    for (int q = lane; q < m.k; q += 64) {
        const double u = val(q);
        cnt += (u < v) || (u == v && q < it);
    }
    const int rank = (int)wave_sum((double)cnt);
    if (lane == 0) {
        if (it < K) w.outnd[base + it] = rank;
        else w.outdf[base + it - K] = rank;
        w.D[base + rank] = v;
    }
}

// merged eigenvectors: Zn[:, outnd[j]] = Zc[:, perm[ndpos[.]]] U[:, j], in
// TS x TS output tiles
template <typename T, int TS>
struct DcMergeProb {
    // Zn(rows of half h, outnd(j)) = sum over the kept columns q with rows in
    // half h of Zc(rows of h, column of q) U(q, j): the merge's eigenvector
    // block is block diagonal except for columns rotated across the halves,
    // so each half multiplies only its own columns (half the flops of the
    // dense product when no rotation crosses).  grid x = half x row tiles x
    // column tiles, y = merge, z = matrix.
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = false;
    static constexpr bool K_UNIFORM = true;  // A's column comes from a q-indexed table
    const int* ns;
    int lev, tdim, tdh;
    MatBatch<T> Zc, Zn, U;
    const int* outnd; const int* Kcnt; const int* ltop; const int* lbot; const int* ktop; const int* kbot;
    const int* ctop; const int* cbot;
    long long sV;
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        t.batch = bz;
        const int n = ns[bz];
        const int o = by << lev;
        if (o >= n) return false;
        const MergeInfo m = merge_of(o, lev, n);
        if (!m.active()) return false;
        const long long base = (long long)bz * sV + o;
        const int h = bx / (tdh * tdim), rem = bx - h * (tdh * tdim);
        const int K = Kcnt[base];
        t.m0 = (rem / tdim) * TS;
        t.n0 = (rem % tdim) * TS;
        t.o = o;
        t.e0 = h ? m.k1 : 0;                  // first row of the half
        t.k = h ? m.k - m.k1 : m.k1;          // rows of the half
        t.K = h ? kbot[base] : ktop[base];    // columns with rows there
        t.e1 = K;
        return t.m0 < t.k && t.n0 < K;        // a half with no columns writes zeros
    }
    __device__ T a(const GemmTile& t, int mm, int q) const {
        if (mm >= t.k || q >= t.K) return T(0);
        const long long base = (long long)t.batch * sV + t.o;
        const long long c = t.o + (t.e0 ? cbot : ctop)[base + q];
        return Zc.at(t.batch)[(t.o + t.e0 + mm) + c * Zc.ld];
    }
    __device__ T b(const GemmTile& t, int q, int jj) const {
        if (q >= t.K || jj >= t.e1) return T(0);
        const long long base = (long long)t.batch * sV + t.o;
        const int kk = (t.e0 ? lbot : ltop)[base + q];
        return U.at(t.batch)[(t.o + kk) + (long long)(t.o + jj) * U.ld];
    }
    __device__ void store(const GemmTile& t, int mm, int jj, T v) const {
        if (mm >= t.k || jj >= t.e1) return;
        const long long base = (long long)t.batch * sV + t.o;
        const long long c = t.o + outnd[base + jj];
        Zn.at(t.batch)[(t.o + t.e0 + mm) + c * Zn.ld] = v;
    }
};

// Operands of the split-FP16 merge product, gathered into contiguous columns
// per half h of a merge at origin o (layout of U, rows and columns counted
// from o):
//   GAh(o + mm, o + q) = Zc(o + e0_h + mm, o + c_h(q)), mm < rows of h, q < K_h
//   GBh(o + q, o + jj) = U(o + l_h(q), o + jj),          q < K_h, jj < K
// grid x = column, y = merge, z = matrix.
template <typename T>
__global__ __launch_bounds__(256) void stedc_gather_merge_kernel(StedcWs<T> w, int lev, int src) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int o = blockIdx.y << lev;
    if (o >= n) return;
    const MergeInfo m = merge_of(o, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + o;
    const int x = blockIdx.x;
    const int K = w.Kcnt[base], kt = w.ktop[base], kb = w.kbot[base];
    const long long ld = w.U.ld;
    const long long off = (long long)b * w.U.stride + (o + (long long)x) * ld + o;
    if (x < K) {
        const T* Uc = w.U.at(b) + (o + (long long)x) * ld + o;
        for (int q = threadIdx.x; q < kt; q += 256) w.GB0[off + q] = Uc[w.ltop[base + q]];
        for (int q = threadIdx.x; q < kb; q += 256) w.GB1[off + q] = Uc[w.lbot[base + q]];
    }
    const MatBatch<T>& Zc = src ? w.Z1 : w.Z0;
    if (x < kt) {
        const T* Zcol = Zc.at(b) + (o + (long long)w.ctop[base + x]) * Zc.ld + o;
        for (int r = threadIdx.x; r < m.k1; r += 256) w.GA0[off + r] = Zcol[r];
    }
    if (x < kb) {
        const T* Zcol = Zc.at(b) + (o + (long long)w.cbot[base + x]) * Zc.ld + o + m.k1;
        for (int r = threadIdx.x; r < m.k - m.k1; r += 256) w.GA1[off + r] = Zcol[r];
    }
}

// The merge product of DcMergeProb on the FP16 matrix cores with split
// operands (FP32 only, 128 x 128 tiles), reading the operands gathered by
// stedc_gather_merge_kernel (B 16 bytes at a time).  Both hold entries of
// orthonormal columns (|z| <= 1), so a fixed 2^14 keeps them in FP16's
// normal range.
struct DcMergeSplitProb {
    const int* ns;
    int lev, tdim, tdh;
    MatBatch<float> Zn, GA0, GA1, GB0, GB1;
    const int* outnd; const int* Kcnt; const int* ktop; const int* kbot;
    long long sV;
    __device__ bool tile(int bx, int by, int bz, GemmTile& t) const {
        t.batch = bz;
        const int n = ns[bz];
        const int o = by << lev;
        if (o >= n) return false;
        const MergeInfo m = merge_of(o, lev, n);
        if (!m.active()) return false;
        const long long base = (long long)bz * sV + o;
        const int h = bx / (tdh * tdim), rem = bx - h * (tdh * tdim);
        const int K = Kcnt[base];
        t.m0 = (rem / tdim) * 128;
        t.n0 = (rem % tdim) * 128;
        t.o = o;
        t.e0 = h ? m.k1 : 0;                  // first row of the half
        t.k = h ? m.k - m.k1 : m.k1;          // rows of the half
        t.K = h ? kbot[base] : ktop[base];    // columns with rows there
        t.e1 = K;
        return t.m0 < t.k && t.n0 < K;
    }
    __device__ float a_scale(const GemmTile&, int) const { return 16384.0f; }
    __device__ float b_scale(const GemmTile&, int) const { return 16384.0f; }
    __device__ float a(const GemmTile& t, int mm, int q) const {
        if (mm >= t.k || q >= t.K) return 0.0f;
        const MatBatch<float>& G = t.e0 ? GA1 : GA0;
        return G.at(t.batch)[(t.o + mm) + (long long)(t.o + q) * G.ld];
    }
    // rows q .. q+3 of gathered column jj (clamped to a listed column); the
    // buffers carry 64 elements of padding past the last matrix
    __device__ gemm_f32x4 b4(const GemmTile& t, int q, int jj) const {
        const MatBatch<float>& G = t.e0 ? GB1 : GB0;
        const int jc = jj < t.e1 ? jj : t.e1 - 1;
        return *reinterpret_cast<const gemm_f32x4*>(G.at(t.batch) + (t.o + q) + (long long)(t.o + jc) * G.ld);
    }
    __device__ bool b_keep(const GemmTile& t, int q, int jj) const { return q < t.K && jj < t.e1; }
    __device__ void store(const GemmTile& t, int mm, int jj, float v) const {
        if (mm >= t.k || jj >= t.e1) return;
        const long long base = (long long)t.batch * sV + t.o;
        const long long c = t.o + outnd[base + jj];
        Zn.at(t.batch)[(t.o + t.e0 + mm) + c * Zn.ld] = v * (1.0f / (16384.0f * 16384.0f));
    }
};

// same product for small merges (k <= 64): one workgroup per merge
template <typename T>
__global__ __launch_bounds__(256) void stedc_small_merge_kernel(StedcWs<T> w, int lev, int src) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int o = blockIdx.x << lev;
    if (o >= n) return;
    const MergeInfo m = merge_of(o, lev, n);
    if (!m.active()) return;
    const long long base = (long long)b * w.sV + o;
    const int K = w.Kcnt[base];
    const MatBatch<T>& Zc = src ? w.Z1 : w.Z0;
    const MatBatch<T>& Zn = src ? w.Z0 : w.Z1;
    const T* Zcb = Zc.at(b);
    T* Znb = Zn.at(b);
    const T* Ub = w.U.at(b);
    for (int idx = threadIdx.x; idx < m.k * K; idx += 256) {
        const int r = idx % m.k, j = idx / m.k;
        T acc = T(0);
        for (int kk = 0; kk < K; kk++) {
            const long long c = o + w.perm[base + w.ndpos[base + kk]];
            acc += Zcb[(o + r) + c * Zc.ld] * Ub[(o + kk) + (long long)(o + j) * w.U.ld];
        }
        Znb[(o + r) + (long long)(o + w.outnd[base + j]) * Zn.ld] = acc;
    }
}

// deflated columns and blocks without a merge at this level are copied
template <typename T>
__global__ __launch_bounds__(256) void stedc_copy_kernel(StedcWs<T> w, int lev, int src) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int p = blockIdx.x;
    if (p >= n) return;
    const MergeInfo m = merge_of(p, lev, n);
    const MatBatch<T>& Zc = src ? w.Z1 : w.Z0;
    const MatBatch<T>& Zn = src ? w.Z0 : w.Z1;
    const T* Zcb = Zc.at(b);
    T* Znb = Zn.at(b);
    long long sc, dc;
    if (!m.active()) {
        sc = dc = p;
    } else {
        const long long base = (long long)b * w.sV + m.o;
        const int K = w.Kcnt[base];
        const int it = p - m.o;
        if (it < K) return;
        const int q = it - K;
        sc = m.o + w.perm[base + w.dfpos[base + q]];
        dc = m.o + w.outdf[base + q];
    }
    for (int r = threadIdx.x; r < m.k; r += 256)
        Znb[(m.o + r) + dc * Zn.ld] = Zcb[(m.o + r) + sc * Zc.ld];
}

template <typename T>
__global__ __launch_bounds__(256) void stedc_final_kernel(StedcWs<T> w) {
    const int b = blockIdx.z;
    const int n = w.ns[b];
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    w.w_out[(long long)b * w.sW + p] = (T)(w.D[(long long)b * w.sV + p] * w.scale[b]);
}

// Host check of the gathered split-merge operands (FP32 merges of order
// GEMM_TS128_MIN_ORDER and more) against their buffers of
// nbatch * stride + 64 elements: the furthest element, counted from a
// matrix's base, that stedc_gather_merge_kernel writes and the split product
// reads, over every merge of every level, with the deflation counts at their
// bounds (K, kt, kb <= merge order k).  Writes (column o + x, row o + r):
// x < K, r < k; reads of B: rows o + q .. o + q + 3 for q up to the 32-deep
// slabs' end, ceil32(K) - 4, in column o + min(jj, K - 1).  Returns the
// element count needed past the last matrix's base.
long long stedc_split_extent(int nmax, long long ld) {
    int L = 0;
    while ((1 << L) < nmax) L++;
    long long far = 0;
    for (int lev = 1; lev <= L; lev++) {
        if ((1 << lev) < GEMM_TS128_MIN_ORDER) continue;
        for (int o = 0; o < nmax; o += 1 << lev) {
            const int k = std::min(1 << lev, nmax - o), k1 = std::min(1 << (lev - 1), nmax - o);
            if (k <= k1) continue;  // inactive merge
            const int K = k;
            const long long col = (long long)(o + K - 1) * ld + o;
            far = std::max(far, col + K);                     // GB0/GB1/GA writes, GA reads
            far = std::max(far, col + (K + 31) / 32 * 32);    // B reads, 16 bytes at a time
        }
    }
    return far;
}

template <typename T>
int stedc_launch(const StedcWs<T>& w, int nbatch, int nmax, hipStream_t st) {
    const int gpos = (nmax + 255) / 256;
    hipLaunchKernelGGL(stedc_init_kernel<T>, dim3(1, 1, nbatch), dim3(256), 0, st, w);
    hipLaunchKernelGGL(stedc_fill_kernel<T>, dim3(nmax, 1, nbatch), dim3(256), 0, st, w);
    int L = 0;
    while ((1 << L) < nmax) L++;
    int src = 0;
    for (int lev = 1; lev <= L; lev++) {
        const int nmerge = (nmax + (1 << lev) - 1) >> lev;
        hipLaunchKernelGGL(stedc_setup_kernel<T>, dim3(gpos, 1, nbatch), dim3(256), 0, st, w, lev, src);
        const int msize = std::min(1 << lev, nmax);
        if (msize > 64 && msize <= DEFL_LDS)
            hipLaunchKernelGGL(stedc_deflate_lds_kernel<T>, dim3(nmerge, 1, nbatch), dim3(256), 0, st, w, lev);
        else
            hipLaunchKernelGGL(stedc_deflate_kernel<T>, dim3((nmerge + 63) / 64, 1, nbatch), dim3(64), 0, st, w,
                               lev);
        hipLaunchKernelGGL(stedc_rotate_kernel<T>, dim3(gpos, 1, nbatch), dim3(256), 0, st, w, lev, src);
        hipLaunchKernelGGL(stedc_secular_kernel<T>, dim3((nmax + 3) / 4, 1, nbatch), dim3(256), 0, st, w, lev);
        hipLaunchKernelGGL(stedc_zhat_kernel<T>, dim3((nmax + 3) / 4, 1, nbatch), dim3(256), 0, st, w, lev);
        hipLaunchKernelGGL(stedc_vectors_kernel<T>, dim3(nmax, 1, nbatch), dim3(256), 0, st, w, lev);
        hipLaunchKernelGGL(stedc_order_kernel<T>, dim3((nmax + 3) / 4, 1, nbatch), dim3(256), 0, st, w, lev);
        if ((1 << lev) <= 64) {
            hipLaunchKernelGGL(stedc_small_merge_kernel<T>, dim3(nmerge, 1, nbatch), dim3(256), 0, st, w, lev,
                               src);
        } else {
            hipLaunchKernelGGL(stedc_split_kernel<T>, dim3(nmerge, 1, nbatch), dim3(256), 0, st, w, lev);
            auto setup = [&](auto& pr, int ts) {
                pr.ns = w.ns; pr.lev = lev;
                pr.tdim = (1 << lev) / ts;
                pr.tdh = (1 << (lev - 1)) / ts;
                pr.Zc = src ? w.Z1 : w.Z0;
                pr.Zn = src ? w.Z0 : w.Z1;
                pr.U = w.U;
                pr.outnd = w.outnd; pr.Kcnt = w.Kcnt; pr.ltop = w.ltop; pr.lbot = w.lbot; pr.ktop = w.ktop;
                pr.kbot = w.kbot; pr.ctop = w.ctop; pr.cbot = w.cbot; pr.sV = w.sV;
            };
            if ((1 << lev) >= GEMM_TS128_MIN_ORDER && sizeof(T) == 4 && w.GA0 && w.GA1 && w.GB0 && w.GB1) {
                // FP32 merges of 2048 and more: both operands gathered into
                // contiguous columns, then the product on the FP16 matrix
                // cores with split operands
                hipLaunchKernelGGL(stedc_gather_merge_kernel<T>, dim3(std::min(1 << lev, nmax), nmerge, nbatch),
                                   dim3(256), 0, st, w, lev, src);
                DcMergeSplitProb pr;
                pr.ns = w.ns; pr.lev = lev;
                pr.tdim = (1 << lev) / 128;
                pr.tdh = (1 << (lev - 1)) / 128;
                pr.Zn = {(float*)(src ? w.Z0 : w.Z1).p, w.Z0.ld, w.Z0.stride};
                pr.GA0 = {(float*)w.GA0, w.U.ld, w.U.stride};
                pr.GA1 = {(float*)w.GA1, w.U.ld, w.U.stride};
                pr.GB0 = {(float*)w.GB0, w.U.ld, w.U.stride};
                pr.GB1 = {(float*)w.GB1, w.U.ld, w.U.stride};
                pr.outnd = w.outnd; pr.Kcnt = w.Kcnt; pr.ktop = w.ktop; pr.kbot = w.kbot; pr.sV = w.sV;
                hipLaunchKernelGGL((gemm_f16x3_kernel<DcMergeSplitProb, 128>), dim3(2 * pr.tdh * pr.tdim, nmerge, nbatch),
                                   dim3(256), 0, st, pr);
            } else if ((1 << lev) >= GEMM_TS128_MIN_ORDER) {
                // merges of 2048 and more: 128 x 128 tiles
                typedef Gemm128Shape<T> S;
                DcMergeProb<T, 128> pr;
                setup(pr, 128);
                hipLaunchKernelGGL((gemm_mfma_kernel<T, DcMergeProb<T, 128>, 128, 128, S::BK, S::WM, S::WN>),
                                   dim3(2 * pr.tdh * pr.tdim, nmerge, nbatch), dim3(64 * S::WM * S::WN), 0, st, pr);
            } else {
                DcMergeProb<T, 64> pr;
                setup(pr, 64);
                hipLaunchKernelGGL((gemm_mfma_kernel<T, DcMergeProb<T, 64>>), dim3(2 * pr.tdh * pr.tdim, nmerge, nbatch),
                                   dim3(256), 0, st, pr);
            }
        }
        hipLaunchKernelGGL(stedc_copy_kernel<T>, dim3(nmax, 1, nbatch), dim3(256), 0, st, w, lev, src);
        src ^= 1;
    }
    hipLaunchKernelGGL(stedc_final_kernel<T>, dim3(gpos, 1, nbatch), dim3(256), 0, st, w);
    return src;
}

template <typename T>
__global__ __launch_bounds__(256) void tridiag_guard_kernel(const int* ns, T* d, T* e, long long sD, int* bad) {
    __shared__ int flag;
    const int b = blockIdx.x;
    const int n = ns[b];
    T* db = d + (long long)b * sD;
    T* eb = e + (long long)b * sD;
    if (threadIdx.x == 0) flag = 0;
    __syncthreads();
    bool f = false;
    for (int i = threadIdx.x; i < n; i += 256) f |= !isfinite(db[i]) || (i + 1 < n && !isfinite(eb[i]));
    if (f) flag = 1;
    __syncthreads();
    if (flag)
        for (int i = threadIdx.x; i < n; i += 256) {
            db[i] = T(0);
            eb[i] = T(0);
        }
    if (threadIdx.x == 0) bad[b] = flag;
}

template <typename T>
void tridiag_guard_launch(const int* ns, int nbatch, T* d, T* e, long long sD, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(tridiag_guard_kernel<T>, dim3(nbatch), dim3(256), 0, st, ns, d, e, sD, bad);
}
template void tridiag_guard_launch<double>(const int*, int, double*, double*, long long, int*, hipStream_t);
template void tridiag_guard_launch<float>(const int*, int, float*, float*, long long, int*, hipStream_t);

template int stedc_launch<double>(const StedcWs<double>&, int, int, hipStream_t);
template int stedc_launch<float>(const StedcWs<float>&, int, int, hipStream_t);
