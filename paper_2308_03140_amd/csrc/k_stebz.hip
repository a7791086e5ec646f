// Eigenvalues of a symmetric tridiagonal matrix without eigenvectors, for
// calls that need no vectors (energy-only FP64 evaluations, the frequency
// route's eigenvalues, mbd_eigh without Z): Sturm-sequence counts with
// multisection.  T = tridiag(e, d, e), d[0..n-1] the diagonal and e[i] the
// element between rows i and i+1.
//
// A group of L lanes (L a power of two, 1..64) works on one eigenvalue index
// k (k-th smallest).  The group keeps an interval [lo, hi] with count(lo) <=
// k < count(hi), count(x) = number of eigenvalues below x; each step
// evaluates the count at L interior points, lane j of the group at lo +
// (hi - lo)(j + 1)/(L + 1), and keeps the sub-interval where the count passes
// k (a ballot finds it), so the interval shrinks (L + 1)-fold per step.  L = 1
// is plain bisection (least work per eigenvalue); larger L trades work for
// fewer sequential steps and is chosen when there are too few eigenvalues to
// fill the device.  The count is the number of negative pivots of the LDL^T
// factorisation of T - x I,
//   q_0 = d_0 - x,  q_i = d_i - x - e_{i-1}^2 / q_{i-1},
// with |q| <= pivmin replaced by -pivmin, pivmin = (smallest normal) *
// max(1, max e^2), which keeps the count monotone in x (the classical
// bisection safeguard).  All arithmetic is FP64.
#include "mbd_internal.h"
#include "mbd_kernels.h"

#define STEBZ_SAFMIN 2.2250738585072014e-308
#define STEBZ_UNROLL 8

template <typename T>
__device__ __forceinline__ int sturm_count(const T* d, const T* e, int n, double x, double pivmin) {
    double q = (double)d[0] - x;
    int c = q < 0.0;
    int i = 1;
    for (; i + STEBZ_UNROLL <= n; i += STEBZ_UNROLL) {
        double dd[STEBZ_UNROLL], ee[STEBZ_UNROLL];
#pragma unroll
        for (int u = 0; u < STEBZ_UNROLL; u++) {
            dd[u] = (double)d[i + u];
            ee[u] = (double)e[i + u - 1];
        }
#pragma unroll
        for (int u = 0; u < STEBZ_UNROLL; u++) {
            if (fabs(q) <= pivmin) q = -pivmin;
            q = (dd[u] - x) - ee[u] * ee[u] / q;
            c += q < 0.0;
        }
    }
    for (; i < n; i++) {
        if (fabs(q) <= pivmin) q = -pivmin;
        const double ev = (double)e[i - 1];
        q = ((double)d[i] - x) - ev * ev / q;
        c += q < 0.0;
    }
    return c;
}

// pairs != 0: T is the tridiagonal of the real embedding [[A, -B], [B, A]]
// of a Hermitian A + iB, whose eigenvalues all come in equal pairs
// (lambda_{2m} = lambda_{2m+1}): only the odd indices are found and each is
// written to both of its pair's slots (an odd order takes every index).
template <typename T>
__global__ __launch_bounds__(256) void stebz_kernel(const int* ns, const T* d, const T* e, long long sD, T* w,
                                                      long long sW, int L, int pairs) {
    const int b = blockIdx.z;
    const int n = ns[b];
    const bool pr = pairs && !(n & 1);
    const int nk = pr ? n / 2 : n;   // eigenvalue indices to find
    const int lane = threadIdx.x & 63;
    const int per_wave = 64 / L;
    const int wave = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave * per_wave >= nk) return;  // the whole wavefront
    const int g = lane / L, j = lane % L;
    const int kq = wave * per_wave + g;
    const bool active = kq < nk;
    const int k = pr ? 2 * kq + 1 : kq;
    const T* db = d + (long long)b * sD;
    const T* eb = e + (long long)b * sD;
    T* wb = w + (long long)b * sW;
    if (n == 1) {
        if (lane == 0) wb[0] = db[0];
        return;
    }
    // Gershgorin interval and the pivot floor
    double gl = 1e300, gu = -1e300, e2max = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double a0 = i > 0 ? fabs((double)eb[i - 1]) : 0.0;
        const double a1 = i < n - 1 ? fabs((double)eb[i]) : 0.0;
        const double di = (double)db[i];
        gl = fmin(gl, di - a0 - a1);
        gu = fmax(gu, di + a0 + a1);
        e2max = fmax(e2max, a1 * a1);
    }
    gl = -wave_max(-gl);
    gu = wave_max(gu);
    e2max = wave_max(e2max);
    const double eps = num_limits<double>::eps;
    const double pivmin = STEBZ_SAFMIN * fmax(1.0, e2max);
    const double tnorm = fmax(fabs(gl), fabs(gu));
    double lo = gl - 2.0 * eps * tnorm * n - 4.0 * pivmin;
    double hi = gu + 2.0 * eps * tnorm * n + 4.0 * pivmin;
    const double sect = (double)(L + 1);
    const unsigned long long gmask = L == 64 ? ~0ull : ((1ull << L) - 1ull);
    // stop at a relative width of 2 eps, or an absolute one of eps ||T|| (the
    // accuracy the count itself supports) for eigenvalues near zero
    const double atol = eps * tnorm + pivmin;
    for (int it = 0; it < 200; it++) {
        const double width = hi - lo;
        const bool done = !active || width <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + atol;
        if (__ballot(!done) == 0ull) break;
        const double x = lo + width * (double)(j + 1) / sect;
        const int c = done ? 0 : sturm_count(db, eb, n, x, pivmin);
        const unsigned long long m = (__ballot(c > k) >> (g * L)) & gmask;
        const int f = m ? __ffsll((long long)m) - 1 : L;  // first lane of the group whose count passes k
        if (!done) {
            const double nlo = f == 0 ? lo : lo + width * (double)f / sect;
            const double nhi = f == L ? hi : lo + width * (double)(f + 1) / sect;
            lo = nlo;
            hi = nhi;
        }
    }
    if (active && j == 0) {
        wb[k] = (T)(0.5 * (lo + hi));
        if (pr) wb[k - 1] = wb[k];
    }
}

// lanes per eigenvalue: as many as keep the launch within the lanes the
// device holds at once (256 CUs x 4 SIMDs x 8 waves x 64 lanes), 1 to 64.
// On 960 embeddings of order 384 (184 320 eigenvalue pairs) this gives two
// lanes: 4.1 ms, against 6.0 ms with one (less work, 2.8 waves per SIMD)
// and 6.0 ms with four (more work than the device holds at once).
static int stebz_lanes(long long eigenvalues) {
    const long long cap = 256LL * 4 * 8 * 64;
    int L = 64;
    while (L > 1 && eigenvalues * L > cap) L >>= 1;
    return L;
}

template <typename T>
void stebz_launch(const int* ns, int nmax, int nbatch, const T* d, const T* e, long long sD, T* w, long long sW,
                  hipStream_t st, bool pairs) {
    // lanes per eigenvalue from the indices actually found; the grid still
    // covers every index of the largest order (waves past a matrix's count exit)
    const int nk = pairs ? (nmax + 1) / 2 : nmax;
    const int L = stebz_lanes((long long)nk * nbatch);
    const int per_wave = 64 / L;
    const int waves = (nmax + per_wave - 1) / per_wave;
    hipLaunchKernelGGL(stebz_kernel<T>, dim3((waves + 3) / 4, 1, nbatch), dim3(256), 0, st, ns, d, e, sD, w, sW, L,
                       pairs ? 1 : 0);
}
template void stebz_launch<double>(const int*, int, int, const double*, const double*, long long, double*, long long,
                                   hipStream_t, bool);
template void stebz_launch<float>(const int*, int, int, const float*, const float*, long long, float*, long long,
                                  hipStream_t, bool);
