// Eigenvalues of a symmetric tridiagonal matrix without eigenvectors, for
// calls that need no vectors (energy-only FP64 evaluations, the frequency
// route's eigenvalues, mbd_eigh without Z): Sturm-sequence counts with
// multisection.  T = tridiag(e, d, e), d[0..n-1] the diagonal and e[i] the
// element between rows i and i+1.
//
// One wavefront per eigenvalue index k (k-th smallest).  The wave keeps an
// interval [lo, hi] with count(lo) <= k < count(hi), count(x) = number of
// eigenvalues below x; each step evaluates the count at 64 interior points,
// lane l at lo + (hi - lo)(l + 1)/65, and keeps the sub-interval where the
// count passes k (a ballot finds it), so the interval shrinks 65-fold per
// step and about nine steps reach rounding level.  The count is the number
// of negative pivots of the LDL^T factorisation of T - x I,
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

template <typename T>
__global__ __launch_bounds__(256) void stebz_kernel(const int* ns, const T* d, const T* e, long long sD, T* w,
                                                      long long sW) {
    const int b = blockIdx.z;
    const int n = ns[b];
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (k >= n) return;  // the whole wavefront
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
    for (int it = 0; it < 64; it++) {
        const double width = hi - lo;
        if (width <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) break;  // uniform over the wave
        const double x = lo + width * (double)(lane + 1) / 65.0;
        const int c = sturm_count(db, eb, n, x, pivmin);
        const unsigned long long m = __ballot(c > k);
        const int f = m ? __ffsll((long long)m) - 1 : 64;  // first lane whose count passes k
        const double nlo = f == 0 ? lo : lo + width * (double)f / 65.0;
        const double nhi = f == 64 ? hi : lo + width * (double)(f + 1) / 65.0;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) wb[k] = (T)(0.5 * (lo + hi));
}

template <typename T>
void stebz_launch(const int* ns, int nmax, int nbatch, const T* d, const T* e, long long sD, T* w, long long sW,
                  hipStream_t st) {
    hipLaunchKernelGGL(stebz_kernel<T>, dim3((nmax + 3) / 4, 1, nbatch), dim3(256), 0, st, ns, d, e, sD, w, sW);
}
template void stebz_launch<double>(const int*, int, int, const double*, const double*, long long, double*, long long,
                                   hipStream_t);
template void stebz_launch<float>(const int*, int, int, const float*, const float*, long long, float*, long long,
                                  hipStream_t);
