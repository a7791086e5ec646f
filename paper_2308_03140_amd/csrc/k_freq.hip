// Frequency route of the MBD energy (paper Sec. 2.5) on the eigenvalues x_k
// of K(u) = alpha(iu)^{1/2} T^lr alpha(iu)^{1/2}, alpha(iu) = alpha0/(1 +
// u^2/omega^2) (eq:dyn-pol), at the points u_f of a Gauss-Legendre grid
// mapped by u = 0.6 (1 + x)/(1 - x) (Sec. 3.3), and for periodic systems at
// every q of the mesh:
//   E      = (1/2pi) int du sum_k ln(1 + x_k)               (eq:log-formula)
//   E_G    = (1/2pi) int du sum_k (ln(1 + x~_k) - x~_k)       (eq:gould-norm)
//   E^(n)  = -(1/2pi) int du ((-1)^n / n) sum_k x_k^n        (eq:rpa)
// K(u) is assembled by the MBD assembly kernels with omega -> 0 on the
// diagonal and c_i -> alpha_i(iu)^{1/2} (periodic: the lattice sums T(q) once,
// then scaled per frequency); every (u, q) matrix is one member of a batch
// for the eigenvalue-only solver.  Periodic matrices are real
// embeddings of order 2n, so each x_k appears twice and carries half weight.
#include "mbd_internal.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

#define FREQ_SQRT_PI 1.7724538509055160273

// c_{f,i} = alpha_i(iu_f)^{1/2}, omega entry 0, for descriptor f + 1 (atom
// offset f N); descriptor 0 holds the validated omega of the system
__global__ __launch_bounds__(256) void mbd_freq_coeff_kernel(const SysDesc* sd, const double* om0, const double* u,
                                                               int N, double* om_f, double* cc_f) {
    const int f = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double w = om0[i];
    const double a = sd[0].alpha0[i] / (1.0 + u[f] * u[f] / (w * w));
    om_f[(long long)f * N + i] = 0.0;
    cc_f[(long long)f * N + i] = sqrt(a);
}

// Periodic K(u_f, q) = C_f T(q) C_f from the embedded lattice sum T(q),
// assembled once (it does not depend on the frequency): element (m, c) of
// the order-2n embedding belongs to atoms (m mod n)/3 and (c mod n)/3.
// Grid (elements / 256, nq, nfreq).
__global__ __launch_bounds__(256) void mbd_freq_scale_kernel(const double* cc_f, int N, int nq, MatBatch<double> T,
                                                               MatBatch<double> K) {
    const int n = 3 * N, n2 = 2 * n;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)n2 * n2) return;
    const int q = blockIdx.y, f = blockIdx.z;
    const int m = (int)(e % n2), c = (int)(e / n2);
    const double* cf = cc_f + (long long)f * N;
    const double s = cf[(m < n ? m : m - n) / 3] * cf[(c < n ? c : c - n) / 3];
    const long long o = m + (long long)c * T.ld;
    K.at(f * nq + q)[m + (long long)c * K.ld] = s * T.at(q)[o];
}

// ln(1 + x~) - x~ (eq:gould-norm); x~ = -erf(y)^{1/4} for x < 0, y =
// (sqrt(pi)/2) x^4, with ln erf(y) from erf for small y and from erfc for
// large y so that 1 + x~ = -expm1(ln erf(y) / 4) keeps its accuracy
__device__ __forceinline__ double gould_term(double x) {
    if (x >= 0.0) return log1p(x) - x;
    const double y = 0.5 * FREQ_SQRT_PI * x * x * x * x;
    const double l = y < 0.5 ? log(erf(y)) : log1p(-erfc(y));
    return log(-expm1(0.25 * l)) + exp(0.25 * l);
}

// per matrix b: {sum ln(1+x) (NaN if some 1+x <= 0), sum gould, min(1+x),
// sum x^n for n = 1..norder} into part[b][3 + norder]
__global__ __launch_bounds__(256) void mbd_freq_terms_kernel(const int* ns, const double* lam, long long sL,
                                                               int norder, double* part) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int n = ns[b];
    const double* L = lam + (long long)b * sL;
    double sl = 0.0, sg = 0.0, mn = 1e300;
    int bad = 0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const double x = L[k];
        mn = fmin(mn, 1.0 + x);
        if (1.0 + x > 0.0) sl += log1p(x);
        else bad = 1;
        sg += gould_term(x);
    }
    sl = block_sum256(sl, red);
    sg = block_sum256(sg, red);
    mn = -block_max256(-mn, red);
    const double nb = block_sum256((double)bad, red);
    double* out = part + (long long)b * (3 + norder);
    if (threadIdx.x == 0) {
        out[0] = nb > 0.0 ? __longlong_as_double(0x7ff8000000000000LL) : sl;
        out[1] = sg;
        out[2] = mn;
    }
    for (int o = 1; o <= norder; o++) {
        double s = 0.0;
        for (int k = threadIdx.x; k < n; k += 256) {
            const double x = L[k];
            double p = x;
            for (int e = 1; e < o; e++) p *= x;
            s += p;
        }
        s = block_sum256(s, red);
        if (threadIdx.x == 0) out[2 + o] = s;
    }
}

// terms = sum over (f, q) of w_f / nq (x 1/2 for embedded matrices) times the
// per-matrix sums, in a fixed order; min(1 + x) over all matrices
__global__ __launch_bounds__(64) void mbd_freq_sum_kernel(const double* part, const double* wf, int nfreq, int nq,
                                                            int embed, int norder, double* terms) {
    const int t = threadIdx.x;
    const int nt = 3 + norder;
    if (t >= nt) return;
    const double h = embed ? 0.5 : 1.0;
    double acc = t == 2 ? 1e300 : 0.0;
    for (int f = 0; f < nfreq; f++)
        for (int q = 0; q < nq; q++) {
            const double v = part[((long long)f * nq + q) * nt + t];
            if (t == 2) {
                acc = fmin(acc, v);
            } else {
                double c = wf[f] / nq * h;
                if (t >= 3) {
                    const int o = t - 2;  // order n
                    c *= ((o & 1) ? 1.0 : -1.0) / o;
                }
                acc += c * v;
            }
        }
    terms[t] = acc;
}

void mbd_freq_coeff_launch(hipStream_t st, const SysDesc* sd, const double* om0, const double* u, int nfreq, int N,
                           double* om_f, double* cc_f) {
    hipLaunchKernelGGL(mbd_freq_coeff_kernel, dim3((N + 255) / 256, nfreq), dim3(256), 0, st, sd, om0, u, N, om_f,
                       cc_f);
}

void mbd_freq_scale_launch(hipStream_t st, const double* cc_f, int N, int nfreq, int nq, MatBatch<double> T,
                           MatBatch<double> K) {
    const long long el = 36LL * N * N;
    hipLaunchKernelGGL(mbd_freq_scale_kernel, dim3((unsigned)((el + 255) / 256), nq, nfreq), dim3(256), 0, st, cc_f, N,
                       nq, T, K);
}

void mbd_freq_terms_launch(hipStream_t st, const int* ns, int nmat, const double* lam, long long sL, int norder,
                           double* part, const double* wf, int nfreq, int nq, int embed, double* terms) {
    hipLaunchKernelGGL(mbd_freq_terms_kernel, dim3(nmat), dim3(256), 0, st, ns, lam, sL, norder, part);
    hipLaunchKernelGGL(mbd_freq_sum_kernel, dim3(1), dim3(64), 0, st, part, wf, nfreq, nq, embed, norder, terms);
}
