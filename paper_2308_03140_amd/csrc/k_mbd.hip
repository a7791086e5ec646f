// MBD-specific kernels: input preparation, assembly of Q (finite systems),
// the energy reduction, Q^{-1/2} from the eigenpairs and the adjoint
// contraction for the gradients (paper Secs. 2.1, 2.4, 2.7).
#include "mbd_internal.h"
#include "gemm_mfma.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

// ---------------------------------------------------------------------------
// pair tensors
// ---------------------------------------------------------------------------
// bare dipole tensor T_ab = (delta_ab r^2 - 3 r_a r_b)/r^5 (eq:dipole, explicit
// form) and the Fermi damping g = 1/(1 + exp(-a (r/(beta (Rv_i+Rv_j)) - 1)))
// (eq:fermi-damping with s_R = beta, a = 6 for MBD: eq:mbd-lr-dipole)
struct PairTD {
    double T[6];      // xx yy zz xy xz yz
    double g, omg, dg_dr, dg_dR0;
    double d, inv_d;
};

__device__ __forceinline__ void fermi_damp(double d, double R0, double a, double& g, double& omg, double& dg_dr,
                                           double& dg_dR0) {
    if (R0 <= 0.0) { g = 1.0; omg = 0.0; dg_dr = 0.0; dg_dR0 = 0.0; return; }
    const double x = a * (d / R0 - 1.0);
    if (x >= 0.0) { const double e = exp(-x); g = 1.0 / (1.0 + e); omg = e / (1.0 + e); }
    else { const double e = exp(x); g = e / (1.0 + e); omg = 1.0 / (1.0 + e); }
    const double gg = g * omg;
    dg_dr = a / R0 * gg;
    dg_dR0 = -a * d / (R0 * R0) * gg;
}

__device__ __forceinline__ int sym_idx(int a, int b) {
    // xx yy zz xy xz yz
    if (a == b) return a;
    const int s = a + b;  // 1: xy, 2: xz, 3: yz
    return 2 + s;
}

// ---------------------------------------------------------------------------
// input preparation and validation: om_i, c_i = om_i sqrt(alpha0_i)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mbd_prep_kernel(const SysDesc* sd, double* om, double* cc,
                                                         unsigned* status) {
    const int s = blockIdx.y;
    const SysDesc& S = sd[s];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= S.N) return;
    const double a0 = S.alpha0[i];
    const double p = S.omega_or_c6[i];
    const double rv = S.rvdw[i];
    const double x = S.coords[3 * i], y = S.coords[3 * i + 1], z = S.coords[3 * i + 2];
    bool ok = isfinite(a0) && isfinite(p) && isfinite(rv) && isfinite(x) && isfinite(y) && isfinite(z) &&
              a0 > 0.0 && p > 0.0 && rv > 0.0;
    double w = S.param_kind == 1 ? 4.0 * p / (3.0 * a0 * a0) : p;
    if (!ok) { w = 1.0; atomicOr(&status[s], MBD_ST_BAD_INPUT); }
    om[S.atom_off + i] = w;
    cc[S.atom_off + i] = ok ? w * sqrt(a0) : 0.0;
}

// Q of eq:q-matrix, finite system, both triangles; optional FP32 copy.
// 16x16 atom pairs per workgroup.
__global__ __launch_bounds__(256) void mbd_assemble_finite_kernel(const SysDesc* sd, const double* om,
                                                                    const double* cc, MatBatch<double> Q,
                                                                    MatBatch<float> Q32, unsigned* status) {
    const int s = blockIdx.z;
    const SysDesc& S = sd[s];
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= S.N || j >= S.N) return;
    double* Qb = Q.at(s);
    float* Qf = Q32.p ? Q32.at(s) : nullptr;
    const long long ld = Q.ld, ldf = Q32.ld;
    double v[3][3];
    if (i == j) {
        const double w = om[S.atom_off + i];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) v[a][b] = (a == b) ? w * w : 0.0;
    } else {
        const double* R = S.coords;
        const double rx = R[3 * j] - R[3 * i], ry = R[3 * j + 1] - R[3 * i + 1], rz = R[3 * j + 2] - R[3 * i + 2];
        const double r2 = rx * rx + ry * ry + rz * rz;
        double d = sqrt(r2);
        const bool coincident = !(d >= 1e-8);
        if (coincident) { atomicOr(&status[s], MBD_ST_COINCIDENT); d = 1.0; }
        const double inv_d = 1.0 / d;
        const double inv3 = inv_d * inv_d * inv_d, inv5 = inv3 * inv_d * inv_d;
        double g, omg, gd, gR;
        fermi_damp(d, S.beta * (S.rvdw[i] + S.rvdw[j]), S.a, g, omg, gd, gR);
        // coincident or invalid pairs contribute nothing, keeping Q finite
        const double pre = coincident ? 0.0 : cc[S.atom_off + i] * cc[S.atom_off + j] * g;
        const double r[3] = {rx, ry, rz};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) v[a][b] = pre * ((a == b ? inv3 : 0.0) - 3.0 * r[a] * r[b] * inv5);
    }
    for (int b = 0; b < 3; b++)
        for (int a = 0; a < 3; a++) {
            const long long row = 3 * i + a, col = 3 * j + b;
            Qb[row + col * ld] = v[a][b];
            if (Qf) Qf[row + col * ldf] = (float)v[a][b];
        }
}

// ---------------------------------------------------------------------------
// energy: E = w sum_k sqrt(lambda_k) - (3/2) sum_i omega_i  (eq:mbd-energy),
// periodic systems average over their q matrices (eq:brillouin-int).
// conv (may be null): per matrix, 0 where the refinement did not converge;
// such a system gets the MBD_ST_NOT_CONVERGED status bit.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mbd_energy_kernel(const SysDesc* sd, const int* ns, const double* lam,
                                                           long long sL, const double* om, unsigned* status,
                                                           double* lmin_out, const int* conv, const double* mmult) {
    __shared__ double red[4];
    const int s = blockIdx.x;
    const SysDesc& S = sd[s];
    double esum = 0.0, lmin = 1e300;
    bool conv_ok = true;
    for (int q = 0; q < S.nmat; q++) {
        const int b = S.mat0 + q;
        if (conv && conv[b] == 0) conv_ok = false;
        const int n = ns[b];
        const double* L = lam + (long long)b * sL;
        double part = 0.0, mn = 1e300;
        for (int k = threadIdx.x; k < n; k += 256) {
            const double x = L[k];
            mn = fmin(mn, x);
            part += x > 0.0 ? sqrt(x) : 0.0;
        }
        part = block_sum256(part, red);
        mn = -block_max256(-mn, red);
        esum += S.weight * (mmult ? mmult[b] : 1.0) * part;
        lmin = fmin(lmin, mn);
    }
    double wsum = 0.0;
    for (int i = threadIdx.x; i < S.N; i += 256) wsum += om[S.atom_off + i];
    wsum = block_sum256(wsum, red);
    if (threadIdx.x == 0) {
        const bool collapse = !(lmin > 0.0);
        if (collapse) atomicOr(&status[s], MBD_ST_COLLAPSE);
        if (!conv_ok) atomicOr(&status[s], MBD_ST_NOT_CONVERGED);
        if (S.energy) *S.energy = collapse ? __longlong_as_double(0x7ff8000000000000LL) : esum - 1.5 * wsum;
        lmin_out[s] = lmin;
        if (S.errors) S.errors[0] = lmin;
    }
    if (S.eigvals) {
        for (int q = 0; q < S.nmat; q++) {
            const int b = S.mat0 + q;
            const double* L = lam + (long long)b * sL;
            const int n3 = 3 * S.N;
            for (int k = threadIdx.x; k < n3; k += 256)
                S.eigvals[(long long)q * n3 + k] = S.embed ? L[2 * k] : L[k];
        }
    }
}

// errors[1..3] of each system that asks for them: over the system's
// matrices, the largest max|X^T X - I| of the FP32 eigenvectors, the number of
// refinement steps taken and the remainder estimate of the last step (all
// zero without refinement: stats == null).  stats holds {delta, max|R|, rho,
// max|X|} per matrix for step one, then for step two; one[b] != 0 where step
// one was enough.
__global__ __launch_bounds__(64) void mbd_errors_kernel(const SysDesc* sd, int nsys, int nmat, const double* stats,
                                                          const int* one) {
    const int s = blockIdx.x * 64 + threadIdx.x;
    if (s >= nsys) return;
    const SysDesc& S = sd[s];
    if (!S.errors) return;
    double e1 = 0.0, e2 = 0.0, e3 = 0.0;
    if (stats) {
        for (int q = 0; q < S.nmat; q++) {
            const int b = S.mat0 + q;
            e1 = fmax(e1, stats[4 * b + 1]);
            e2 = fmax(e2, one[b] ? 1.0 : 2.0);
            e3 = fmax(e3, one[b] ? stats[4 * b + 2] : stats[4 * (nmat + b) + 2]);
        }
    }
    S.errors[1] = e1;
    S.errors[2] = e2;
    S.errors[3] = e3;
}

// sc_k = lambda_k^{-1/4}, so that Q^{-1/2} = (X sc)(X sc)^T
__global__ __launch_bounds__(256) void mbd_invsqrt4_kernel(const int* ns, const double* lam, long long sL,
                                                             double* sc) {
    const int b = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= ns[b]) return;
    const double x = lam[(long long)b * sL + k];
    sc[(long long)b * sL + k] = x > 0.0 ? 1.0 / sqrt(sqrt(x)) : 0.0;
}

// X(:, c) *= sc_c (X is not needed afterwards); one workgroup per column
__global__ __launch_bounds__(256) void mbd_scale_cols_kernel(const int* ns, MatBatch<double> X, const double* sc,
                                                               long long sL) {
    const int b = blockIdx.z;
    const int n = ns[b];
    const int c = blockIdx.x;
    if (c >= n) return;
    const double f = sc[(long long)b * sL + c];
    double* x = X.at(b) + (long long)c * X.ld;
    for (int r = threadIdx.x; r < n; r += 256) x[r] *= f;
}

// M = (X sc)(X sc)^T, lower triangle: the columns of X are scaled in place,
// then the symmetric product runs as a plain lower-triangle GEMM
void mbd_inv_sqrt_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> X,
                         const double* sc, long long sL, MatBatch<double> M) {
    hipLaunchKernelGGL(mbd_scale_cols_kernel, dim3(nmax, 1, nbatch), dim3(256), 0, st, ns, X, sc, sL);
    gemm_batched<double>(st, false, true, ns, nmax, nbatch, X.p, X.ld, X.stride, X.p, X.ld, X.stride, M.p, M.ld,
                         M.stride, 1.0, 0.0, true);
}

// copy the lower triangle to the upper one
// upper triangle := transpose of the lower one, in 64 x 64 tiles: tile
// (I, J), I >= J, is read by columns (rows and columns clamped into the
// matrix, so the loads are unconditional), transposed through LDS and
// written by columns into tile (J, I); only elements below the diagonal are
// copied.  Matrices whose skip flag is set are left alone.
__global__ __launch_bounds__(256) void mbd_mirror_kernel(const int* ns, MatBatch<double> M, const int* skip) {
    __shared__ double tile[64][65];
    const int b = blockIdx.z;
    if (skip && skip[b]) return;
    const int n = ns[b];
    const int ti = blockIdx.x, tj = blockIdx.y;
    const int r0 = ti * 64, c0 = tj * 64;
    if (tj > ti || r0 >= n) return;
    double* Mb = M.at(b);
    const long long ld = M.ld;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = min(r0 + lane, n - 1), c = min(c0 + wv + 4 * k, n - 1);
        v[k] = Mb[r + (long long)c * ld];
    }
#pragma unroll
    for (int k = 0; k < 16; k++) tile[wv + 4 * k][lane] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = r0 + wv + 4 * k, c = c0 + lane;
        if (r < n && r > c) Mb[c + (long long)r * ld] = tile[lane][wv + 4 * k];
    }
}

// ---------------------------------------------------------------------------
// adjoint contraction, finite systems.  With M = Q^{-1/2}:
//   dE/dR_k   = -1/2 sum_j c_k c_j sum_ab M_{ka,jb} d/dr (g T_ab)(R_j - R_k)
//   dE/dalpha_k = S_k / (4 alpha_k),  S_k = sum_j c_k c_j sum_ab M_{ka,jb} g T_ab
//   dE/domega_k = S_k / (2 omega_k) + omega_k/2 sum_a M_{ka,ka} - 3/2
//   dE/dRv_k  = sum_j 1/2 c_k c_j beta dg/dR0 sum_ab M_{ka,jb} T_ab
// (eq:mbd-gradient as (1/4) Tr(Q^{-1/2} dQ/dX); C6 input by the chain rule
// through 4 C6 = 3 omega alpha0^2).  One workgroup per atom k; M_{ka,jb} is
// read from columns 3k+a (M symmetric), so the loads are contiguous in j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mbd_grad_finite_kernel(const SysDesc* sd, const double* om,
                                                                const double* cc, MatBatch<double> M) {
    __shared__ double red[4];
    const int s = blockIdx.z;
    const SysDesc& S = sd[s];
    const int k = blockIdx.x;
    if (k >= S.N) return;
    const double* Mb = M.at(s);
    const long long ld = M.ld;
    const double* R = S.coords;
    const double ck = cc[S.atom_off + k];
    double f0 = 0, f1 = 0, f2 = 0, Ssum = 0, Usum = 0;
    for (int j = threadIdx.x; j < S.N; j += 256) {
        if (j == k) continue;
        const double r[3] = {R[3 * j] - R[3 * k], R[3 * j + 1] - R[3 * k + 1], R[3 * j + 2] - R[3 * k + 2]};
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double d = sqrt(r2), inv_d = 1.0 / d;
        const double inv3 = inv_d * inv_d * inv_d, inv5 = inv3 * inv_d * inv_d, inv7 = inv5 * inv_d * inv_d;
        double g, omg, gd, gR0;
        fermi_damp(d, S.beta * (S.rvdw[k] + S.rvdw[j]), S.a, g, omg, gd, gR0);
        const double cj = cc[S.atom_off + j];
        double m[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) m[a][b] = Mb[(3 * j + b) + (long long)(3 * k + a) * ld];
        double mt = 0.0, fc[3] = {0, 0, 0};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                const double Tab = (a == b ? inv3 : 0.0) - 3.0 * r[a] * r[b] * inv5;
                mt += m[a][b] * Tab;
                for (int c = 0; c < 3; c++) {
                    double dT = 15.0 * r[a] * r[b] * r[c] * inv7;
                    if (a == b) dT -= 3.0 * r[c] * inv5;
                    if (a == c) dT -= 3.0 * r[b] * inv5;
                    if (b == c) dT -= 3.0 * r[a] * inv5;
                    fc[c] += m[a][b] * (gd * r[c] * inv_d * Tab + g * dT);
                }
            }
        const double pc = ck * cj;
        f0 += pc * fc[0]; f1 += pc * fc[1]; f2 += pc * fc[2];
        Ssum += pc * g * mt;
        Usum += 0.5 * pc * S.beta * gR0 * mt;
    }
    f0 = block_sum256(f0, red);
    f1 = block_sum256(f1, red);
    f2 = block_sum256(f2, red);
    Ssum = block_sum256(Ssum, red);
    Usum = block_sum256(Usum, red);
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int a = 0; a < 3; a++) tr += Mb[(3 * k + a) + (long long)(3 * k + a) * ld];
        const double a0 = S.alpha0[k];
        const double w = om[S.atom_off + k];
        const double dEda = Ssum / (4.0 * a0);
        const double dEdw = Ssum / (2.0 * w) + 0.5 * w * tr - 1.5;
        if (S.grad_coords) {
            S.grad_coords[3 * k] = -0.5 * f0;
            S.grad_coords[3 * k + 1] = -0.5 * f1;
            S.grad_coords[3 * k + 2] = -0.5 * f2;
        }
        if (S.param_kind == 1) {
            // omega = 4 C6/(3 alpha0^2)
            if (S.grad_alpha0) S.grad_alpha0[k] = dEda - 2.0 * w / a0 * dEdw;
            if (S.grad_omega) S.grad_omega[k] = dEdw * w / S.omega_or_c6[k];
        } else {
            if (S.grad_alpha0) S.grad_alpha0[k] = dEda;
            if (S.grad_omega) S.grad_omega[k] = dEdw;
        }
        if (S.grad_rvdw) S.grad_rvdw[k] = Usum;
    }
}

void mbd_prep_launch(hipStream_t st, const SysDesc* sd, int nsys, int Nmax, double* om, double* cc,
                     unsigned* status) {
    hipLaunchKernelGGL(mbd_prep_kernel, dim3((Nmax + 255) / 256, nsys), dim3(256), 0, st, sd, om, cc, status);
}

void mbd_assemble_finite_launch(hipStream_t st, const SysDesc* sd, int nsys, int Nmax, const double* om,
                                const double* cc, MatBatch<double> Q, MatBatch<float> Q32, unsigned* status) {
    const int g = (Nmax + 15) / 16;
    hipLaunchKernelGGL(mbd_assemble_finite_kernel, dim3(g, g, nsys), dim3(256), 0, st, sd, om, cc, Q, Q32, status);
}

void mbd_energy_launch(hipStream_t st, const SysDesc* sd, int nsys, const int* ns, const double* lam, long long sL,
                       const double* om, unsigned* status, double* lmin, const int* conv, const double* mmult) {
    hipLaunchKernelGGL(mbd_energy_kernel, dim3(nsys), dim3(256), 0, st, sd, ns, lam, sL, om, status, lmin, conv,
                       mmult);
}

void mbd_errors_launch(hipStream_t st, const SysDesc* sd, int nsys, int nmat, const double* stats, const int* one) {
    hipLaunchKernelGGL(mbd_errors_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, sd, nsys, nmat, stats, one);
}

void mbd_invsqrt4_launch(hipStream_t st, const int* ns, int nmax, int nbatch, const double* lam, long long sL,
                         double* sc) {
    hipLaunchKernelGGL(mbd_invsqrt4_kernel, dim3((nmax + 255) / 256, nbatch), dim3(256), 0, st, ns, lam, sL, sc);
}

void mbd_mirror_launch(hipStream_t st, const int* ns, int nmax, int nbatch, MatBatch<double> M, const int* skip) {
    const int t = (nmax + 63) / 64;
    hipLaunchKernelGGL(mbd_mirror_kernel, dim3(t, t, nbatch), dim3(256), 0, st, ns, M, skip);
}

void mbd_grad_finite_launch(hipStream_t st, const SysDesc* sd, int nsys, int Nmax, const double* om,
                            const double* cc, MatBatch<double> M) {
    hipLaunchKernelGGL(mbd_grad_finite_kernel, dim3(Nmax, 1, nsys), dim3(256), 0, st, sd, om, cc, M);
}
