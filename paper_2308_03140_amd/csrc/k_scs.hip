// Self-consistent screening (MBD@rsSCS, paper Secs. 2.3 and 2.7) for finite
// systems, and the chain rule of its gradient.
//
// At u = 0 and at every point u_f of the frequency grid:
//   A(u) = diag(1/alpha_i(iu)) (x) I_3 + T^scs,  alpha(iu) = alpha0/(1 + u^2/omega^2)
//   T^scs_ij = (1 - g(r)) T^GG(r; sigma_i, sigma_j),  i != j            (eq:scs-sr-dipole)
//   T^GG_ab = (erf(z) - Th) T_ab + 2 z^2 Th r_a r_b / r^5,
//             z = r/sqrt(sigma_i^2 + sigma_j^2), Th = (2 z/sqrt(pi)) e^{-z^2}  (eq:tgg)
//   sigma = ((1/3) sqrt(2/pi) alpha(iu))^{1/3}                              (eq:mayer)
// (g the Fermi damping with the MBD steepness a and s_R = beta on the input
// R_vdW; T the explicit dipole tensor).  alpha_bar(u) = A(u)^-1 (eq:scs) is
// used only through V = alpha_bar (1 (x) I_3), solved from the batched
// Cholesky factors of A(u); contracted per atom,
// alpha_bar_i(u) = (1/3) sum_a sum_j alpha_bar_{ia,ja} = (1/3) sum_a V_{ia,a}
// (eq:contraction).  The
// screened parameters are alpha_bar_i(0), C6_i = (3/pi) int alpha_bar_i(iu)^2
// du on the grid (eq:casimir-polder), omega_i = 4 C6_i/(3 alpha_bar_i(0)^2)
// and R_vdW,i (alpha_bar_i(0)/alpha0_i)^{1/3} (eq:scale-rvdw-scs).
//
// Gradient: with w_i(u) the weight of alpha_bar_i(u) in E (from the MBD
// gradients with respect to the screened parameters), d alpha_bar/dR =
// -alpha_bar (dA/dR) alpha_bar gives
//   sum_i w_i d alpha_bar_i/dR_mc = (1/3) sum_{l != m} sum_pq
//        [d T^scs_pq / d r_c](R_l - R_m) H_ml[p][q],
//   H_ml[p][q] = sum_a (U_{a,3m+p} V_{3l+q,a} + U_{a,3l+q} V_{3m+p,a}),
//   U_{a,k} = sum_i w_i alpha_bar_{ia,k},  V_{k,a} = sum_j alpha_bar_{k,ja},
// i.e. U^T = alpha_bar (w (x) I_3) (a second three-column solve) and V as
// above, so the contraction is a pair loop, like the MBD adjoint.
#include "mbd_internal.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

#define SCS_SQRT_PI 1.7724538509055160273
#define SCS_PI 3.14159265358979323846

__device__ __forceinline__ double scs_sigma(double alpha) {
    return cbrt(sqrt(2.0 / SCS_PI) * alpha / 3.0);
}

__device__ __forceinline__ void scs_fermi(double d, double R0, double a, double& omg, double& dg_dd) {
    if (R0 <= 0.0) { omg = 0.0; dg_dd = 0.0; return; }
    const double x = a * (d / R0 - 1.0);
    double g;
    if (x >= 0.0) { const double e = exp(-x); g = 1.0 / (1.0 + e); omg = e / (1.0 + e); }
    else { const double e = exp(x); g = e / (1.0 + e); omg = 1.0 / (1.0 + e); }
    dg_dd = a / R0 * g * omg;
}

// T^GG = C1 delta + C2 r r^T and the radial derivatives C1', C2'
__device__ __forceinline__ void tgg_coeffs(double d, double s, double& c1, double& c2, double& c1p, double& c2p) {
    const double z = d / s, z2 = z * z;
    const double th = 2.0 * z / SCS_SQRT_PI * exp(-z2);
    const double em = erf(z) - th;
    const double id = 1.0 / d, id2 = id * id;
    c1 = em * id2 * id;
    c2 = (2.0 * z2 * th - 3.0 * em) * id2 * id2 * id;
    c1p = (2.0 * z2 * th - 3.0 * em) * id2 * id2;
    c2p = (15.0 * em - 10.0 * z2 * th - 4.0 * z2 * z2 * th) * id2 * id2 * id2;
}

// A(u_f) for f = 0..nf-1 (u_0 = 0), both triangles; 16 x 16 atom pairs per
// workgroup, grid (ceil(N/16), ceil(N/16), nf)
__global__ __launch_bounds__(256) void scs_assemble_kernel(const SysDesc* sd, const double* om, const double* u,
                                                             MatBatch<double> A, unsigned* status) {
    const SysDesc& S = sd[0];
    const int f = blockIdx.z;
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= S.N || j >= S.N) return;
    const double uf = u[f];
    const double wi = om[i], wj = om[j];
    const double ai = S.alpha0[i] / (1.0 + uf * uf / (wi * wi));
    double v[3][3];
    if (i == j) {
        for (int p = 0; p < 3; p++)
            for (int q = 0; q < 3; q++) v[p][q] = p == q ? 1.0 / ai : 0.0;
    } else {
        const double aj = S.alpha0[j] / (1.0 + uf * uf / (wj * wj));
        const double* R = S.coords;
        const double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
        double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const bool coincident = !(d >= 1e-8);
        if (coincident) { atomicOr(&status[0], MBD_ST_COINCIDENT); d = 1.0; }
        const double si = scs_sigma(ai), sj = scs_sigma(aj);
        double c1, c2, c1p, c2p, omg, gd;
        tgg_coeffs(d, sqrt(si * si + sj * sj), c1, c2, c1p, c2p);
        scs_fermi(d, S.beta * (S.rvdw[i] + S.rvdw[j]), S.a, omg, gd);
        const double pre = coincident ? 0.0 : omg;
        for (int p = 0; p < 3; p++)
            for (int q = 0; q < 3; q++) v[p][q] = pre * ((p == q ? c1 : 0.0) + c2 * r[p] * r[q]);
    }
    double* Ab = A.at(f);
    for (int q = 0; q < 3; q++)
        for (int p = 0; p < 3; p++) Ab[(3 * i + p) + (long long)(3 * j + q) * A.ld] = v[p][q];
}

// right-hand sides R_f[3i+a][c] = x_i delta_ac, x_i = 1 (contraction) or the
// gradient weight w_i(u_f); layout [nf][3N][3]
__global__ __launch_bounds__(256) void scs_rhs_kernel(int N, int nf, const double* w, double* R) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long tot = (long long)nf * N * 9;
    if (t >= tot) return;
    const int c = (int)(t % 3), a = (int)((t / 3) % 3);
    const long long fi = t / 9;  // f * N + i
    R[t] = a == c ? (w ? w[fi] : 1.0) : 0.0;
}

// alpha_bar_i(u_f) = (1/3) sum_a V_f[3i+a][a]
__global__ __launch_bounds__(256) void scs_contract_kernel(int N, int nf, const double* V, double* abar) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)nf * N) return;
    const double* v = V + t * 9;
    abar[t] = (v[0] + v[4] + v[8]) / 3.0;
}

// UV[f][k][6] = {U_f[k][0..2], V_f[k][0..2]} for the gradient pair loop
__global__ __launch_bounds__(256) void scs_pack_uv_kernel(int n, int nf, const double* U, const double* V, double* UV) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)nf * n) return;
    for (int a = 0; a < 3; a++) {
        UV[t * 6 + a] = U[t * 3 + a];
        UV[t * 6 + 3 + a] = V[t * 3 + a];
    }
}

// screened parameters per atom: alpha_bar(0), C6 (quadrature weights wq_f,
// including 3/pi), omega, R_vdW; out [4][N]: alpha, C6, omega, R_vdW
__global__ __launch_bounds__(256) void scs_params_kernel(const SysDesc* sd, const double* abar, const double* wq,
                                                           int nf, double* out) {
    const SysDesc& S = sd[0];
    const int N = S.N;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    double c6 = 0.0;
    for (int f = 1; f < nf; f++) {
        const double x = abar[(long long)f * N + i];
        c6 += wq[f] * x * x;
    }
    const double a0 = abar[i];
    out[i] = a0;
    out[N + i] = c6;
    out[2 * N + i] = 4.0 * c6 / (3.0 * a0 * a0);
    out[3 * N + i] = S.rvdw[i] * cbrt(a0 / S.alpha0[i]);
}

// weights w_i(u_f) of alpha_bar_i(u_f) in E from the MBD gradients with
// respect to the screened alpha0 (ga), omega (gw), R_vdW (gv):
//   u = 0:  ga - (2 omega/alpha) gw + gv R_vdW/(3 alpha)
//   u_f:    gw (4/(3 alpha^2)) wq_f 2 alpha_bar_i(u_f)
__global__ __launch_bounds__(256) void scs_weights_kernel(int N, int nf, const double* par, const double* abar,
                                                            const double* wq, const double* ga, const double* gw,
                                                            const double* gv, double* w) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int f = blockIdx.y;
    if (i >= N) return;
    const double a = par[i], om = par[2 * N + i], rv = par[3 * N + i];
    double v;
    if (f == 0) v = ga[i] - 2.0 * om / a * gw[i] + gv[i] * rv / (3.0 * a);
    else v = gw[i] * 4.0 / (3.0 * a * a) * wq[f] * 2.0 * abar[(long long)f * N + i];
    w[(long long)f * N + i] = v;
}

// dE/dR_m += sum_f (1/3) sum_{l != m} sum_pq [d T^scs_pq / d r_c] H_ml[p][q];
// one workgroup per atom m
__global__ __launch_bounds__(256) void scs_grad_kernel(const SysDesc* sd, const double* om, const double* u, int nf,
                                                         const double* UV, double* grad) {
    __shared__ double red[4];
    const SysDesc& S = sd[0];
    const int N = S.N;
    const int m = blockIdx.x;
    if (m >= N) return;
    const double* R = S.coords;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (long long t = threadIdx.x; t < (long long)nf * N; t += 256) {
        const int f = (int)(t / N), l = (int)(t % N);
        if (l == m) continue;
        const double uf = u[f];
        const double am = S.alpha0[m] / (1.0 + uf * uf / (om[m] * om[m]));
        const double al = S.alpha0[l] / (1.0 + uf * uf / (om[l] * om[l]));
        const double r[3] = {R[3 * l] - R[3 * m], R[3 * l + 1] - R[3 * m + 1], R[3 * l + 2] - R[3 * m + 2]};
        const double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const double sm = scs_sigma(am), sl = scs_sigma(al);
        double c1, c2, c1p, c2p, omg, gd;
        tgg_coeffs(d, sqrt(sm * sm + sl * sl), c1, c2, c1p, c2p);
        scs_fermi(d, S.beta * (S.rvdw[m] + S.rvdw[l]), S.a, omg, gd);
        const double* Um = UV + ((long long)f * 3 * N + 3 * m) * 6;
        const double* Ul = UV + ((long long)f * 3 * N + 3 * l) * 6;
        // H[p][q] = sum_a (U_a(3m+p) V_a(3l+q) + U_a(3l+q) V_a(3m+p))
        double H[3][3];
        for (int p = 0; p < 3; p++)
            for (int q = 0; q < 3; q++) {
                double h = 0.0;
                for (int a = 0; a < 3; a++) h += Um[6 * p + a] * Ul[6 * q + 3 + a] + Ul[6 * q + a] * Um[6 * p + 3 + a];
                H[p][q] = h;
            }
        // sum_pq H_pq T^GG_pq and sum_pq H_pq r_p r_q, for the radial terms
        double hT = 0.0, hrr = 0.0, hd = 0.0, Hr[3] = {0.0, 0.0, 0.0};
        for (int p = 0; p < 3; p++) {
            hd += H[p][p];
            for (int q = 0; q < 3; q++) {
                hrr += H[p][q] * r[p] * r[q];
                Hr[p] += (H[p][q] + H[q][p]) * r[q];
            }
        }
        hT = c1 * hd + c2 * hrr;
        // d/dr_c [(1-g) (C1 delta + C2 r r^T)] contracted with H:
        //   -g' r_c/d hT + (1-g) [(C1' hd + C2' hrr) r_c/d + C2 (H r + H^T r)_c]
        const double rad = -gd * hT / d + omg * (c1p * hd + c2p * hrr) / d;
        g0 += rad * r[0] + omg * c2 * Hr[0];
        g1 += rad * r[1] + omg * c2 * Hr[1];
        g2 += rad * r[2] + omg * c2 * Hr[2];
    }
    g0 = block_sum256(g0, red);
    g1 = block_sum256(g1, red);
    g2 = block_sum256(g2, red);
    if (threadIdx.x == 0) {
        grad[3 * m] += g0 / 3.0;
        grad[3 * m + 1] += g1 / 3.0;
        grad[3 * m + 2] += g2 / 3.0;
    }
}

void scs_assemble_launch(hipStream_t st, const SysDesc* sd, int N, const double* om, const double* u, int nf,
                         MatBatch<double> A, unsigned* status) {
    const int g = (N + 15) / 16;
    hipLaunchKernelGGL(scs_assemble_kernel, dim3(g, g, nf), dim3(256), 0, st, sd, om, u, A, status);
}
void scs_rhs_launch(hipStream_t st, int N, int nf, const double* w, double* R) {
    const long long tot = (long long)nf * N * 9;
    hipLaunchKernelGGL(scs_rhs_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, N, nf, w, R);
}
void scs_contract_launch(hipStream_t st, int N, int nf, const double* V, double* abar) {
    hipLaunchKernelGGL(scs_contract_kernel, dim3((unsigned)(((long long)nf * N + 255) / 256)), dim3(256), 0, st, N,
                       nf, V, abar);
}
void scs_params_launch(hipStream_t st, const SysDesc* sd, int N, const double* abar, const double* wq, int nf,
                       double* out) {
    hipLaunchKernelGGL(scs_params_kernel, dim3((N + 255) / 256), dim3(256), 0, st, sd, abar, wq, nf, out);
}
void scs_weights_launch(hipStream_t st, int N, int nf, const double* par, const double* abar, const double* wq,
                        const double* ga, const double* gw, const double* gv, double* w) {
    hipLaunchKernelGGL(scs_weights_kernel, dim3((N + 255) / 256, nf), dim3(256), 0, st, N, nf, par, abar, wq, ga, gw,
                       gv, w);
}
void scs_grad_launch(hipStream_t st, const SysDesc* sd, int N, int nf, const double* om, const double* u,
                     const double* U, const double* V, double* UV, double* grad) {
    const int n = 3 * N;
    hipLaunchKernelGGL(scs_pack_uv_kernel, dim3((unsigned)(((long long)nf * n + 255) / 256)), dim3(256), 0, st, n, nf,
                       U, V, UV);
    hipLaunchKernelGGL(scs_grad_kernel, dim3(N), dim3(256), 0, st, sd, om, u, nf, UV, grad);
}
