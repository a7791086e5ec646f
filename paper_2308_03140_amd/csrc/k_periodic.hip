// Periodic systems: Q(q) of eq:q-matrix with T^lr(q) the Bloch sum of g T
// (paper Sec. 2.2), evaluated with the Ewald split of eq:ewald/eq:terfc plus
// a real-space damping correction, for every q of the mesh in one launch, and
// the matching adjoint contraction for dE/dR, dE/dalpha0 and dE/dA (lattice).
//
// For the pair (i, j), r = R_j - R_i and x_n = r + R_n:
//   T_ij(q) = sum_n [T^erfc(x_n) (|x_n| < Rc) - (1 - g(x_n)) T(x_n)] e^{-i q.x_n}
//           + (4 pi/Omega) sum_{0<|k|<kc} k^ k^ e^{-k^2/(4 gamma^2)} e^{+i G.r},  k = G + q
//           - delta_ij 4 gamma^3/(3 sqrt(pi)) I
// The terms with n = 0, i = j are skipped; the surface term and k = 0 are
// omitted; the damping correction runs over every image with (1 - g) > 1e-18.
// T^erfc_ab = (delta_ab r^2 B - r_a r_b C)/r^5 with B, C of eq:terfc (the
// factor 3 of the printed r_a r_b term is part of C).
//
// The Hermitian Q(q) is stored as its real embedding [[Re, -Im], [Im, Re]]
// (order 2n) so the batched real eigensolver serves it; every eigenvalue of
// Q(q) appears twice.  The reciprocal sums are evaluated in FP64.
#include "mbd_internal.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

#define DAMP_TAIL 1e-18
#define SQRT_PI 1.7724538509055160273

__device__ __forceinline__ void fermi_pair(double d, double R0, double a, double& g, double& omg, double& dg_dr) {
    if (R0 <= 0.0) { g = 1.0; omg = 0.0; dg_dr = 0.0; return; }
    const double x = a * (d / R0 - 1.0);
    if (x >= 0.0) { const double e = exp(-x); g = 1.0 / (1.0 + e); omg = e / (1.0 + e); }
    else { const double e = exp(x); g = e / (1.0 + e); omg = 1.0 / (1.0 + e); }
    dg_dr = a / R0 * g * omg;
}

// Real-space image term F(x) = T^erfc(x) [|x| < rc] - (1-g) T(x) and, if
// dF != nullptr, dF[c][ab] = dF_ab/dx_c and F0[ab] = dF_ab/dR0 = (dg/dR0) T(x),
// R0 = beta (Rv_i + Rv_j) the damping radius (dg/dR0 = -(d/R0) dg/dd).
// Returns false when the term is empty.
__device__ __forceinline__ bool image_term(const double* x, double gamma, double rc, double R0, double a,
                                           double* F, double* dF, double* F0 = nullptr) {
    const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    const double d = sqrt(r2);
    const bool erfc_on = d < rc;
    double g, omg, gd;
    fermi_pair(d, R0, a, g, omg, gd);
    const bool damp_on = omg > DAMP_TAIL;
    if (!erfc_on && !damp_on) return false;
    const double inv_d = 1.0 / d;
    const double inv3 = inv_d * inv_d * inv_d, inv5 = inv3 * inv_d * inv_d;
    double B = 0.0, C = 0.0, dbr = 0.0, dcr = 0.0;
    if (erfc_on) {
        const double z = gamma * d;
        const double ex = exp(-z * z);
        const double ec = erfc(z);
        B = ec + 2.0 * z / SQRT_PI * ex;
        C = 3.0 * ec + 2.0 * z / SQRT_PI * (3.0 + 2.0 * z * z) * ex;
        if (dF) {
            const double dB = -4.0 * gamma * gamma * gamma * r2 / SQRT_PI * ex;
            const double dC = -8.0 * gamma * z * z * z * z / SQRT_PI * ex;
            dbr = dB * inv3 - 3.0 * B * inv3 * inv_d;
            dcr = dC * inv5 - 5.0 * C * inv5 * inv_d;
        }
    }
    // bare part scaled by (1 - g): subtracted
    const double w = damp_on ? omg : 0.0;
    // F = (B - w) delta/r^3 - (C - 3 w) r_a r_b / r^5
    const double b = B - w, cc = C - 3.0 * w;
    for (int p = 0; p < 3; p++)
        for (int s = 0; s < 3; s++) F[p * 3 + s] = (p == s ? b * inv3 : 0.0) - cc * x[p] * x[s] * inv5;
    if (F0) {
        const double g0 = damp_on ? -gd * d / R0 : 0.0;
        for (int p = 0; p < 3; p++)
            for (int s = 0; s < 3; s++) F0[p * 3 + s] = g0 * ((p == s ? inv3 : 0.0) - 3.0 * x[p] * x[s] * inv5);
    }
    if (dF) {
        // d/dd of the bare tensor pieces: d(1/d^3) = -3/d^4, d(3/d^5) = -15/d^6
        // damping: -(1-g) T, d(1-g)/dd = -gd
        const double inv7 = inv5 * inv_d * inv_d;
        for (int c = 0; c < 3; c++) {
            const double xc = x[c] * inv_d;
            for (int p = 0; p < 3; p++)
                for (int s = 0; s < 3; s++) {
                    double v = 0.0;
                    // erfc part
                    if (erfc_on) {
                        v += -dcr * xc * x[p] * x[s];
                        if (p == s) v += dbr * xc;
                        if (p == c) v -= C * x[s] * inv5;
                        if (s == c) v -= C * x[p] * inv5;
                    }
                    if (damp_on) {
                        double dT = 15.0 * x[p] * x[s] * x[c] * inv7;
                        if (p == s) dT -= 3.0 * x[c] * inv5;
                        if (p == c) dT -= 3.0 * x[s] * inv5;
                        if (s == c) dT -= 3.0 * x[p] * inv5;
                        const double T0 = (p == s ? inv3 : 0.0) - 3.0 * x[p] * x[s] * inv5;
                        v += -omg * dT + gd * xc * T0;
                    }
                    dF[c * 9 + p * 3 + s] = v;
                }
        }
    }
    return true;
}

// Assembly of the embedded Q(q).  A wavefront holds 64 / lpp ordered atom
// pairs (i, j), lpp lanes each, one lane per q-point (lpp: the q count
// rounded up to a power of two, at most 64; grid y covers further groups of
// q-points).  The real-space image terms depend on the pair and the image
// only: each is formed once, by one lane of its pair, into LDS (lpp images
// per round), and every lane of the pair adds it with its own phase
// e^{-i q.x}.  Lanes of a pair index past N^2 follow the barriers and store
// nothing.
#define PER_LANES 64
__global__ __launch_bounds__(PER_LANES) void mbd_assemble_periodic_kernel(const SysDesc* sd, const double* om,
                                                                          const double* cc, const double* qcart,
                                                                          int nq, int lpp, const int* img, int nimg,
                                                                          const int* rec, int nrec, MatBatch<double> Q,
                                                                          MatBatch<float> Q32, unsigned* status) {
    __shared__ double xs[PER_LANES][3], Fs[PER_LANES][9];
    __shared__ int oks[PER_LANES];
    const SysDesc& S = sd[0];
    const int N = S.N, n = 3 * N;
    const int slot = threadIdx.x / lpp, ql = threadIdx.x % lpp;
    const long long pid0 = (long long)blockIdx.x * (PER_LANES / lpp) + slot;
    const bool pv = pid0 < (long long)N * N;
    const long long pid = pv ? pid0 : 0;
    const int q = blockIdx.y * lpp + ql;
    const bool qv_ok = pv && q < nq;
    const int i = (int)(pid % N), j = (int)(pid / N);
    const double* R = S.coords;
    const double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
    const int qc = qv_ok ? q : 0;
    const double qv[3] = {qcart[3 * qc], qcart[3 * qc + 1], qcart[3 * qc + 2]};
    const double R0 = S.beta * (S.rvdw[i] + S.rvdw[j]);
    double Tre[9], Tim[9];
    for (int k = 0; k < 9; k++) { Tre[k] = 0.0; Tim[k] = 0.0; }
    for (int t0 = 0; t0 < nimg; t0 += lpp) {
        {
            const int t = t0 + ql;
            int ok = 0;
            if (t < nimg) {
                const double n0 = img[3 * t], n1 = img[3 * t + 1], n2 = img[3 * t + 2];
                double x[3];
                for (int c = 0; c < 3; c++) x[c] = r[c] + n0 * S.lat[c] + n1 * S.lat[3 + c] + n2 * S.lat[6 + c];
                const double d2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
                if (d2 != 0.0) {
                    if (pv && i != j && d2 < 1e-16 && blockIdx.y == 0) atomicOr(&status[0], MBD_ST_COINCIDENT);
                    double F[9];
                    if (image_term(x, S.gamma, S.rc, R0, S.a, F, nullptr)) {
                        ok = 1;
                        for (int c = 0; c < 3; c++) xs[threadIdx.x][c] = x[c];
                        for (int k = 0; k < 9; k++) Fs[threadIdx.x][k] = F[k];
                    }
                }
            }
            oks[threadIdx.x] = ok;
        }
        __syncthreads();
        const int tn = min(lpp, nimg - t0);
        for (int u0 = 0; u0 < tn; u0++) {
            const int u = slot * lpp + u0;
            if (!oks[u]) continue;
            double sph, cph;
            sincos(-(qv[0] * xs[u][0] + qv[1] * xs[u][1] + qv[2] * xs[u][2]), &sph, &cph);
            for (int k = 0; k < 9; k++) { Tre[k] += Fs[u][k] * cph; Tim[k] += Fs[u][k] * sph; }
        }
        __syncthreads();
    }
    if (!qv_ok) return;
    const double pref = 4.0 * M_PI / S.vol;
    const double g4 = 1.0 / (4.0 * S.gamma * S.gamma);
    for (int t = 0; t < nrec; t++) {
        const double m0 = rec[3 * t], m1 = rec[3 * t + 1], m2 = rec[3 * t + 2];
        double G[3], k[3];
        for (int c = 0; c < 3; c++) {
            G[c] = m0 * S.recip[c] + m1 * S.recip[3 + c] + m2 * S.recip[6 + c];
            k[c] = G[c] + qv[c];
        }
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        if (k2 == 0.0 || k2 >= S.kc * S.kc) continue;
        const double E = pref * exp(-k2 * g4) / k2;
        double sph, cph;
        sincos(G[0] * r[0] + G[1] * r[1] + G[2] * r[2], &sph, &cph);
        for (int p = 0; p < 3; p++)
            for (int s = 0; s < 3; s++) {
                const double h = k[p] * k[s] * E;
                Tre[p * 3 + s] += h * cph;
                Tim[p * 3 + s] += h * sph;
            }
    }
    if (i == j) {
        const double self = 4.0 * S.gamma * S.gamma * S.gamma / (3.0 * SQRT_PI);
        Tre[0] -= self; Tre[4] -= self; Tre[8] -= self;
    }
    const double pc = cc[S.atom_off + i] * cc[S.atom_off + j];
    double* Qb = Q.at(q);
    float* Qf = Q32.p ? Q32.at(q) : nullptr;
    const long long ld = Q.ld, ldf = Q32.ld;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            const double re = pc * Tre[a * 3 + b] + ((i == j && a == b) ? om[S.atom_off + i] * om[S.atom_off + i] : 0.0);
            const double im = pc * Tim[a * 3 + b];
            const long long r0 = 3 * i + a, c0 = 3 * j + b;
            Qb[r0 + c0 * ld] = re;
            Qb[(r0 + n) + (c0 + n) * ld] = re;
            Qb[r0 + (c0 + n) * ld] = -im;
            Qb[(r0 + n) + c0 * ld] = im;
            if (Qf) {
                Qf[r0 + c0 * ldf] = (float)re;
                Qf[(r0 + n) + (c0 + n) * ldf] = (float)re;
                Qf[r0 + (c0 + n) * ldf] = (float)-im;
                Qf[(r0 + n) + c0 * ldf] = (float)im;
            }
        }
}

// Adjoint contraction.  With M(q) = Q(q)^{-1/2} read from the embedded
// inverse square root (Re in the top-left block, Im in the bottom-left), the
// ordered pair (i, j) at q contributes, with X = d T_ij(q) and
// c_i c_j (1/4) (1/n_q) Re sum_ab M_{jb,ia} X_ab:
//   to dE/dR_j (+) and dE/dR_i (-)    X = dT/dr_c
//   to dE/dA_vc                        X = dT/dA_vc (Cartesian positions and
//                                      fractional q fixed: dR_n/dA_vc = n_v e_c,
//                                      dG/dA_vc = -G_c Ainv[:, v], dOmega/dA_vc =
//                                      Omega Ainv_cv)
//   to dE/dalpha_i, dE/dalpha_j        X = T_ij(q) / (2 alpha)
//   to dE/domega_i, dE/domega_j        X = T_ij(q) / omega (through c = omega
//                                      sqrt(alpha0); the omega^2 diagonal adds
//                                      (1/2) omega_i Re Tr M_ii(q) per q)
//   to dE/dRv_i, dE/dRv_j              X = beta dT_ij(q)/dR0 (damping radius
//                                      R0 = beta (Rv_i + Rv_j))
// Partial results per (q, i, j): {P, dR[3], dA[9], P0}.
// Same layout as the assembly: one workgroup per ordered pair, one lane per
// q-point, each real-space image term (F and its derivatives) formed once
// into LDS and added by every lane with its own phase and M(q).
__global__ __launch_bounds__(PER_LANES) void mbd_grad_periodic_kernel(const SysDesc* sd, const double* om,
                                                                      const double* cc, const double* qcart, int nq,
                                                                      int lpp, const int* img, int nimg,
                                                                      const int* rec, int nrec, MatBatch<double> M,
                                                                      double* part) {
    __shared__ double xs[PER_LANES][3], Fs[PER_LANES][9], dFs[PER_LANES][27], F0s[PER_LANES][9];
    __shared__ int ns_[PER_LANES][3], oks[PER_LANES];
    const SysDesc& S = sd[0];
    const int N = S.N, n = 3 * N;
    const int slot = threadIdx.x / lpp, ql = threadIdx.x % lpp;
    const long long pid0 = (long long)blockIdx.x * (PER_LANES / lpp) + slot;
    const bool pv = pid0 < (long long)N * N;
    const long long pid = pv ? pid0 : 0;
    const int q0 = blockIdx.y * lpp + ql;
    const bool qv_ok = pv && q0 < nq;
    const int q = q0 < nq ? q0 : 0;
    const int i = (int)(pid % N), j = (int)(pid / N);
    double* out = part + ((long long)q * N * N + pid) * PER_PART;
    if (S.N == 0) return;
    const double* R = S.coords;
    const double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
    const double qv[3] = {qcart[3 * q], qcart[3 * q + 1], qcart[3 * q + 2]};
    const double R0 = S.beta * (S.rvdw[i] + S.rvdw[j]);
    // M_{jb,ia}
    double Mr[9], Mi[9];
    const double* Mb = M.at(q);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            Mr[a * 3 + b] = Mb[(3 * j + b) + (long long)(3 * i + a) * M.ld];
            Mi[a * 3 + b] = Mb[(n + 3 * j + b) + (long long)(3 * i + a) * M.ld];
        }
    // rho = A^{-T} r  (rho_v = sum_d Ainv[d][v] r_d)
    double rho[3];
    for (int v = 0; v < 3; v++) rho[v] = S.linv[v] * r[0] + S.linv[3 + v] * r[1] + S.linv[6 + v] * r[2];
    double P = 0.0, P0 = 0.0, dR[3] = {0, 0, 0}, dA[9];
    for (int k = 0; k < 9; k++) dA[k] = 0.0;
    for (int t0 = 0; t0 < nimg; t0 += lpp) {
        {
            const int t = t0 + ql;
            int ok = 0;
            if (t < nimg) {
                const int nn[3] = {img[3 * t], img[3 * t + 1], img[3 * t + 2]};
                double x[3];
                for (int c = 0; c < 3; c++) x[c] = r[c] + nn[0] * S.lat[c] + nn[1] * S.lat[3 + c] + nn[2] * S.lat[6 + c];
                const double d2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
                double F[9], dF[27], F0[9];
                if (d2 != 0.0 && image_term(x, S.gamma, S.rc, R0, S.a, F, dF, F0)) {
                    ok = 1;
                    for (int c = 0; c < 3; c++) { xs[threadIdx.x][c] = x[c]; ns_[threadIdx.x][c] = nn[c]; }
                    for (int k = 0; k < 9; k++) Fs[threadIdx.x][k] = F[k];
                    for (int k = 0; k < 27; k++) dFs[threadIdx.x][k] = dF[k];
                    for (int k = 0; k < 9; k++) F0s[threadIdx.x][k] = F0[k];
                }
            }
            oks[threadIdx.x] = ok;
        }
        __syncthreads();
        const int tn = min(lpp, nimg - t0);
        for (int u0 = 0; u0 < tn; u0++) {
        const int u = slot * lpp + u0;
        if (!oks[u]) continue;
        const double* x = xs[u];
        const double* F = Fs[u];
        const double* dF = dFs[u];
        const int* nn = ns_[u];
        double sph, cph;
        sincos(-(qv[0] * x[0] + qv[1] * x[1] + qv[2] * x[2]), &sph, &cph);
        double SF = 0.0, SFi = 0.0, SdF[3] = {0, 0, 0}, SdFi[3] = {0, 0, 0}, SF0 = 0.0, SF0i = 0.0;
        for (int k = 0; k < 9; k++) {
            SF += Mr[k] * F[k];
            SFi += Mi[k] * F[k];
            SF0 += Mr[k] * F0s[u][k];
            SF0i += Mi[k] * F0s[u][k];
        }
        P0 += SF0 * cph - SF0i * sph;
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < 9; k++) {
                SdF[c] += Mr[k] * dF[c * 9 + k];
                SdFi[c] += Mi[k] * dF[c * 9 + k];
            }
        P += SF * cph - SFi * sph;
        for (int c = 0; c < 3; c++) {
            // (dF_c - i q_c F) e^{i ph}
            dR[c] += SdF[c] * cph - SdFi[c] * sph + qv[c] * (SF * sph + SFi * cph);
            for (int v = 0; v < 3; v++) {
                // (dF_c n_v + i q_c rho_v F) e^{i ph}
                dA[v * 3 + c] += nn[v] * (SdF[c] * cph - SdFi[c] * sph) -
                                 qv[c] * rho[v] * (SF * sph + SFi * cph);
            }
        }
        }
        __syncthreads();
    }
    const double pref = 4.0 * M_PI / S.vol;
    const double g4 = 1.0 / (4.0 * S.gamma * S.gamma);
    for (int t = 0; t < nrec; t++) {
        const double m0 = rec[3 * t], m1 = rec[3 * t + 1], m2 = rec[3 * t + 2];
        double G[3], k[3];
        for (int c = 0; c < 3; c++) {
            G[c] = m0 * S.recip[c] + m1 * S.recip[3 + c] + m2 * S.recip[6 + c];
            k[c] = G[c] + qv[c];
        }
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        if (k2 == 0.0 || k2 >= S.kc * S.kc) continue;
        const double E = exp(-k2 * g4);
        double sph, cph;
        sincos(G[0] * r[0] + G[1] * r[1] + G[2] * r[2], &sph, &cph);
        // S_h = sum_ab M h_ab with h = k_a k_b E / k^2
        double Sh = 0.0, Shi = 0.0, Sdh[3] = {0, 0, 0}, Sdhi[3] = {0, 0, 0};
        for (int p = 0; p < 3; p++)
            for (int s = 0; s < 3; s++) {
                const double h = k[p] * k[s] * E / k2;
                Sh += Mr[p * 3 + s] * h;
                Shi += Mi[p * 3 + s] * h;
                for (int dd = 0; dd < 3; dd++) {
                    double dh = -2.0 * k[p] * k[s] * k[dd] / (k2 * k2) * E - h * k[dd] * 2.0 * g4;
                    if (p == dd) dh += k[s] / k2 * E;
                    if (s == dd) dh += k[p] / k2 * E;
                    Sdh[dd] += Mr[p * 3 + s] * dh;
                    Sdhi[dd] += Mi[p * 3 + s] * dh;
                }
            }
        P += pref * (Sh * cph - Shi * sph);
        for (int c = 0; c < 3; c++) {
            // pref h (i G_c) e^{i ph}
            dR[c] += -pref * G[c] * (Sh * sph + Shi * cph);
            for (int v = 0; v < 3; v++) {
                double ure = 0.0, uim = 0.0;  // sum_ab M (u_ab) with u = -Ainv_cv h - k_c dh.Ainv[:, v]
                const double aiv = S.linv[c * 3 + v];
                double dv = 0.0, dvi = 0.0;
                for (int dd = 0; dd < 3; dd++) {
                    dv += Sdh[dd] * S.linv[dd * 3 + v];
                    dvi += Sdhi[dd] * S.linv[dd * 3 + v];
                }
                ure = -aiv * Sh - k[c] * dv;
                uim = -aiv * Shi - k[c] * dvi;
                // im part of the bracket: -h G_c rho_v
                const double wv = -G[c] * rho[v];
                dA[v * 3 + c] += pref * ((ure * cph - uim * sph) - wv * (Sh * sph + Shi * cph));
            }
        }
    }
    if (i == j) {
        const double self = 4.0 * S.gamma * S.gamma * S.gamma / (3.0 * SQRT_PI);
        P -= self * (Mr[0] + Mr[4] + Mr[8]);
    }
    if (!qv_ok) return;
    out[0] = P;
    for (int c = 0; c < 3; c++) out[1 + c] = dR[c];
    for (int k = 0; k < 9; k++) out[4 + k] = dA[k];
    out[13] = P0;
}

// per-atom reduction in a fixed order; atom N (one extra block) sums the lattice term
__global__ __launch_bounds__(256) void mbd_grad_periodic_reduce_kernel(const SysDesc* sd, int nq, const double* qmult,
                                                                         double wq, const double* om,
                                                                         const double* cc, const double* part,
                                                                         MatBatch<double> M) {
    __shared__ double red[4];
    const SysDesc& S = sd[0];
    const int N = S.N;
    if (N == 0) return;
    const int k = blockIdx.x;
    if (k < N) {
        double g0 = 0, g1 = 0, g2 = 0, ga = 0, gv = 0, tr = 0;
        const long long NN = (long long)N * N;
        for (long long idx = threadIdx.x; idx < (long long)nq * N; idx += 256) {
            const int q = (int)(idx / N), o = (int)(idx % N);
            // k as j (second index), partner i = o
            const double* pj = part + ((long long)q * NN + (long long)k * N + o) * PER_PART;   // pid = i + j*N: i=o, j=k
            const double* pi = part + ((long long)q * NN + (long long)o * N + k) * PER_PART;   // i=k, j=o
            const double cj = qmult[q] * cc[S.atom_off + o] * cc[S.atom_off + k];
            if (o != k) {
                g0 += cj * (pj[1] - pi[1]);
                g1 += cj * (pj[2] - pi[2]);
                g2 += cj * (pj[3] - pi[3]);
            }
            ga += cj * (pj[0] + pi[0]);
            gv += cj * (pj[13] + pi[13]);
        }
        // Re Tr M_kk(q), summed over q
        for (int q = threadIdx.x; q < nq; q += 256) {
            const double* Mb = M.at(q);
            for (int c = 0; c < 3; c++) tr += qmult[q] * Mb[(3 * k + c) + (long long)(3 * k + c) * M.ld];
        }
        g0 = block_sum256(g0, red);
        g1 = block_sum256(g1, red);
        g2 = block_sum256(g2, red);
        ga = block_sum256(ga, red);
        gv = block_sum256(gv, red);
        tr = block_sum256(tr, red);
        if (threadIdx.x == 0) {
            if (S.grad_coords) {
                S.grad_coords[3 * k] = wq * g0;
                S.grad_coords[3 * k + 1] = wq * g1;
                S.grad_coords[3 * k + 2] = wq * g2;
            }
            const double a0 = S.alpha0[k];
            const double w = om[S.atom_off + k];
            const double dEda = wq * ga / (2.0 * a0);
            const double dEdw = wq * ga / w + wq * 2.0 * w * tr - 1.5;
            if (S.param_kind == 1) {
                // omega = 4 C6/(3 alpha0^2)
                if (S.grad_alpha0) S.grad_alpha0[k] = dEda - 2.0 * w / a0 * dEdw;
                if (S.grad_omega) S.grad_omega[k] = dEdw * w / S.omega_or_c6[k];
            } else {
                if (S.grad_alpha0) S.grad_alpha0[k] = dEda;
                if (S.grad_omega) S.grad_omega[k] = dEdw;
            }
            if (S.grad_rvdw) S.grad_rvdw[k] = wq * S.beta * gv;
        }
    } else {
        double la[9];
        for (int v = 0; v < 9; v++) la[v] = 0.0;
        const long long total = (long long)nq * N * N;
        for (long long idx = threadIdx.x; idx < total; idx += 256) {
            const long long pid = idx % ((long long)N * N);
            const int i = (int)(pid % N), j = (int)(pid / N);
            const double cij = qmult[idx / ((long long)N * N)] * cc[S.atom_off + i] * cc[S.atom_off + j];
            const double* p = part + idx * PER_PART;
            for (int v = 0; v < 9; v++) la[v] += cij * p[4 + v];
        }
        for (int v = 0; v < 9; v++) {
            const double s = block_sum256(la[v], red);
            if (threadIdx.x == 0 && S.grad_lattice) S.grad_lattice[v] = wq * s;
        }
    }
}

// lanes per atom pair: the q count rounded up to a power of two, at most 64
static int per_lanes_per_pair(int nq) {
    int l = 1;
    while (l < nq && l < PER_LANES) l *= 2;
    return l;
}

void mbd_assemble_periodic_launch(hipStream_t st, const SysDesc* sd, const double* om, const double* cc,
                                  const double* qcart, int nq, const int* img, int nimg, const int* rec,
                                  int nrec, MatBatch<double> Q, MatBatch<float> Q32, unsigned* status, int N) {
    const long long pairs = (long long)N * N;
    const int lpp = per_lanes_per_pair(nq), ppw = PER_LANES / lpp;
    hipLaunchKernelGGL(mbd_assemble_periodic_kernel, dim3((unsigned)((pairs + ppw - 1) / ppw), (nq + lpp - 1) / lpp),
                       dim3(PER_LANES), 0, st, sd, om, cc, qcart, nq, lpp, img, nimg, rec, nrec, Q, Q32, status);
}

void mbd_grad_periodic_launch(hipStream_t st, const SysDesc* sd, const double* om, const double* cc,
                              const double* qcart, const double* qmult, double wq, int nq, const int* img,
                              int nimg, const int* rec, int nrec, MatBatch<double> M, double* partial, int N) {
    const long long pairs = (long long)N * N;
    const int lpp = per_lanes_per_pair(nq), ppw = PER_LANES / lpp;
    hipLaunchKernelGGL(mbd_grad_periodic_kernel, dim3((unsigned)((pairs + ppw - 1) / ppw), (nq + lpp - 1) / lpp),
                       dim3(PER_LANES), 0, st, sd, om, cc, qcart, nq, lpp, img, nimg, rec, nrec, M, partial);
    hipLaunchKernelGGL(mbd_grad_periodic_reduce_kernel, dim3(N + 1), dim3(256), 0, st, sd, nq, qmult, wq, om, cc,
                       partial, M);
}
