// Periodic systems: Q(q) of eq:q-matrix with T^lr(q) the Bloch sum of g T
// (paper Sec. 2.2), evaluated with the Ewald split of eq:ewald/eq:terfc plus
// a real-space damping correction, for every q of the mesh, and the matching
// adjoint contraction for dE/dR, dE/dalpha0 and dE/dA (lattice).
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
// The reciprocal-space term is a sum of rank-one 3x3 blocks k k^T times a
// pair phase, so over all pairs it is the low-rank product U U^H with
// U_{ia,g} = sqrt(w_g) k_a e^{-i G_g.R_i}, w = (4 pi/Omega) e^{-k^2/(4 gamma^2)}/k^2,
// one column per reciprocal vector of the q point's sphere.  It is formed on
// the matrix cores (a product over the ~265 columns instead of that many
// exponentials and phases per pair and q), and the adjoint contracts M with U
// the same way: W = M C U, then per atom and column a few products of U and W.
//
// The Hermitian Q(q) is stored as its real embedding [[Re, -Im], [Im, Re]]
// (order 2n) so the batched real eigensolver serves it; every eigenvalue of
// Q(q) appears twice.  The reciprocal sums are evaluated in FP64.
#include "gemm_mfma.h"
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
// nothing.  Writes the real-space and self terms and omega^2 into the left
// block column [Re; Im] of the embedding; the reciprocal-space product then
// adds its term and fills the right block column.
#define PER_LANES 64
__global__ __launch_bounds__(PER_LANES) void mbd_assemble_periodic_kernel(const SysDesc* sd, const double* om,
                                                                          const double* cc, const double* qcart,
                                                                          int nq, int lpp, const int* img, int nimg,
                                                                          const double* phase, MatBatch<double> Q,
                                                                          unsigned* status) {
    __shared__ double Fs[PER_LANES][9];
    __shared__ int oks[PER_LANES];   // image index + 1 of the slot's term, 0 if empty
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
    // e^{-i q.x} = e^{-i q.r} e^{-i q.R_n}, the second factor from the table
    double sb, cb;
    sincos(-(qv[0] * r[0] + qv[1] * r[1] + qv[2] * r[2]), &sb, &cb);
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
                        ok = t + 1;
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
            const double* pt = phase + 2 * ((long long)(oks[u] - 1) * nq + qc);
            const double cph = cb * pt[0] - sb * pt[1], sph = cb * pt[1] + sb * pt[0];
            for (int k = 0; k < 9; k++) { Tre[k] += Fs[u][k] * cph; Tim[k] += Fs[u][k] * sph; }
        }
        __syncthreads();
    }
    if (!qv_ok) return;
    if (i == j) {
        const double self = 4.0 * S.gamma * S.gamma * S.gamma / (3.0 * SQRT_PI);
        Tre[0] -= self; Tre[4] -= self; Tre[8] -= self;
    }
    // without cc and om: the lattice sum T(q) itself (c = 1, no omega^2)
    const double pc = cc ? cc[S.atom_off + i] * cc[S.atom_off + j] : 1.0;
    double* Qb = Q.at(q);
    const long long ld = Q.ld;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            const double re = pc * Tre[a * 3 + b] +
                              ((om && i == j && a == b) ? om[S.atom_off + i] * om[S.atom_off + i] : 0.0);
            const long long r0 = 3 * i + a, c0 = 3 * j + b;
            Qb[r0 + c0 * ld] = re;
            Qb[(r0 + n) + c0 * ld] = pc * Tim[a * 3 + b];
        }
}

// Reciprocal vector and weights of column g of q point q's list (t >= 0):
// G, k = G + q, sw = sqrt(w), w = (4 pi/Omega) e^{-k^2/(4 gamma^2)}/k^2, and
// f = (dw/dk_d)/(w k_d) = -1/(2 gamma^2) - 2/k^2.
__device__ __forceinline__ void recip_column(const SysDesc& S, const int* rec, int t, const double* qv, double* G,
                                             double* k, double& sw, double& f) {
    const double m0 = rec[3 * t], m1 = rec[3 * t + 1], m2 = rec[3 * t + 2];
    for (int c = 0; c < 3; c++) {
        G[c] = m0 * S.recip[c] + m1 * S.recip[3 + c] + m2 * S.recip[6 + c];
        k[c] = G[c] + qv[c];
    }
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const double g4 = 1.0 / (4.0 * S.gamma * S.gamma);
    sw = sqrt(4.0 * M_PI / S.vol * exp(-k2 * g4) / k2);
    f = -2.0 * g4 - 2.0 / k2;
}

// Columns of U(q), embedded: rows 0 .. n-1 Re U, rows n .. 2n-1 Im U; the
// columns past the q point's count are zero.  Grid (ncol, nq), 64 threads
// over the atoms.
__global__ __launch_bounds__(64) void per_recip_basis_kernel(const SysDesc* sd, const double* qcart, PerEwald pr) {
    const SysDesc& S = sd[0];
    const int N = S.N, n = 3 * N;
    const int g = blockIdx.x, q = blockIdx.y;
    double* Zc = pr.Z + (long long)q * pr.sZ + (long long)g * pr.ldz;
    const int t = pr.col[(long long)q * pr.ncol + g];
    double G[3] = {0.0, 0.0, 0.0}, k[3] = {0.0, 0.0, 0.0}, sw = 0.0, f;
    if (t >= 0) recip_column(S, pr.rec, t, qcart + 3 * q, G, k, sw, f);
    const double* R = S.coords;
    for (int i = threadIdx.x; i < N; i += 64) {
        double sn = 0.0, cs = 1.0;
        if (t >= 0) sincos(G[0] * R[3 * i] + G[1] * R[3 * i + 1] + G[2] * R[3 * i + 2], &sn, &cs);
        for (int a = 0; a < 3; a++) {
            Zc[3 * i + a] = sw * k[a] * cs;      // e^{-i G.R} = cos - i sin
            Zc[n + 3 * i + a] = -sw * k[a] * sn;
        }
    }
}

// Real-space phases: phase[t][q] = (cos, sin) of -q.R_n for image t, so that
// the lanes of a pair (one q each) read consecutive entries.
__global__ __launch_bounds__(256) void per_phase_kernel(const SysDesc* sd, const double* qcart, int nq,
                                                        const int* img, int nimg, double* phase) {
    const SysDesc& S = sd[0];
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)nimg * nq) return;
    const int t = (int)(e / nq), q = (int)(e % nq);
    double Rn[3];
    for (int c = 0; c < 3; c++) Rn[c] = img[3 * t] * S.lat[c] + img[3 * t + 1] * S.lat[3 + c] + img[3 * t + 2] * S.lat[6 + c];
    double sn, cs;
    sincos(-(qcart[3 * q] * Rn[0] + qcart[3 * q + 1] * Rn[1] + qcart[3 * q + 2] * Rn[2]), &sn, &cs);
    phase[2 * e] = cs;
    phase[2 * e + 1] = sn;
}

// Reciprocal term of the embedding: [Re; Im] of C U U^H C is [U_r, -U_i;
// U_i, U_r] times the first n rows of the same, transposed (K = 2 ncol), so
// one product per q over the left block column.  The epilogue adds it to the
// real-space part there, mirrors it into the right block column (Re to the
// bottom right, -Im to the top right) and writes the FP32 copy.
struct PerRecAsmProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = true;
    const SysDesc* sd;
    const double* cc;
    const double* Z; int ldz; long long sZ; int ncol; int n;
    MatBatch<double> Q; MatBatch<float> Q32;
    int tiles_m, tiles_n;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        int ti, tj;
        band_tile(xcd_virtual(bx, gridDim.x), tiles_m, tiles_n, ti, tj);
        t.batch = bz;
        t.m0 = ti * GEMM_BM; t.n0 = tj * GEMM_BN; t.K = 2 * ncol;
        return t.m0 < 2 * n && t.n0 < n;
    }
    // row m, column k of [U_r, -U_i; U_i, U_r]
    __device__ double zf(const GemmTile& t, int m, int k) const {
        const double* Zb = Z + (long long)t.batch * sZ;
        if (k < ncol) return Zb[m + (long long)k * ldz];
        const long long o = (long long)(k - ncol) * ldz;
        return m < n ? -Zb[m + n + o] : Zb[m - n + o];
    }
    __device__ double a(const GemmTile& t, int m, int k) const { return (m < 2 * n && k < t.K) ? zf(t, m, k) : 0.0; }
    __device__ double b(const GemmTile& t, int k, int c) const { return (c < n && k < t.K) ? zf(t, c, k) : 0.0; }
    __device__ void store(const GemmTile& t, int m, int c, double v) const {
        if (m >= 2 * n || c >= n) return;
        const bool top = m < n;
        const int off = sd->atom_off;
        const int i = (top ? m : m - n) / 3, j = c / 3;
        double* Qb = Q.at(t.batch);
        const long long ld = Q.ld;
        const double val = Qb[m + (long long)c * ld] + (cc ? cc[off + i] * cc[off + j] : 1.0) * v;
        const int mm = top ? m + n : m - n;
        const double mv = top ? val : -val;
        Qb[m + (long long)c * ld] = val;
        Qb[mm + (long long)(c + n) * ld] = mv;
        if (Q32.p) {
            float* Qf = Q32.at(t.batch);
            Qf[m + (long long)c * Q32.ld] = (float)val;
            Qf[mm + (long long)(c + n) * Q32.ld] = (float)mv;
        }
    }
};

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
// Partial results per (q, i, j) of the real-space and self terms: {P, dR[3],
// dA[9], P0}; the reciprocal-space term is contracted through U below.
// Same layout as the assembly: one workgroup per ordered pair, one lane per
// q-point, each real-space image term (F and its derivatives) formed once
// into LDS and added by every lane with its own phase and M(q).  Two
// wavefronts per SIMD (at most 256 registers, a few spilled: 587 -> 519 us
// for the 64-atom cell's 64 q against one wavefront at 268 registers).
__global__ __launch_bounds__(PER_LANES, 2) void mbd_grad_periodic_kernel(const SysDesc* sd, const double* om,
                                                                      const double* cc, const double* qcart, int nq,
                                                                      int lpp, const int* img, int nimg,
                                                                      const double* phase, MatBatch<double> M,
                                                                      double* part) {
    __shared__ double Fs[PER_LANES][9], dFs[PER_LANES][27], F0s[PER_LANES][9];
    __shared__ int ns_[PER_LANES][3], oks[PER_LANES];   // oks: image index + 1 of the slot's term, 0 if empty
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
    // e^{-i q.x} = e^{-i q.r} e^{-i q.R_n}, the second factor from the table
    double sb, cb;
    sincos(-(qv[0] * r[0] + qv[1] * r[1] + qv[2] * r[2]), &sb, &cb);
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
                // the term is written straight into this lane's slot
                if (d2 != 0.0 && image_term(x, S.gamma, S.rc, R0, S.a, Fs[threadIdx.x], dFs[threadIdx.x], F0s[threadIdx.x])) {
                    ok = t + 1;
                    for (int c = 0; c < 3; c++) ns_[threadIdx.x][c] = nn[c];
                }
            }
            oks[threadIdx.x] = ok;
        }
        __syncthreads();
        const int tn = min(lpp, nimg - t0);
        for (int u0 = 0; u0 < tn; u0++) {
        const int u = slot * lpp + u0;
        if (!oks[u]) continue;
        const double* F = Fs[u];
        const double* dF = dFs[u];
        const int* nn = ns_[u];
        const double* pt = phase + 2 * ((long long)(oks[u] - 1) * nq + q);
        const double cph = cb * pt[0] - sb * pt[1], sph = cb * pt[1] + sb * pt[0];
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

// Reciprocal term of the adjoint, W = M C U: M(q) the full embedded inverse
// square root (2n x 2n), C U the basis with row (i, a) scaled by c_i;
// W (2n x ncol) is [Re; Im] of the complex product.
struct PerRecMZProb {
    static constexpr bool A_M_CONTIG = true;
    static constexpr bool B_N_CONTIG = false;
    const SysDesc* sd;
    const double* cc;
    MatBatch<double> M;
    const double* Z; double* W; int ldz; long long sZ; int ncol; int n;
    int tiles_m, tiles_n;
    __device__ bool tile(int bx, int, int bz, GemmTile& t) const {
        int ti, tj;
        band_tile(xcd_virtual(bx, gridDim.x), tiles_m, tiles_n, ti, tj);
        t.batch = bz;
        t.m0 = ti * GEMM_BM; t.n0 = tj * GEMM_BN; t.K = 2 * n;
        return t.m0 < 2 * n && t.n0 < ncol;
    }
    __device__ double a(const GemmTile& t, int m, int k) const {
        return (m < 2 * n && k < 2 * n) ? M.at(t.batch)[m + (long long)k * M.ld] : 0.0;
    }
    __device__ double b(const GemmTile& t, int k, int g) const {
        if (k >= 2 * n || g >= ncol) return 0.0;
        return cc[sd->atom_off + (k < n ? k : k - n) / 3] * Z[(long long)t.batch * sZ + k + (long long)g * ldz];
    }
    __device__ void store(const GemmTile& t, int m, int g, double v) const {
        if (m < 2 * n && g < ncol) W[(long long)t.batch * sZ + m + (long long)g * ldz] = v;
    }
};

// Reciprocal term of the adjoint, per atom k and column g (k = G + q,
// u = U_{k., g}, z = c_k sum_a conj(u_a) W_{ka, g}):
//   dE/dalpha, dE/domega partial  2 Re z (the pair sum over both orders)
//   dE/dR_k                        -2 G Im z
//   dE/dA_vc  -Ainv_cv s - sum_d Ainv_dv [k_c k_d f s + 2 sw k_c b_d
//             + G_c sum_k R_kd e_k], s = sum_k Re z, e_k = -2 Im z,
//             b_d = sum_k c_k Re(conj(W_{kd,g}) e^{-i G.R_k})
// (derivatives of the weight w, of k and of the pair phase through G with
// the fractional q fixed, and of the prefactor through Omega).  Grid (nq,
// chunks of PER_RCOLS columns); writes per (q, chunk, atom) {2 Re z, dR[3]}
// and per (q, chunk) {s, L[c][d]}, L the bracket's matrix without Ainv.
#define PER_RCOLS 16
__global__ __launch_bounds__(64) void per_recip_grad_kernel(const SysDesc* sd, const double* cc, const double* qcart,
                                                            PerEwald pr, int nchunk, double* rq, double* rl) {
    const SysDesc& S = sd[0];
    const int N = S.N, n = 3 * N;
    const int q = blockIdx.x, ch = blockIdx.y;
    const double* Wq = pr.W + (long long)q * pr.sZ;
    const int* cols = pr.col + (long long)q * pr.ncol;
    const double* qv = qcart + 3 * q;
    const double* R = S.coords;
    const int g0 = ch * PER_RCOLS, g1 = min(pr.ncol, g0 + PER_RCOLS);
    double sre = 0.0, L[9];
    for (int v = 0; v < 9; v++) L[v] = 0.0;
    for (int k = threadIdx.x; k < N; k += 64) {
        const double ck = cc[S.atom_off + k];
        const double Rk[3] = {R[3 * k], R[3 * k + 1], R[3 * k + 2]};
        double ga = 0.0, gr[3] = {0.0, 0.0, 0.0};
        for (int g = g0; g < g1; g++) {
            const int t = cols[g];
            if (t < 0) break;
            double G[3], kv[3], sw, f;
            recip_column(S, pr.rec, t, qv, G, kv, sw, f);
            double sn, cs;
            sincos(G[0] * Rk[0] + G[1] * Rk[1] + G[2] * Rk[2], &sn, &cs);
            const double pr_ = cs, pi_ = -sn;  // e^{-i G.R_k}
            double zr = 0.0, zi = 0.0, bd[3];
            for (int a = 0; a < 3; a++) {
                const double wr = Wq[3 * k + a + (long long)g * pr.ldz];
                const double wi = Wq[n + 3 * k + a + (long long)g * pr.ldz];
                const double ur = sw * kv[a] * pr_, ui = sw * kv[a] * pi_;
                zr += ur * wr + ui * wi;
                zi += ur * wi - ui * wr;
                bd[a] = ck * (wr * pr_ + wi * pi_);
            }
            zr *= ck;
            zi *= ck;
            const double e = -2.0 * zi;
            ga += 2.0 * zr;
            for (int c = 0; c < 3; c++) gr[c] += G[c] * e;
            sre += zr;
            for (int c = 0; c < 3; c++)
                for (int d = 0; d < 3; d++)
                    L[c * 3 + d] += f * zr * kv[c] * kv[d] + 2.0 * sw * kv[c] * bd[d] + e * G[c] * Rk[d];
        }
        double* o = rq + (((long long)q * nchunk + ch) * N + k) * 4;
        o[0] = ga;
        for (int c = 0; c < 3; c++) o[1 + c] = gr[c];
    }
    sre = wave_sum(sre);
    for (int v = 0; v < 9; v++) L[v] = wave_sum(L[v]);
    if (threadIdx.x == 0) {
        double* o = rl + ((long long)q * nchunk + ch) * 10;
        o[0] = sre;
        for (int v = 0; v < 9; v++) o[1 + v] = L[v];
    }
}

// Per-atom reduction in a fixed order: the pair partials (k as either atom)
// over all q, the reciprocal partials of every (q, chunk), and the lattice
// partials of the pairs with k as second atom, to latpart[k].
__global__ __launch_bounds__(256) void mbd_grad_periodic_reduce_kernel(const SysDesc* sd, int nq, const double* qmult,
                                                                         double wq, const double* om,
                                                                         const double* cc, const double* part,
                                                                         MatBatch<double> M, const double* rq,
                                                                         int nchunk, double* latpart) {
    __shared__ double red[4];
    const SysDesc& S = sd[0];
    const int N = S.N;
    if (N == 0) return;
    const int k = blockIdx.x;
    double g0 = 0, g1 = 0, g2 = 0, ga = 0, gv = 0, tr = 0, la[9];
    for (int v = 0; v < 9; v++) la[v] = 0.0;
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
        for (int v = 0; v < 9; v++) la[v] += cj * pj[4 + v];
    }
    for (long long idx = threadIdx.x; idx < (long long)nq * nchunk; idx += 256) {
        const double w = qmult[idx / nchunk];
        const double* r = rq + (idx * N + k) * 4;
        ga += w * r[0];
        g0 += w * r[1];
        g1 += w * r[2];
        g2 += w * r[3];
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
    for (int v = 0; v < 9; v++) la[v] = block_sum256(la[v], red);
    if (threadIdx.x == 0) {
        for (int v = 0; v < 9; v++) latpart[9 * k + v] = la[v];
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
}

// dE/dA: the per-atom pair partials and the reciprocal (q, chunk) partials,
// each summed in a fixed order, the latter contracted with Ainv once.
__global__ __launch_bounds__(256) void mbd_grad_periodic_lattice_kernel(const SysDesc* sd, int nq, int nchunk,
                                                                          const double* qmult, double wq,
                                                                          const double* latpart, const double* rl) {
    __shared__ double red[4];
    const SysDesc& S = sd[0];
    const int N = S.N;
    double la[9], r[10];
    for (int v = 0; v < 9; v++) la[v] = 0.0;
    for (int v = 0; v < 10; v++) r[v] = 0.0;
    for (int k = threadIdx.x; k < N; k += 256)
        for (int v = 0; v < 9; v++) la[v] += latpart[9 * k + v];
    for (long long idx = threadIdx.x; idx < (long long)nq * nchunk; idx += 256) {
        const double w = qmult[idx / nchunk];
        for (int v = 0; v < 10; v++) r[v] += w * rl[idx * 10 + v];
    }
    for (int v = 0; v < 9; v++) la[v] = block_sum256(la[v], red);
    for (int v = 0; v < 10; v++) r[v] = block_sum256(r[v], red);
    if (threadIdx.x != 0 || !S.grad_lattice) return;
    // linv[d * 3 + v] = Ainv[d][v]
    for (int v = 0; v < 3; v++)
        for (int c = 0; c < 3; c++) {
            double t = -S.linv[c * 3 + v] * r[0];
            for (int d = 0; d < 3; d++) t -= S.linv[d * 3 + v] * r[1 + c * 3 + d];
            S.grad_lattice[v * 3 + c] = wq * (la[v * 3 + c] + t);
        }
}

// lanes per atom pair: the q count rounded up to a power of two, at most 64
static int per_lanes_per_pair(int nq) {
    int l = 1;
    while (l < nq && l < PER_LANES) l *= 2;
    return l;
}

void per_recip_basis_launch(hipStream_t st, const SysDesc* sd, const double* qcart, int nq, const int* img,
                            int nimg, const PerEwald& pr) {
    if (nq == 0) return;
    if (nimg > 0)
        hipLaunchKernelGGL(per_phase_kernel, dim3((unsigned)(((long long)nimg * nq + 255) / 256)), dim3(256), 0, st,
                           sd, qcart, nq, img, nimg, pr.phase);
    if (pr.ncol == 0) return;
    hipLaunchKernelGGL(per_recip_basis_kernel, dim3(pr.ncol, nq), dim3(64), 0, st, sd, qcart, pr);
}

void mbd_assemble_periodic_launch(hipStream_t st, const SysDesc* sd, const double* om, const double* cc,
                                  const double* qcart, int nq, const int* img, int nimg, const PerEwald& pr,
                                  MatBatch<double> Q, MatBatch<float> Q32, unsigned* status, int N) {
    const long long pairs = (long long)N * N;
    const int lpp = per_lanes_per_pair(nq), ppw = PER_LANES / lpp;
    hipLaunchKernelGGL(mbd_assemble_periodic_kernel, dim3((unsigned)((pairs + ppw - 1) / ppw), (nq + lpp - 1) / lpp),
                       dim3(PER_LANES), 0, st, sd, om, cc, qcart, nq, lpp, img, nimg, pr.phase, Q, status);
    // always launched: besides the reciprocal term, the epilogue fills the
    // right block column and the FP32 copy
    PerRecAsmProb p;
    p.sd = sd; p.cc = cc; p.Z = pr.Z; p.ldz = pr.ldz; p.sZ = pr.sZ; p.ncol = pr.ncol; p.n = 3 * N;
    p.Q = Q; p.Q32 = Q32;
    p.tiles_m = (6 * N + GEMM_BM - 1) / GEMM_BM;
    p.tiles_n = (3 * N + GEMM_BN - 1) / GEMM_BN;
    hipLaunchKernelGGL((gemm_mfma_kernel<double, PerRecAsmProb>), dim3(p.tiles_m * p.tiles_n, 1, nq), dim3(256), 0,
                       st, p);
}

int per_recip_chunks(int ncol) { return (ncol + PER_RCOLS - 1) / PER_RCOLS; }

void mbd_grad_periodic_launch(hipStream_t st, const SysDesc* sd, const double* om, const double* cc,
                              const double* qcart, const double* qmult, double wq, int nq, const int* img,
                              int nimg, const PerEwald& pr, MatBatch<double> M, double* partial, double* rq,
                              double* rl, double* latpart, int N) {
    const long long pairs = (long long)N * N;
    const int lpp = per_lanes_per_pair(nq), ppw = PER_LANES / lpp;
    hipLaunchKernelGGL(mbd_grad_periodic_kernel, dim3((unsigned)((pairs + ppw - 1) / ppw), (nq + lpp - 1) / lpp),
                       dim3(PER_LANES), 0, st, sd, om, cc, qcart, nq, lpp, img, nimg, pr.phase, M, partial);
    const int nchunk = per_recip_chunks(pr.ncol);
    if (nchunk > 0) {
        PerRecMZProb p;
        p.sd = sd; p.cc = cc; p.M = M; p.Z = pr.Z; p.W = pr.W; p.ldz = pr.ldz; p.sZ = pr.sZ; p.ncol = pr.ncol;
        p.n = 3 * N;
        p.tiles_m = (6 * N + GEMM_BM - 1) / GEMM_BM;
        p.tiles_n = (pr.ncol + GEMM_BN - 1) / GEMM_BN;
        hipLaunchKernelGGL((gemm_mfma_kernel<double, PerRecMZProb>), dim3(p.tiles_m * p.tiles_n, 1, nq), dim3(256),
                           0, st, p);
        hipLaunchKernelGGL(per_recip_grad_kernel, dim3(nq, nchunk), dim3(64), 0, st, sd, cc, qcart, pr, nchunk, rq,
                           rl);
    }
    hipLaunchKernelGGL(mbd_grad_periodic_reduce_kernel, dim3(N), dim3(256), 0, st, sd, nq, qmult, wq, om, cc,
                       partial, M, rq, nchunk, latpart);
    hipLaunchKernelGGL(mbd_grad_periodic_lattice_kernel, dim3(1), dim3(256), 0, st, sd, nq, nchunk, qmult, wq,
                       latpart, rl);
}
