// Pairwise (TS) dispersion energy and gradients (paper Sec. 2.6):
//   E = -1/2 sum_{i != j} C6_ij f(R_ij) / R_ij^6,
//   C6_ij = (3/2) alpha_i alpha_j / (1/omega_i + 1/omega_j)        (eq:pairwise)
//   f = 1/(1 + exp(-a (R/(s_R (Rv_i + Rv_j)) - 1))), TS: a = 20     (eq:fermi-damping)
// Periodic systems (energy per cell) sum over every image, the term n = 0,
// i = j excluded: the undamped R^-6 lattice sum by the Ewald split of
// eq:ts-ewald,
//   sum'_n R^-6 = sum_{0<|x_n|<Rc} gamma^6 phi_r(gamma |x_n|)
//               + (1/Omega) sum_{|G|<kc, G = 0 included} gamma^3 phi_k(|G|/gamma) cos(G.r)
//               - delta_ij gamma^6/6,
//   phi_r(z) = (z^-6 + z^-4 + z^-2/2) e^{-z^2},
//   phi_k(k) = (pi^{3/2}/12)((4 - 2k^2) e^{-k^2/4} + k^3 sqrt(pi) erfc(k/2)),
// minus the real-space sum of (1 - f)/R^6 over every image with (1-f) > 1e-18
// (the damped lattice sum exactly).  The G = 0 term, the sign of the self term
// and the cosine argument are read from the derivation of the split; the
// printed formula omits G = 0 and has them garbled.
//
// Atom i's row of (j, term) pairs is shared by one workgroup, so the atom's
// energy share, its gradient and its parameter derivatives come out of one
// block reduction each (each ordered pair's energy is counted at i; dE/dR_i =
// sum_j C6_ij grad S_ij(R_j - R_i) gathers both orders).  A finite row has
// one term per pair, so its 256 lanes take about N/256 pairs each and the
// N workgroups keep several wavefronts on every SIMD to hide the neighbour
// loads.  Per pair the divisions are shared: C6 and its omega derivative
// through 1/(omega_i + omega_j), the Fermi factor through 1/R0 and
// 1/(1 + e^{-|x|}), and 1/R.
#include "mbd_internal.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"

#define TS_DAMP_TAIL 1e-18
#define TS_SQRT_PI 1.7724538509055160273

// f = 1/(1 + e^{-x}), x = a (d/R0 - 1), with 1 - f and the derivatives in d
// and R0, from e = e^{-|x|} (no overflow on either side)
__device__ __forceinline__ void ts_fermi(double d, double R0, double a, double& f, double& omf, double& df_dd,
                                         double& df_dR0) {
    if (R0 <= 0.0) { f = 1.0; omf = 0.0; df_dd = 0.0; df_dR0 = 0.0; return; }
    const double iR0 = 1.0 / R0;
    const double x = a * (d * iR0 - 1.0);
    const double e = exp(-fabs(x));
    const double p = 1.0 / (1.0 + e);
    if (x >= 0.0) { f = p; omf = e * p; }
    else { f = e * p; omf = p; }
    const double ff = a * iR0 * (f * omf);
    df_dd = ff;
    df_dR0 = -d * iR0 * ff;
}

// one instance per case, so the finite kernel carries none of the lattice
// code's registers
template <bool periodic>
__global__ __launch_bounds__(256) void mbd_ts_kernel(const SysDesc* sd, const double* om, const int* img, int nimg,
                                                       const int* rec, int nrec, double* eatom, unsigned* status) {
    __shared__ double red[4];
    const SysDesc& S = sd[0];
    const int N = S.N;
    const int i = blockIdx.x;
    const int t0 = (int)threadIdx.x;
    if (i >= N) return;
    const double* R = S.coords;
    const double ai = S.alpha0[i], wi = om[S.atom_off + i], rvi = S.rvdw[i];
    const double iwi = 1.0 / wi;
    const double g = S.gamma, g3 = g * g * g, g6 = g3 * g3;
    const int nterm = periodic ? nimg + nrec : 1;
    double Ei = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, dw = 0.0, dv = 0.0;
    // lane steps of 256 over the flat (j, term) index, carried into j
    // without an integer division per step (finite: one term per pair)
    int j = periodic ? t0 / nterm : t0, u = periodic ? t0 % nterm : 0;
    auto advance = [&]() {
        if (!periodic) { j += 256; return; }
        u += 256;
        while (u >= nterm) { u -= nterm; j++; }
    };
    for (; j < N; advance()) {
        if (!periodic && j == i) continue;
        const double r[3] = {R[3 * j] - R[3 * i], R[3 * j + 1] - R[3 * i + 1], R[3 * j + 2] - R[3 * i + 2]};
        const double aj = S.alpha0[j], wj = om[S.atom_off + j];
        // C6 = (3/2) ai aj wi wj/(wi + wj); dC6/dwi = C6 wj/(wi (wi + wj))
        const double h = 1.0 / (wi + wj);
        const double c6 = 1.5 * ai * aj * wi * wj * h;
        const double c6w = c6 * wj * h * iwi;
        const double R0 = S.beta * (rvi + S.rvdw[j]);
        if (periodic && j == i && u == 0) {
            // self term -gamma^6/6 of the reciprocal sum, once per atom
            Ei += -0.5 * c6 * (-g6 / 6.0);
            dw += -c6w * (-g6 / 6.0);
        }
        double s = 0.0, ds[3] = {0.0, 0.0, 0.0}, ds0 = 0.0;
        if (!periodic || u < nimg) {
            double x[3] = {r[0], r[1], r[2]};
            if (periodic)
                for (int c = 0; c < 3; c++)
                    x[c] += img[3 * u] * S.lat[c] + img[3 * u + 1] * S.lat[3 + c] + img[3 * u + 2] * S.lat[6 + c];
            const double d2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            if (d2 == 0.0) {  // n = 0, i = j; any other zero distance is a coincident pair
                if (j != i) atomicOr(&status[0], MBD_ST_COINCIDENT);
                continue;
            }
            double d = sqrt(d2);
            if (!(d >= 1e-8)) {
                atomicOr(&status[0], MBD_ST_COINCIDENT);
                continue;
            }
            const double id = 1.0 / d, id2 = id * id, id6 = id2 * id2 * id2;
            double f, omf, fd, fR0;
            ts_fermi(d, R0, S.a, f, omf, fd, fR0);
            double dd = 0.0;
            if (!periodic) {
                s = f * id6;
                dd = fd * id6 - 6.0 * f * id6 * id;
                ds0 = fR0 * id6;
            } else {
                if (d < S.rc) {
                    const double z = g * d, iz = 1.0 / z, iz2 = iz * iz, ez = exp(-z * z);
                    s += g6 * (iz2 * iz2 * iz2 + iz2 * iz2 + 0.5 * iz2) * ez;
                    dd += -g6 * g * (6.0 * iz2 * iz2 * iz2 * iz + 6.0 * iz2 * iz2 * iz + 3.0 * iz2 * iz + iz) * ez;
                }
                if (omf > TS_DAMP_TAIL) {
                    s -= omf * id6;
                    dd += fd * id6 + 6.0 * omf * id6 * id;
                    ds0 = fR0 * id6;
                }
            }
            for (int c = 0; c < 3; c++) ds[c] = dd * x[c] * id;
        } else {
            const int m = u - nimg;
            double G[3];
            for (int c = 0; c < 3; c++)
                G[c] = rec[3 * m] * S.recip[c] + rec[3 * m + 1] * S.recip[3 + c] + rec[3 * m + 2] * S.recip[6 + c];
            const double k = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
            if (k >= S.kc) continue;
            const double kk = k / g;
            const double phik = (TS_SQRT_PI * TS_SQRT_PI * TS_SQRT_PI / 12.0) *
                                ((4.0 - 2.0 * kk * kk) * exp(-0.25 * kk * kk) + kk * kk * kk * TS_SQRT_PI * erfc(0.5 * kk));
            const double w = g3 * phik / S.vol;
            double sn, cs;
            sincos(G[0] * r[0] + G[1] * r[1] + G[2] * r[2], &sn, &cs);
            s = w * cs;
            for (int c = 0; c < 3; c++) ds[c] = -w * sn * G[c];
        }
        Ei += -0.5 * c6 * s;
        gx += c6 * ds[0];
        gy += c6 * ds[1];
        gz += c6 * ds[2];
        dw += -c6w * s;
        dv += -S.beta * c6 * ds0;
    }
    Ei = block_sum256(Ei, red);
    gx = block_sum256(gx, red);
    gy = block_sum256(gy, red);
    gz = block_sum256(gz, red);
    dw = block_sum256(dw, red);
    dv = block_sum256(dv, red);
    if (t0 == 0) {
        eatom[i] = Ei;
        if (S.grad_coords) {
            S.grad_coords[3 * i] = gx;
            S.grad_coords[3 * i + 1] = gy;
            S.grad_coords[3 * i + 2] = gz;
        }
        const double dEda = 2.0 * Ei / ai;
        if (S.param_kind == 1) {
            // omega = 4 C6/(3 alpha0^2)
            if (S.grad_alpha0) S.grad_alpha0[i] = dEda - 2.0 * wi / ai * dw;
            if (S.grad_omega) S.grad_omega[i] = dw * wi / S.omega_or_c6[i];
        } else {
            if (S.grad_alpha0) S.grad_alpha0[i] = dEda;
            if (S.grad_omega) S.grad_omega[i] = dw;
        }
        if (S.grad_rvdw) S.grad_rvdw[i] = dv;
    }
}

// energy = sum of the per-atom shares, in a fixed order; errors[0..3] = 0
__global__ __launch_bounds__(256) void mbd_ts_sum_kernel(const SysDesc* sd, const double* eatom,
                                                           const unsigned* status) {
    __shared__ double red[4];
    const SysDesc& S = sd[0];
    double e = 0.0;
    for (int i = threadIdx.x; i < S.N; i += 256) e += eatom[i];
    e = block_sum256(e, red);
    if (threadIdx.x == 0) {
        if (S.energy) *S.energy = status[0] ? __longlong_as_double(0x7ff8000000000000LL) : e;
        if (S.errors)
            for (int k = 0; k < 4; k++) S.errors[k] = 0.0;
    }
}

void mbd_ts_launch(hipStream_t st, const SysDesc* sd, int N, const double* om, const int* img, int nimg,
                   const int* rec, int nrec, int periodic, double* eatom, unsigned* status, LaunchProfiler* prof) {
    auto kern = periodic ? mbd_ts_kernel<true> : mbd_ts_kernel<false>;
    if (prof && prof->enabled && prof->launches) {
        // work: the pair terms of the launch
        const double terms = periodic ? (double)N * N * (nimg + nrec) : (double)N * (N - 1);
        hipEvent_t e0, e1;
        prof->pair(&e0, &e1, 11, terms);
        hipExtLaunchKernelGGL(kern, dim3(N), dim3(256), 0, st, e0, e1, 0, sd, om, img, nimg, rec, nrec, eatom,
                              status);
    } else {
        hipLaunchKernelGGL(kern, dim3(N), dim3(256), 0, st, sd, om, img, nimg, rec, nrec, eatom, status);
    }
    hipLaunchKernelGGL(mbd_ts_sum_kernel, dim3(1), dim3(256), 0, st, sd, eatom, status);
}
