// Workspace descriptors and launch entry points of the MBD kernels (internal).
#pragma once
#include "mbd_internal.h"

#define SYTRD_NBP 32     // Householder panel width
#define ORMTR_NBB 64     // reflectors per compact-WY block in the back-transform
#define ORMTR_CHUNK 512  // rows per split-K chunk of V^T X

// --- Householder tridiagonalisation --------------------------------------
template <typename T>
struct SytrdWs {
    MatBatch<T> A;     // matrices, lower triangle used, overwritten by reflectors
    const int* ns;     // per-matrix order (device)
    int nmax, nbk_max, maxchunk;
    T* Vp; T* Wp; int ldp; long long sP;   // panels, column-major nmax x SYTRD_NBP
    T* colbuf; long long sC;               // updated current column
    T* normpart; long long sNP;            // per 64-row block squared norms
    T* P1; long long sP1;                  // row-sum partial per tile [nbk][nbk][64]
    T* P2; long long sP2;                  // column-sum partial per chunk [nbk][maxchunk][64]
    T* PS; long long sPS;                  // panel products per block [nbk][2*NBP]
    T* PV; long long sPV;                  // v^T A v partial per workgroup
    T* d; T* e; T* tau; long long sD;      // outputs
};
template <typename T>
void sytrd_launch(const SytrdWs<T>& w, int nbatch, int nmax, hipStream_t st);

// --- Divide and conquer ------------------------------------------------------
template <typename T>
struct StedcWs {
    const int* ns;
    int nmax;
    const T* d_in; const T* e_in; long long sDin;
    T* D; T* E; long long sV;     // per-matrix vectors of length nmax (stride sV)
    T* scale;                     // [nbatch]
    MatBatch<T> Z0, Z1, U;        // eigenvector ping-pong and secular vector blocks
    T* ds; T* zs; T* dn; T* zn; T* mu; T* lam; T* zh; T* rho; T* rc; T* rs;
    int* perm; int* ndpos; int* dfpos; int* org; int* outnd; int* outdf; int* rp; int* rq;
    int* Kcnt; int* rotcnt;
    T* w_out; long long sW;       // eigenvalues (ascending) out
};
// Returns 0 if the eigenvectors ended in Z0, 1 if in Z1.
template <typename T>
int stedc_launch(const StedcWs<T>& w, int nbatch, int nmax, hipStream_t st);

// --- Back-transformation ---------------------------------------------------
template <typename T>
struct OrmtrWs {
    MatBatch<T> A;     // reflectors (columns below the diagonal, implicit unit)
    const T* tau; long long sD;
    const int* ns;
    MatBatch<T> X;     // in: tridiagonal eigenvectors; out: eigenvectors of A
    T* Gpart; long long sG;   // [nsplit][64*64]
    T* Tm; long long sT;      // [64*64]
    T* Ypart; long long sYp;  // [nsplit][64*nmax]
    T* Y; long long sY;       // [64*nmax]
    int nmax;
};
template <typename T>
void ormtr_launch(const OrmtrWs<T>& w, int nbatch, int nmax, hipStream_t st);

// --- generic batched GEMM (C = alpha op(A) op(B) + beta C, order ns[b]) ------
template <typename T>
void gemm_batched(hipStream_t st, bool ta, bool tb, const int* ns, int nmax, int nbatch,
                  const T* A, int lda, long long sA, const T* B, int ldb, long long sB, T* C,
                  int ldc, long long sC, T alpha, T beta, bool lower_only);
