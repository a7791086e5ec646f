// Workspace descriptors and launch entry points of the MBD kernels (internal).
#pragma once
#include "mbd_internal.h"

#include <chrono>
#include <vector>
#include <hip/hip_ext.h>

// Optional HIP-event timing of individual launches and of whole phases
// (measurement tools only).  kind 0: per-column SYMV of the reduction
// (BLAS-2), 1: trailing SYR2K (BLAS-3); phases: 2 input preparation and
// assembly, 3 Householder reduction, 4 divide and conquer, 5 back-transform,
// 6 refinement, 7 energy, Q^{-1/2} and gradients; 8 fused per-column
// launch, 9 screening stage, 10 one-workgroup-per-matrix reduction, 11 the
// pairwise (TS) kernel.  `work` is the algorithmic bytes (kinds 0, 8, 10),
// flops (kind 1) or pair terms (kind 11) of the launch, 0 for phases.
#define PROF_KINDS 12
struct LaunchProfiler {
    bool enabled = false;
    bool launches = true;  // per-launch records (kinds 0, 1); phases are always recorded when enabled
    std::vector<hipEvent_t> pool;
    std::vector<int> kind;
    std::vector<double> work;
    size_t used = 0;
    std::vector<int> host_kind;     // phases timed on the host clock (phases-only mode)
    std::vector<double> host_ms;
    void reset() { used = 0; kind.clear(); work.clear(); host_kind.clear(); host_ms.clear(); }
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            pool.push_back(e);
        }
        return pool[used++];
    }
    // Event pair for one launch through hipExtLaunchKernelGGL, which stamps
    // the dispatch's own start and end (no extra packets on the stream).
    void pair(hipEvent_t* start, hipEvent_t* stop, int k, double w) {
        *start = next();
        *stop = next();
        kind.push_back(k);
        work.push_back(w);
    }
    // total milliseconds, launches and work of one kind (after a stream sync)
    void summary(int k, double* ms, long long* n, double* w) const {
        double t = 0, ww = 0;
        long long c = 0;
        for (size_t i = 0; i < kind.size(); i++) {
            if (kind[i] != k) continue;
            float e = 0;
            (void)hipEventElapsedTime(&e, pool[2 * i], pool[2 * i + 1]);
            t += e; ww += work[i]; c++;
        }
        for (size_t i = 0; i < host_kind.size(); i++) {
            if (host_kind[i] != k) continue;
            t += host_ms[i];
            c++;
        }
        *ms = t; *n = c; *w = ww;
    }
    ~LaunchProfiler() { for (auto e : pool) (void)hipEventDestroy(e); }
};

// Timing of a phase on a stream (no-op unless profiling is enabled).  With
// per-launch records on, an event pair brackets the phase.  Phases-only mode
// uses no timing events at all (a timing event switches the queue to
// timestamped dispatches, which slows every later launch): the stream is
// synchronised at both ends and the host clock taken.
struct PhaseTimer {
    LaunchProfiler* p;
    hipStream_t st;
    int k = 0;
    hipEvent_t e1 = nullptr;
    double t0 = -1.0;
    static double now_ms() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
    }
    PhaseTimer(LaunchProfiler* prof, hipStream_t s, int kind) : p(prof), st(s), k(kind) {
        if (!p || !p->enabled) return;
        if (p->launches) {
            hipEvent_t e0;
            p->pair(&e0, &e1, k, 0.0);
            (void)hipEventRecord(e0, st);
        } else {
            (void)hipStreamSynchronize(st);
            t0 = now_ms();
        }
    }
    void stop() {
        if (e1) (void)hipEventRecord(e1, st);
        e1 = nullptr;
        if (t0 >= 0.0) {
            (void)hipStreamSynchronize(st);
            p->host_kind.push_back(k);
            p->host_ms.push_back(now_ms() - t0);
            t0 = -1.0;
        }
    }
    ~PhaseTimer() { stop(); }
};

#define SYTRD_NBP 32       // Householder panel width
#define SYTRD_YCOPIES 4    // atomic accumulator copies (y, panel products; 8 -> 4 measured faster, 2 no better)
#define SYTRD_VCOPIES 256  // atomic accumulator copies (v^T A v)
#define SYTRD_SLOTS 3      // accumulator slots: column i accumulates into slot i % 3
#define ORMTR_NBB 64     // reflectors per compact-WY block in the back-transform
#define ORMTR_CHUNK 512  // rows per split-K chunk of V^T X

// --- Householder tridiagonalisation --------------------------------------
template <typename T>
struct SytrdWs {
    MatBatch<T> A;     // matrices, lower triangle used, overwritten by reflectors
    const int* ns;     // per-matrix order (device)
    int nmax, nbk_max;
    T* Vp; T* Wp; int ldp; long long sP;   // panels, column-major nmax x SYTRD_NBP
    T* colbuf; long long sC;               // updated current column, [2 slots] of sC (rows padded to 64 nbk_max)
    T* normacc;                            // ||col(i+2:n)||^2, [SYTRD_SLOTS] per matrix
    T* yacc; long long sY;                 // y = A v, [SYTRD_SLOTS][SYTRD_YCOPIES][nmax] per matrix
    T* sacc; long long sS;                 // W^T v, V^T v, [SYTRD_SLOTS][SYTRD_YCOPIES][2*NBP]
    T* vacc;                               // v^T A v, [SYTRD_SLOTS][SYTRD_VCOPIES] per matrix
    T* d; T* e; T* tau; long long sD;      // outputs
    int chunk_target;                      // SYMV workgroups per launch, trailing sizes in the upper quarter (tuned)
    int chunk_target_lo;                   // the same below it (tuned)
    int* order;                            // [nbatch] matrices by decreasing order (one-workgroup path)
};
template <typename T>
void sytrd_launch(const SytrdWs<T>& w, int nbatch, int nmax, hipStream_t st, const int* ns_host,
                  LaunchProfiler* prof);
// elements past a matrix's base that the split merges of divide and conquer
// touch in the gathered-operand buffers (host check of their sizes)
long long stedc_split_extent(int nmax, long long ld);

// --- Divide and conquer ------------------------------------------------------
template <typename T>
struct StedcWs {
    const int* ns;
    int nmax;
    const T* d_in; const T* e_in; long long sDin;
    // The rank-one-update algebra (poles, updating vector, secular roots,
    // Loewner vector, eigenvector formation) runs in FP64 for both T; only
    // the eigenvector matrices and their products are in T.
    double* D; double* E; long long sV;  // per-matrix vectors of length nmax (stride sV)
    double* scale;                       // [nbatch]
    MatBatch<T> Z0, Z1, U;               // eigenvector ping-pong and secular vector blocks
    double* ds; double* zs; double* dn; double* zn; double* mu; double* lam; double* zh; double* rho;
    double* rc; double* rs;
    int* perm; int* ndpos; int* dfpos; int* org; int* outnd; int* outdf; int* rp; int* rq;
    int* Kcnt; int* rotcnt;
    // support of each kept column of a merge (1: first half's rows, 2: second
    // half's, 3: both, after a rotation across the halves) and, per half, the
    // kept columns with support there (count at the merge origin)
    int* sup; int* ltop; int* lbot; int* ktop; int* kbot;
    int* ctop; int* cbot;  // the listed columns' positions in the merge's eigenvector block
    // FP32 merges of 2048 and more: their operands gathered per half (layout
    // of U, 64 elements of padding), or null
    T* GA0; T* GA1; T* GB0; T* GB1;
    T* w_out; long long sW;       // eigenvalues (ascending) out
};
// Returns 0 if the eigenvectors ended in Z0, 1 if in Z1.
template <typename T>
int stedc_launch(const StedcWs<T>& w, int nbatch, int nmax, hipStream_t st);

// Tridiagonals with a non-finite entry are replaced by zeros and flagged in
// bad[b] (1, else 0): the merges of divide and conquer rank each half's poles
// by binary search in the other, which assumes ordered values (a NaN makes
// two poles share a position and leaves another unset, whose stale index
// would then address the eigenvector blocks), and the multisection's
// brackets assume finite bounds.
template <typename T>
void tridiag_guard_launch(const int* ns, int nbatch, T* d, T* e, long long sD, int* bad, hipStream_t st);

// Eigenvalues only (Sturm counts with multisection, FP64 arithmetic): d, e of
// the reduction ([nbatch] x sD), w [nbatch] x sW ascending.  pairs: the
// matrices are real embeddings of Hermitian ones (every eigenvalue twice),
// and each pair is found once.
template <typename T>
void stebz_launch(const int* ns, int nmax, int nbatch, const T* d, const T* e, long long sD, T* w, long long sW,
                  hipStream_t st, bool pairs = false);

// --- Back-transformation ---------------------------------------------------
template <typename T>
struct OrmtrWs {
    MatBatch<T> A;     // reflectors (columns below the diagonal, implicit unit)
    const T* tau; long long sD;
    const int* ns;
    MatBatch<T> X;     // in: tridiagonal eigenvectors; out: eigenvectors of A
    T* Gpart; long long sG;   // [nblk][nsplit][64*64]
    T* Tm; long long sT;      // [nblk][64*64]
    T* VT; long long sVT;     // [nblk][64][nmax]: V T of each block, rows b0+1.. from 0
    T* Ypart; long long sYp;  // [nsplit][128*nmax]
    T* Y; long long sY;       // [128*nmax]: Y of a block, or Y_k over P_h of a pair
    T* Cp; long long sC;      // [nblk/2][64*64]: V_k^T VT_h per pair of blocks
    int nmax;
};
template <typename T>
void ormtr_launch(const OrmtrWs<T>& w, int nbatch, int nmax, hipStream_t st);

// --- generic batched GEMM (C = alpha op(A) op(B) + beta Cin, order ns[b]; Cin
// defaults to C) ---------------------------------------------------------------
// Output tile of the general batched GEMM (64 or 128), set per evaluation
// from the autotuner's table (thread-local: a context is driven by one
// thread at a time); 0 picks by order (128 from GEMM_TS128_MIN_ORDER).
extern thread_local int g_gemm_tile;
struct GemmTileScope {
    int saved;
    explicit GemmTileScope(int ts) : saved(g_gemm_tile) { g_gemm_tile = ts; }
    ~GemmTileScope() { g_gemm_tile = saved; }
};
template <typename T>
void gemm_batched(hipStream_t st, bool ta, bool tb, const int* ns, int nmax, int nbatch,
                  const T* A, int lda, long long sA, const T* B, int ldb, long long sB, T* C,
                  int ldc, long long sC, T alpha, T beta, bool lower_only, const int* skip = nullptr,
                  const T* Cin = nullptr, int ldcin = 0, long long sCin = 0);
// the second product of a pair launch: C2 = alpha op(A) op(B2) + beta C2
template <typename T>
struct GemmSecond {
    const T* B; int ldb; long long sB;
    T* C; int ldc; long long sC;
};
template <typename T>
void gemm_batched_pair(hipStream_t st, bool ta, bool tb, const int* ns, int nmax, int nbatch, const T* A, int lda,
                       long long sA, const T* B, int ldb, long long sB, T* C, int ldc, long long sC,
                       const GemmSecond<T>& second, T alpha, T beta, bool lower_only, const int* skip = nullptr);
