// Host runtime and C ABI of libmbd_hip.so (declared in include/mbd.h):
// context, device workspaces, validation, and the orchestration of the MBD
// stages on one stream.
#include "mbd.h"
#include "mbd_internal.h"
#include "mbd_kernels.h"
#include "mbd_sys.h"
#include "gemm_mfma.h"  // GEMM_TS128_MIN_ORDER (merge sizes that take the split product)

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

// Device scratch of mbd_evaluate_noalloc: every workspace of that entry point
// is carved from this array, so it calls no allocator.  Each device that runs
// the library holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress gives on that device.
static __device__ __align__(256) unsigned char scratch[MBD_NOALLOC_SCRATCH_BYTES];

// One row of the autotuner's table: SYMV work-item targets for trailing
// sizes in the upper quarter and below it, and the general GEMM's output
// tile (0: chosen by order).
struct TuneEntry {
    int hi = 1536, lo = 1536, gemm_ts = 0;
};

struct mbd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    mbd_precision prec = MBD_FP64;
    std::map<std::string, std::pair<void*, size_t>> bufs;
    size_t total = 0, limit = 0;
    int err_code = 0;
    std::string err_origin, err_msg;
    LaunchProfiler prof;
    double refine_tol = 0.0;  // second refinement step threshold (MBD_REFINE_TOL; <= 0: library default)
    bool refine_fallback = true;  // FP64 re-evaluation of unconverged systems (MBD_REFINE_FALLBACK=0: off)
    // autotuned SYMV work-item targets per matrix order, per precision (0 FP64, 1 FP32)
    std::map<int, TuneEntry> tune[2];  // order -> SYMV work-item targets, GEMM tile
    // captured batch launch sequences, keyed by batch signature
    struct Graph {
        hipGraphExec_t exec = nullptr;
        SysDesc* h_desc = nullptr;     // pinned staging of the system descriptors
        int* h_ns = nullptr;           // pinned matrix orders
        unsigned* h_status = nullptr;  // pinned status read-back
        int nsys = 0, nmat = 0;
        bool ok = false;
    };
    std::map<std::string, Graph> graphs;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // workspace arena (set only inside mbd_evaluate_noalloc): named workspaces
    // are bump-allocated from [arena, arena + arena_cap) instead of hipMalloc
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    std::map<std::string, std::pair<void*, size_t>> arena_bufs;
    void drop_graphs() {
        for (auto& kv : graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            (void)hipHostFree(kv.second.h_desc);
            (void)hipHostFree(kv.second.h_ns);
            (void)hipHostFree(kv.second.h_status);
        }
        graphs.clear();
    }
};

namespace {

// How run_core is being driven: eagerly (nullptr) or while capturing a graph,
// in which case uploads come from and the status goes to pinned buffers.
struct RunMode {
    bool capturing = false;
    mbd_ctx::Graph* g = nullptr;
};

mbd_status fail(mbd_ctx* c, mbd_status code, const char* origin, const std::string& msg) {
    if (c) {
        c->err_code = (int)code;
        c->err_origin = origin;
        c->err_msg = msg;
    }
    return code;
}

#define HIPCHK(expr, origin)                                                         \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) return fail(c, MBD_ERR_DEVICE, origin, hipGetErrorString(e_)); \
    } while (0)

// Named, growable device buffer.  Returns nullptr (and records the error) on
// allocation failure or when MBD_WORKSPACE_LIMIT would be exceeded.
void* ws(mbd_ctx* c, const char* name, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    if (c->arena) {
        // the same name returns the same memory within a call, as below
        auto at = c->arena_bufs.find(name);
        if (at != c->arena_bufs.end() && at->second.second >= bytes) return at->second.first;
        if (c->arena_used + bytes > c->arena_cap) {
            fail(c, MBD_ERR_OUT_OF_MEMORY, "workspace",
                 std::string("the no-allocation scratch is too small for ") + name);
            return nullptr;
        }
        void* p = c->arena + c->arena_used;
        c->arena_used += bytes;
        c->arena_bufs[name] = {p, bytes};
        return p;
    }
    auto it = c->bufs.find(name);
    if (it != c->bufs.end() && it->second.second >= bytes) return it->second.first;
    size_t old = it != c->bufs.end() ? it->second.second : 0;
    if (c->limit && c->total - old + bytes > c->limit) {
        fail(c, MBD_ERR_OUT_OF_MEMORY, "workspace", std::string("workspace limit exceeded for ") + name);
        return nullptr;
    }
    if (it != c->bufs.end()) {
        (void)hipStreamSynchronize(c->stream);
        if (c->gstream) (void)hipStreamSynchronize(c->gstream);
        c->drop_graphs();  // captured sequences hold the old address
        (void)hipFree(it->second.first);
        c->total -= old;
        c->bufs.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
        (void)hipGetLastError();
        fail(c, MBD_ERR_OUT_OF_MEMORY, "workspace", std::string("hipMalloc failed for ") + name);
        return nullptr;
    }
    c->bufs[name] = {p, bytes};
    c->total += bytes;
    return p;
}

template <typename T>
T* wsT(mbd_ctx* c, const std::string& name, size_t count) {
    return (T*)ws(c, name.c_str(), count * sizeof(T));
}

template <typename T> const char* tname();
template <> const char* tname<double>() { return "d"; }
template <> const char* tname<float>() { return "f"; }

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Table row for a matrix order: that of the tuned order nearest to n on a
// log scale; the defaults (1536 for both SYMV ranges, GEMM tile by order)
// when nothing is tuned.  The GEMM tile is taken only from a tuned order
// within a factor 2 of n.
TuneEntry tuned_entry(const mbd_ctx* c, int prec, int n) {
    const auto& t = c->tune[prec];
    TuneEntry best;
    double bd = 1e300;
    for (const auto& kv : t) {
        const double d = std::fabs(std::log((double)kv.first) - std::log((double)n));
        if (d < bd) { bd = d; best = kv.second; }
    }
    // a tile timed at an order more than a factor 2 away says little about
    // this one: leave the choice by order
    if (bd > std::log(2.0)) best.gemm_ts = 0;
    return best;
}

// Reduction workspace for a batch of nbatch matrices of order <= nmax.
template <typename T>
mbd_status make_sytrd_ws(mbd_ctx* c, MatBatch<T> A, const int* ns, int nmax, int nbatch, SytrdWs<T>& sw) {
    const std::string t = tname<T>();
    const int nbk = (nmax + 63) / 64;
    sw.A = A; sw.ns = ns; sw.nmax = nmax; sw.nbk_max = nbk;
    sw.ldp = round_up(nmax, 64);
    sw.sP = (long long)sw.ldp * SYTRD_NBP;
    sw.Vp = wsT<T>(c, "Vp" + t, sw.sP * nbatch);
    sw.Wp = wsT<T>(c, "Wp" + t, sw.sP * nbatch);
    // padded to whole 64-row blocks: the SYMV phase reads it in 16-byte segments
    sw.sC = round_up(nmax, 64); sw.colbuf = wsT<T>(c, "colbuf" + t, (size_t)2 * sw.sC * nbatch);
    sw.normacc = wsT<T>(c, "normacc" + t, (size_t)SYTRD_SLOTS * nbatch);
    sw.sY = (long long)SYTRD_SLOTS * SYTRD_YCOPIES * nmax; sw.yacc = wsT<T>(c, "yacc" + t, (size_t)sw.sY * nbatch);
    sw.sS = (long long)SYTRD_SLOTS * SYTRD_YCOPIES * 2 * SYTRD_NBP;
    sw.sacc = wsT<T>(c, "sacc" + t, (size_t)sw.sS * nbatch);
    sw.vacc = wsT<T>(c, "vacc" + t, (size_t)SYTRD_SLOTS * SYTRD_VCOPIES * nbatch);
    sw.sD = nmax;
    sw.d = wsT<T>(c, "d" + t, (size_t)nmax * nbatch);
    sw.e = wsT<T>(c, "e" + t, (size_t)nmax * nbatch);
    sw.tau = wsT<T>(c, "tau" + t, (size_t)nmax * nbatch);
    sw.order = wsT<int>(c, "sorder" + t, (size_t)nbatch);
    if (!sw.Vp || !sw.Wp || !sw.colbuf || !sw.normacc || !sw.yacc || !sw.sacc || !sw.vacc || !sw.d ||
        !sw.e || !sw.tau || !sw.order)
        return (mbd_status)c->err_code;
    return MBD_OK;
}

// Full dense symmetric eigensolver on a batch: reduction, D&C, back-transform.
template <typename T>
mbd_status run_eig(mbd_ctx* c, MatBatch<T> A, const int* ns, const int* ns_host, int nmax, int nbatch, bool vectors,
                   T* w_out, long long sW, MatBatch<T>* Xout, int** bad_out = nullptr, bool embed_pairs = false) {
    const std::string t = tname<T>();
    const hipStream_t st = c->stream;
    const int nbk = (nmax + 63) / 64;
    const int ldz = round_up(nmax, 64);
    const long long sZ = (long long)ldz * nmax;
    // --- reduction
    SytrdWs<T> sw;
    if (make_sytrd_ws<T>(c, A, ns, nmax, nbatch, sw) != MBD_OK) return (mbd_status)c->err_code;
    const TuneEntry te = tuned_entry(c, sizeof(T) == 8 ? 0 : 1, nmax);
    const std::pair<int, int> tg = {te.hi, te.lo};
    GemmTileScope tile_scope(te.gemm_ts);
    sw.chunk_target = tg.first;
    sw.chunk_target_lo = tg.second;
    {
        PhaseTimer ph(&c->prof, st, 3);
        sytrd_launch<T>(sw, nbatch, nmax, st, ns_host, &c->prof);
    }
    HIPCHK(hipGetLastError(), "sytrd");
    // a non-finite tridiagonal (from non-finite matrix entries) is zeroed and
    // flagged before the tridiagonal solvers see it
    int* bad = wsT<int>(c, "eig_bad", (size_t)nbatch);
    if (!bad) return (mbd_status)c->err_code;
    tridiag_guard_launch<T>(ns, nbatch, sw.d, sw.e, sw.sD, bad, st);
    if (bad_out) *bad_out = bad;
    if (!vectors) {
        // eigenvalues only: Sturm-count multisection on the tridiagonal
        PhaseTimer ph(&c->prof, st, 4);
        stebz_launch<T>(ns, nmax, nbatch, sw.d, sw.e, sw.sD, w_out, sW, st, embed_pairs);
        HIPCHK(hipGetLastError(), "stebz");
        if (Xout) *Xout = MatBatch<T>{nullptr, 0, 0};
        return MBD_OK;
    }

    // --- divide and conquer
    StedcWs<T> dw;
    dw.ns = ns; dw.nmax = nmax; dw.d_in = sw.d; dw.e_in = sw.e; dw.sDin = nmax;
    dw.sV = nmax;
    const size_t nv = (size_t)nmax * nbatch;
    double* tv[12];
    const char* tn[12] = {"D", "E", "ds", "zs", "dn", "zn", "mu", "lam", "zh", "rho", "rc", "rs"};
    for (int k = 0; k < 12; k++) {
        tv[k] = wsT<double>(c, std::string("dc_") + tn[k], nv);
        if (!tv[k]) return (mbd_status)c->err_code;
    }
    dw.D = tv[0]; dw.E = tv[1]; dw.ds = tv[2]; dw.zs = tv[3]; dw.dn = tv[4]; dw.zn = tv[5];
    dw.mu = tv[6]; dw.lam = tv[7]; dw.zh = tv[8]; dw.rho = tv[9]; dw.rc = tv[10]; dw.rs = tv[11];
    int* iv[17];
    const char* in[17] = {"perm", "ndpos", "dfpos", "org", "outnd", "outdf", "rp", "rq", "Kcnt", "rotcnt",
                          "sup", "ltop", "lbot", "ktop", "kbot", "ctop", "cbot"};
    for (int k = 0; k < 17; k++) {
        iv[k] = wsT<int>(c, std::string("dc_") + in[k], nv);
        if (!iv[k]) return (mbd_status)c->err_code;
    }
    dw.perm = iv[0]; dw.ndpos = iv[1]; dw.dfpos = iv[2]; dw.org = iv[3]; dw.outnd = iv[4]; dw.outdf = iv[5];
    dw.rp = iv[6]; dw.rq = iv[7]; dw.Kcnt = iv[8]; dw.rotcnt = iv[9];
    dw.sup = iv[10]; dw.ltop = iv[11]; dw.lbot = iv[12]; dw.ktop = iv[13]; dw.kbot = iv[14];
    dw.ctop = iv[15]; dw.cbot = iv[16];
    dw.scale = wsT<double>(c, "dc_scale", nbatch);
    dw.Z0 = {wsT<T>(c, "Z0" + t, (size_t)sZ * nbatch), ldz, sZ};
    dw.Z1 = {wsT<T>(c, "Z1" + t, (size_t)sZ * nbatch), ldz, sZ};
    dw.U = {wsT<T>(c, "U" + t, (size_t)sZ * nbatch), ldz, sZ};
    if (!dw.scale || !dw.Z0.p || !dw.Z1.p || !dw.U.p) return (mbd_status)c->err_code;
    dw.GA0 = dw.GA1 = dw.GB0 = dw.GB1 = nullptr;
    // FP32 merges of 2048 and more (which exist once the order exceeds half
    // of that) take the split product on gathered operands
    if (sizeof(T) == 4 && 2 * nmax > GEMM_TS128_MIN_ORDER) {
        if (stedc_split_extent(nmax, ldz) > sZ + 64)
            return fail(c, MBD_ERR_UNSUPPORTED, "eigensolver", "split-merge operands exceed their buffers");
        dw.GA0 = wsT<T>(c, "GA0" + t, (size_t)sZ * nbatch + 64);
        dw.GA1 = wsT<T>(c, "GA1" + t, (size_t)sZ * nbatch + 64);
        dw.GB0 = wsT<T>(c, "GB0" + t, (size_t)sZ * nbatch + 64);
        dw.GB1 = wsT<T>(c, "GB1" + t, (size_t)sZ * nbatch + 64);
        if (!dw.GA0 || !dw.GA1 || !dw.GB0 || !dw.GB1) return (mbd_status)c->err_code;
    }
    dw.w_out = w_out; dw.sW = sW;
    PhaseTimer ph_dc(&c->prof, st, 4);
    const int src = stedc_launch<T>(dw, nbatch, nmax, st);
    ph_dc.stop();
    HIPCHK(hipGetLastError(), "stedc");
    MatBatch<T> Z = src ? dw.Z1 : dw.Z0;

    {
        OrmtrWs<T> ow;
        const int nsplit = (nmax + ORMTR_CHUNK - 1) / ORMTR_CHUNK;
        ow.A = A; ow.tau = sw.tau; ow.sD = nmax; ow.ns = ns; ow.X = Z; ow.nmax = nmax;
        const int nblk = (nmax - 1 + 63) / 64;
        ow.sG = (long long)nblk * nsplit * 4096; ow.Gpart = wsT<T>(c, "Gpart" + t, ow.sG * nbatch);
        ow.sT = (long long)nblk * 4096; ow.Tm = wsT<T>(c, "Tm" + t, (size_t)ow.sT * nbatch);
        ow.sYp = (long long)nsplit * 128 * nmax; ow.Ypart = wsT<T>(c, "Ypart" + t, ow.sYp * nbatch);
        ow.sY = (long long)128 * nmax; ow.Y = wsT<T>(c, "Yb" + t, ow.sY * nbatch);
        ow.sC = (long long)(nblk / 2 + 1) * 4096; ow.Cp = wsT<T>(c, "Cpair" + t, (size_t)ow.sC * nbatch);
        ow.sVT = (long long)nblk * 64 * nmax; ow.VT = wsT<T>(c, "VT" + t, (size_t)ow.sVT * nbatch);
        if (!ow.Gpart || !ow.Tm || !ow.Ypart || !ow.Y || !ow.VT || !ow.Cp) return (mbd_status)c->err_code;
        PhaseTimer ph(&c->prof, st, 5);
        ormtr_launch<T>(ow, nbatch, nmax, st);
        HIPCHK(hipGetLastError(), "ormtr");
    }
    if (Xout) *Xout = Z;
    return MBD_OK;
}

bool finite_ok(double x) { return std::isfinite(x); }

// status word of a system -> its mbd_status
int status_code(unsigned st) {
    if (st & (MBD_ST_BAD_INPUT | MBD_ST_COINCIDENT)) return MBD_ERR_INVALID_ARGUMENT;
    if (st & MBD_ST_COLLAPSE) return MBD_ERR_NEGATIVE_EIGENVALUE;
    if (st & MBD_ST_NOT_CONVERGED) return MBD_ERR_NOT_CONVERGED;
    return MBD_OK;
}

// Validates the host-visible parts of a system.
mbd_status check_system(mbd_ctx* c, const mbd_system* s, unsigned want, const mbd_result* o, bool allow_periodic) {
    if (!s || !o) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "null system or result");
    if (s->n_atoms < 1) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "n_atoms must be >= 1");
    if (!s->coords || !s->alpha0 || !s->omega_or_c6 || !s->rvdw)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "null input array");
    if (!(s->beta >= 0.0) || !finite_ok(s->beta))
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "beta must be finite and >= 0");
    if (!(s->a > 0.0) || !finite_ok(s->a)) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "a must be > 0");
    if (s->param_kind != MBD_PARAM_OMEGA && s->param_kind != MBD_PARAM_C6)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "unknown param_kind");
    if (want & ~255u) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "unknown want bits");
    if ((want & MBD_WANT_ENERGY) && !o->energy) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "energy output is NULL");
    if ((want & MBD_WANT_GRAD_COORDS) && !o->grad_coords)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "grad_coords output is NULL");
    if ((want & MBD_WANT_GRAD_ALPHA0) && !o->grad_alpha0)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "grad_alpha0 output is NULL");
    if ((want & MBD_WANT_GRAD_OMEGA) && !o->grad_omega_or_c6)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "grad_omega_or_c6 output is NULL");
    if ((want & MBD_WANT_GRAD_RVDW) && !o->grad_rvdw)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "grad_rvdw output is NULL");
    if ((want & MBD_WANT_GRAD_LATTICE) && !o->grad_lattice)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "grad_lattice output is NULL");
    if ((want & MBD_WANT_EIGVALS) && !o->eigvals) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "eigvals output is NULL");
    if ((want & MBD_WANT_ERRORS) && !o->errors) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "errors output is NULL");
    if (s->lattice) {
        if (!allow_periodic) return fail(c, MBD_ERR_UNSUPPORTED, "mbd_evaluate_batch", "periodic systems are evaluated one at a time");
    } else if (want & MBD_WANT_GRAD_LATTICE) {
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "grad_lattice needs a lattice");
    }
    return MBD_OK;
}

SysDesc make_desc(const mbd_system* s, unsigned want, const mbd_result* o) {
    SysDesc d;
    std::memset(&d, 0, sizeof(d));
    d.coords = s->coords; d.alpha0 = s->alpha0; d.omega_or_c6 = s->omega_or_c6; d.rvdw = s->rvdw;
    d.N = s->n_atoms; d.param_kind = (int)s->param_kind; d.beta = s->beta; d.a = s->a;
    d.energy = (want & MBD_WANT_ENERGY) ? o->energy : nullptr;
    d.grad_coords = (want & MBD_WANT_GRAD_COORDS) ? o->grad_coords : nullptr;
    d.grad_alpha0 = (want & MBD_WANT_GRAD_ALPHA0) ? o->grad_alpha0 : nullptr;
    d.grad_omega = (want & MBD_WANT_GRAD_OMEGA) ? o->grad_omega_or_c6 : nullptr;
    d.grad_rvdw = (want & MBD_WANT_GRAD_RVDW) ? o->grad_rvdw : nullptr;
    d.grad_lattice = (want & MBD_WANT_GRAD_LATTICE) ? o->grad_lattice : nullptr;
    d.eigvals = (want & MBD_WANT_EIGVALS) ? o->eigvals : nullptr;
    d.errors = (want & MBD_WANT_ERRORS) ? o->errors : nullptr;
    return d;
}

// a matrix whose tridiagonal was not finite fails its system
__global__ void eig_bad_status_kernel(const int* bad, int nmat, unsigned* status, int one_system) {
    const int m = blockIdx.x * 64 + threadIdx.x;
    if (m < nmat && bad[m]) atomicOr(&status[one_system ? 0 : m], MBD_ST_BAD_INPUT);
}

__global__ void grad_gate_kernel(const unsigned* status, int nsys, SysDesc* sd) {
    // systems whose evaluation failed keep their gradient outputs untouched
    const int s = blockIdx.x * 64 + threadIdx.x;
    if (s >= nsys || status[s] == 0) return;
    sd[s].grad_coords = nullptr; sd[s].grad_alpha0 = nullptr; sd[s].grad_omega = nullptr;
    sd[s].grad_rvdw = nullptr; sd[s].grad_lattice = nullptr;
    sd[s].N = 0;
}

// Host-side description of a periodic evaluation: Cartesian q points, the
// integer image list of the real-space sum and the reciprocal-vector list.
struct PeriodicSetup {
    std::vector<double> qcart;
    std::vector<double> qmult;  // weight of each q point (2: it stands for its time-reversed partner too)
    std::vector<int> img, rec;
    int nq_all = 0;             // q points of the mesh before pairing
    std::vector<int> rcol;      // [nq][ncol]: reciprocal vectors of each q point's sphere, -1 padded
    int ncol = 0;
};

// Per q point, the reciprocal vectors G of the list with 0 < |G + q| < kc:
// the columns of its reciprocal-space basis.
static void recip_columns(const SysDesc& d, PeriodicSetup& ps) {
    const int nq = (int)ps.qcart.size() / 3, nr = (int)ps.rec.size() / 3;
    std::vector<std::vector<int>> lists(nq);
    size_t ncol = 0;
    for (int q = 0; q < nq; q++) {
        for (int t = 0; t < nr; t++) {
            double k[3];
            for (int c = 0; c < 3; c++)
                k[c] = ps.rec[3 * t] * d.recip[c] + ps.rec[3 * t + 1] * d.recip[3 + c] + ps.rec[3 * t + 2] * d.recip[6 + c] +
                       ps.qcart[3 * q + c];
            const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            if (k2 == 0.0 || k2 >= d.kc * d.kc) continue;
            lists[q].push_back(t);
        }
        ncol = std::max(ncol, lists[q].size());
    }
    ps.ncol = (int)ncol;
    ps.rcol.assign((size_t)nq * ncol, -1);
    for (int q = 0; q < nq; q++)
        std::copy(lists[q].begin(), lists[q].end(), ps.rcol.begin() + (size_t)q * ncol);
}

// Device column lists and basis workspaces of the reciprocal-space product
// (W, the adjoint's, only when gradients are wanted).
static mbd_status make_per_ewald(mbd_ctx* c, const PeriodicSetup& ps, int N, int nq, const int* rec_dev, bool with_w,
                                 PerEwald& pr) {
    pr.rec = rec_dev;
    pr.ncol = ps.ncol;
    pr.ldz = round_up(6 * N, 64);
    pr.sZ = (long long)pr.ldz * std::max(ps.ncol, 1);
    int* col = wsT<int>(c, "rcol", std::max<size_t>(1, ps.rcol.size()));
    pr.Z = wsT<double>(c, "rZ", (size_t)pr.sZ * nq);
    pr.W = with_w ? wsT<double>(c, "rW", (size_t)pr.sZ * nq) : nullptr;
    pr.phase = wsT<double>(c, "rphase", std::max<size_t>(2, ps.img.size() / 3 * 2 * (size_t)nq));
    if (!col || !pr.Z || (with_w && !pr.W) || !pr.phase) return (mbd_status)c->err_code;
    if (!ps.rcol.empty())
        HIPCHK(hipMemcpyAsync(col, ps.rcol.data(), sizeof(int) * ps.rcol.size(), hipMemcpyHostToDevice, c->stream),
               "upload");
    pr.col = col;
    return MBD_OK;
}

// Time reversal: Q(-q) is the complex conjugate of Q(q) (the lattice sums
// are real), and Q(q + G) the similarity D Q(q) D^* with the diagonal phases
// D = diag(exp(-i G.R_i)), whose derivative terms cancel in the gradient
// (D^* dD is imaginary and diagonal, Q^{1/2} Hermitian).  So a mesh point
// whose negative is also in the mesh, modulo the reciprocal lattice,
// contributes exactly what that partner does to the energy (eq:brillouin-int)
// and to every gradient (eq:mbd-gradient): one of each such pair is kept
// with weight 2.  Fractions as given; a pair must sum to an integer vector
// within 1e-10.
void pair_time_reversal(const std::vector<double>& qf, std::vector<double>& rep, std::vector<double>& mult) {
    const int nq = (int)qf.size() / 3;
    std::vector<char> used(nq, 0);
    rep.clear();
    mult.clear();
    for (int t = 0; t < nq; t++) {
        if (used[t]) continue;
        used[t] = 1;
        double m = 1.0;
        for (int u = t + 1; u < nq; u++) {
            if (used[u]) continue;
            bool match = true;
            for (int k = 0; k < 3; k++) {
                const double sum = qf[3 * t + k] + qf[3 * u + k];
                if (std::fabs(sum - std::nearbyint(sum)) > 1e-10) match = false;
            }
            if (match) {
                used[u] = 1;
                m = 2.0;
                break;
            }
        }
        for (int k = 0; k < 3; k++) rep.push_back(qf[3 * t + k]);
        mult.push_back(m);
    }
}

void inv3(const double* A, double* Ai) {
    const double dt = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                      A[2] * (A[3] * A[7] - A[4] * A[6]);
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / dt; Ai[1] = (A[2] * A[7] - A[1] * A[8]) / dt;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / dt; Ai[3] = (A[5] * A[6] - A[3] * A[8]) / dt;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / dt; Ai[5] = (A[2] * A[3] - A[0] * A[5]) / dt;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / dt; Ai[7] = (A[1] * A[6] - A[0] * A[7]) / dt;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / dt;
}

// Lattice, Ewald parameters (defaults of the paper's Sec. 3.3 when not
// given), q mesh and term lists.  Reads coords and R_vdW back to the host.
mbd_status setup_periodic(mbd_ctx* c, const mbd_system* s, SysDesc& d, PeriodicSetup& ps, bool pair_q = false) {
    const double* A = s->lattice;
    for (int k = 0; k < 9; k++) {
        if (!std::isfinite(A[k])) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "non-finite lattice");
        d.lat[k] = A[k];
    }
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0)) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "det(lattice) must be > 0");
    inv3(A, d.linv);
    const double twopi = 6.283185307179586476925;
    for (int u = 0; u < 3; u++)
        for (int k = 0; k < 3; k++) d.recip[u * 3 + k] = twopi * d.linv[k * 3 + u];
    d.vol = det;
    d.gamma = s->ewald_gamma > 0 ? s->ewald_gamma : 2.5 / std::cbrt(det);
    d.rc = s->ewald_rc > 0 ? s->ewald_rc : 6.0 / d.gamma;
    d.kc = s->ewald_kc > 0 ? s->ewald_kc : 10.0 * d.gamma;
    const int N = s->n_atoms;
    std::vector<double> R(3 * N), rv(N);
    // read on the context stream, so the values are those of the work queued before this call
    HIPCHK(hipMemcpyAsync(R.data(), s->coords, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c->stream), "read coords");
    HIPCHK(hipMemcpyAsync(rv.data(), s->rvdw, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream), "read rvdw");
    HIPCHK(hipStreamSynchronize(c->stream), "read coords");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, rvmax = 0.0;
    for (int i = 0; i < N; i++) {
        for (int k = 0; k < 3; k++) { lo[k] = std::min(lo[k], R[3 * i + k]); hi[k] = std::max(hi[k], R[3 * i + k]); }
        rvmax = std::max(rvmax, rv[i]);
    }
    if (!std::isfinite(rvmax)) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "non-finite rvdw");
    const double maxd = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));
    if (!std::isfinite(maxd)) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "non-finite coordinates");
    // (1 - g) > 1e-18  <=>  eta < 1 + ln(1e18 - 1)/a
    const double rdamp = s->beta > 0 ? (1.0 + std::log(1.0 / 1e-18 - 1.0) / s->a) * s->beta * 2.0 * rvmax * 1.0000001 : 0.0;
    d.rdamp = rdamp;
    const double rreal = std::max(d.rc, rdamp);
    // q mesh
    ps.qcart.clear();
    std::vector<double> qf;
    if (s->n_q > 0) {
        if (!s->q_frac) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "q_frac is NULL");
        qf.assign(s->q_frac, s->q_frac + 3 * s->n_q);
    } else {
        for (int k = 0; k < 3; k++)
            if (s->kgrid[k] < 1) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate", "kgrid must be >= 1");
        for (int a = 1; a <= s->kgrid[0]; a++)
            for (int b = 1; b <= s->kgrid[1]; b++)
                for (int e = 1; e <= s->kgrid[2]; e++) {
                    const int r3[3] = {a, b, e};
                    for (int k = 0; k < 3; k++)
                        qf.push_back((2.0 * r3[k] - s->kgrid[k] - 1) / (2.0 * s->kgrid[k]) + s->kshift[k]);
                }
    }
    ps.nq_all = (int)qf.size() / 3;
    // every q point is one matrix of a batch (grid z of the batched products)
    if (ps.nq_all > MBD_MAX_BATCH)
        return fail(c, MBD_ERR_UNSUPPORTED, "mbd_evaluate", "at most 65535 q points per evaluation");
    if (pair_q) {
        std::vector<double> rep;
        pair_time_reversal(qf, rep, ps.qmult);
        qf.swap(rep);
    } else {
        ps.qmult.assign(qf.size() / 3, 1.0);
    }
    double qmax = 0.0;
    for (size_t t = 0; t < qf.size() / 3; t++) {
        double q[3];
        for (int k = 0; k < 3; k++)
            q[k] = qf[3 * t] * d.recip[k] + qf[3 * t + 1] * d.recip[3 + k] + qf[3 * t + 2] * d.recip[6 + k];
        for (int k = 0; k < 3; k++) ps.qcart.push_back(q[k]);
        qmax = std::max(qmax, std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
    }
    // image and reciprocal lists (box bound, then sphere filter)
    ps.img.clear();
    ps.rec.clear();
    int nv[3], mv[3];
    for (int v = 0; v < 3; v++) {
        const double bl = std::sqrt(d.recip[3 * v] * d.recip[3 * v] + d.recip[3 * v + 1] * d.recip[3 * v + 1] +
                                    d.recip[3 * v + 2] * d.recip[3 * v + 2]);
        const double al = std::sqrt(A[3 * v] * A[3 * v] + A[3 * v + 1] * A[3 * v + 1] + A[3 * v + 2] * A[3 * v + 2]);
        nv[v] = (int)std::ceil((rreal + maxd) * bl / twopi) + 1;
        mv[v] = (int)std::ceil((d.kc + qmax) * al / twopi) + 1;
    }
    for (int x = -nv[0]; x <= nv[0]; x++)
        for (int y = -nv[1]; y <= nv[1]; y++)
            for (int z = -nv[2]; z <= nv[2]; z++) {
                double Rn[3];
                for (int k = 0; k < 3; k++) Rn[k] = x * A[k] + y * A[3 + k] + z * A[6 + k];
                if (std::sqrt(Rn[0] * Rn[0] + Rn[1] * Rn[1] + Rn[2] * Rn[2]) > rreal + maxd + 1e-9) continue;
                ps.img.push_back(x); ps.img.push_back(y); ps.img.push_back(z);
            }
    for (int x = -mv[0]; x <= mv[0]; x++)
        for (int y = -mv[1]; y <= mv[1]; y++)
            for (int z = -mv[2]; z <= mv[2]; z++) {
                double G[3];
                for (int k = 0; k < 3; k++) G[k] = x * d.recip[k] + y * d.recip[3 + k] + z * d.recip[6 + k];
                if (std::sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]) > d.kc + qmax + 1e-9) continue;
                ps.rec.push_back(x); ps.rec.push_back(y); ps.rec.push_back(z);
            }
    recip_columns(d, ps);
    return MBD_OK;
}

// One or more finite systems, or one periodic system (per != nullptr: one
// embedded matrix per q point), all stages on the context stream.
mbd_status run_core(mbd_ctx* c, std::vector<SysDesc>& sds, unsigned want, std::vector<int>& codes,
                    const PeriodicSetup* per, const RunMode* mode = nullptr) {
    const bool capturing = mode && mode->capturing;
    const hipStream_t st = c->stream;
    const int nsys = (int)sds.size();
    int Nmax = 0, ntot = 0;
    for (auto& d : sds) {
        d.atom_off = ntot;
        ntot += d.N;
        Nmax = std::max(Nmax, d.N);
    }
    const int nq = per ? (int)per->qcart.size() / 3 : 1;
    const int nmat = per ? nq : nsys;
    for (int s = 0; s < nsys; s++) {
        sds[s].mat0 = per ? 0 : s;
        sds[s].nmat = per ? nq : 1;
        sds[s].weight = per ? 0.25 / per->nq_all : 0.5;
        sds[s].embed = per ? 1 : 0;
    }
    const int nmax = per ? 6 * Nmax : 3 * Nmax;
    const int ld = round_up(nmax, 64);
    const long long stride = (long long)ld * nmax;
    const bool grads = (want & (MBD_WANT_GRAD_COORDS | MBD_WANT_GRAD_ALPHA0 | MBD_WANT_GRAD_OMEGA |
                                MBD_WANT_GRAD_RVDW | MBD_WANT_GRAD_LATTICE)) != 0;
    const bool fp32 = c->prec == MBD_FP32_REFINED;
    GemmTileScope tile_scope(tuned_entry(c, fp32 ? 1 : 0, nmax).gemm_ts);

    SysDesc* sd_dev = (SysDesc*)ws(c, "sysdesc", sizeof(SysDesc) * nsys);
    int* ns_dev = wsT<int>(c, "ns", nmat);
    unsigned* status = wsT<unsigned>(c, "status", nsys);
    double* lmin = wsT<double>(c, "lmin", nsys);
    double* om = wsT<double>(c, "om", ntot);
    double* cc = wsT<double>(c, "cc", ntot);
    double* lam = wsT<double>(c, "lam64", (size_t)nmax * nmat);
    double* sc = wsT<double>(c, "sc64", (size_t)nmax * nmat);
    MatBatch<double> A64 = {wsT<double>(c, "A64", (size_t)stride * nmat), ld, stride};
    MatBatch<float> A32 = {nullptr, ld, stride};
    if (fp32) A32.p = wsT<float>(c, "A32", (size_t)stride * nmat);
    if (!sd_dev || !ns_dev || !status || !lmin || !om || !cc || !lam || !sc || !A64.p || (fp32 && !A32.p))
        return (mbd_status)c->err_code;
    std::vector<int> nsh(nmat);
    for (int b = 0; b < nmat; b++) nsh[b] = per ? 6 * sds[0].N : 3 * sds[b].N;
    if (capturing) {
        HIPCHK(hipMemcpyAsync(sd_dev, mode->g->h_desc, sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(ns_dev, mode->g->h_ns, sizeof(int) * nmat, hipMemcpyHostToDevice, st), "upload");
    } else {
        HIPCHK(hipMemcpyAsync(sd_dev, sds.data(), sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(ns_dev, nsh.data(), sizeof(int) * nmat, hipMemcpyHostToDevice, st), "upload");
    }
    PhaseTimer ph_asm(&c->prof, st, 2);
    fill_u32_launch(st, status, nsys, 0u);
    mbd_prep_launch(st, sd_dev, nsys, Nmax, om, cc, status);
    double* qcart = nullptr;
    double* qmult = nullptr;
    int* img = nullptr;
    int* rec = nullptr;
    PerEwald prc = {};
    if (per) {
        qcart = wsT<double>(c, "qcart", per->qcart.size());
        qmult = wsT<double>(c, "qmult", (size_t)nq);
        img = wsT<int>(c, "img", per->img.size());
        rec = wsT<int>(c, "rec", per->rec.size());
        if (!qcart || !qmult || !img || !rec) return (mbd_status)c->err_code;
        HIPCHK(hipMemcpyAsync(qcart, per->qcart.data(), sizeof(double) * per->qcart.size(), hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(qmult, per->qmult.data(), sizeof(double) * nq, hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(img, per->img.data(), sizeof(int) * per->img.size(), hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(rec, per->rec.data(), sizeof(int) * per->rec.size(), hipMemcpyHostToDevice, st), "upload");
        const mbd_status rr = make_per_ewald(c, *per, sds[0].N, nq, rec, grads, prc);
        if (rr != MBD_OK) return rr;
        per_recip_basis_launch(st, sd_dev, qcart, nq, img, (int)per->img.size() / 3, prc);
        mbd_assemble_periodic_launch(st, sd_dev, om, cc, qcart, nq, img, (int)per->img.size() / 3, prc, A64, A32,
                                     status, sds[0].N);
    } else {
        mbd_assemble_finite_launch(st, sd_dev, nsys, Nmax, om, cc, A64, A32, status);
    }
    HIPCHK(hipGetLastError(), "assemble");
    ph_asm.stop();

    MatBatch<double> X;
    double* stats = nullptr;
    int* skip_dev = nullptr;  // per matrix: refinement step one was enough
    int* conv_dev = nullptr;  // per matrix: the last step met its target
    int* eig_bad = nullptr;  // per matrix: non-finite tridiagonal
    if (!fp32) {
        // periodic matrices are real embeddings: without vectors each
        // eigenvalue pair is found once
        mbd_status r = run_eig<double>(c, A64, ns_dev, nsh.data(), nmax, nmat, grads, lam, nmax, &X, &eig_bad,
                                       per != nullptr);
        if (r != MBD_OK) return r;
    } else {
        float* lam32 = wsT<float>(c, "lam32", (size_t)nmax * nmat);
        if (!lam32) return (mbd_status)c->err_code;
        MatBatch<float> X32;
        mbd_status r = run_eig<float>(c, A32, ns_dev, nsh.data(), nmax, nmat, true, lam32, nmax, &X32, &eig_bad);
        if (r != MBD_OK) return r;
        // refinement in FP64 against the FP64 Q held in A64: step one for
        // every matrix, step two where step one's remainder estimate is large
        MatBatch<double> Xd = {wsT<double>(c, "oaX", (size_t)stride * nmat), ld, stride};
        MatBatch<double> Y = {wsT<double>(c, "oaY", (size_t)stride * nmat), ld, stride};
        MatBatch<double> S = {wsT<double>(c, "oaS", (size_t)stride * nmat), ld, stride};
        MatBatch<double> G = {wsT<double>(c, "oaG", (size_t)stride * nmat), ld, stride};
        OaWork ow;
        ow.rho_next = c->refine_tol;
        ow.colpart = wsT<double>(c, "oacol", oa_colpart_doubles(nmax, nmat));
        ow.nclust = wsT<unsigned>(c, "oanclust", nmat);
        ow.wstart = wsT<int>(c, "oawstart", (size_t)nmax * nmat);
        ow.wlen = wsT<int>(c, "oawlen", (size_t)nmax * nmat);
        ow.wv = wsT<double>(c, "oawv", (size_t)OA_KMAX * nmax * nmat);
        ow.gdiag = wsT<double>(c, "oagdiag", (size_t)nmax * nmat);
        ow.fexp = wsT<int>(c, "oafexp", (size_t)nmax * nmat);
        stats = wsT<double>(c, "oastats", (size_t)8 * nmat);
        int* skip2 = wsT<int>(c, "oaskip2", nmat);
        int* skip3 = wsT<int>(c, "oaskip3", nmat);
        if (!Xd.p || !Y.p || !S.p || !G.p || !ow.colpart || !ow.nclust || !ow.wstart || !ow.wlen || !ow.wv || !ow.gdiag || !ow.fexp ||
            !stats || !skip2 || !skip3)
            return (mbd_status)c->err_code;
        PhaseTimer ph(&c->prof, st, 6);
        oa_f2d_launch(st, ns_dev, nmax, nmat, X32, Xd);
        oa_step_launch(st, ns_dev, nmax, nmat, A64, Xd, Y, S, G, lam, nmax, ow, stats, nullptr, skip2, X32);  // X1 in Y
        // the second step is accepted only far below the threshold
        OaWork ow2 = ow;
        ow2.rho_next = (ow.rho_next > 0.0 ? ow.rho_next : OA_RHO_NEXT) / OA_RHO_FINAL_DIV;
        oa_step_launch(st, ns_dev, nmax, nmat, A64, Y, S, Xd, G, lam, nmax, ow2, stats + 4 * nmat, skip2,
                       skip3, MatBatch<float>{nullptr, 0, 0});                                                                   // X2 in S
        skip_dev = skip2;
        conv_dev = skip3;
        HIPCHK(hipGetLastError(), "refine");
        X = S;
    }
    hipLaunchKernelGGL(eig_bad_status_kernel, dim3((nmat + 63) / 64), dim3(64), 0, st, eig_bad, nmat, status,
                       per ? 1 : 0);
    PhaseTimer ph_eg(&c->prof, st, 7);
    mbd_energy_launch(st, sd_dev, nsys, ns_dev, lam, nmax, om, status, lmin, conv_dev, per ? qmult : nullptr);
    mbd_errors_launch(st, sd_dev, nsys, nmat, stats, skip_dev);
    HIPCHK(hipGetLastError(), "energy");
    if (grads) {
        hipLaunchKernelGGL(grad_gate_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, status, nsys, sd_dev);
        mbd_invsqrt4_launch(st, ns_dev, nmax, nmat, lam, nmax, sc);
        MatBatch<double> M = A64;  // FP64: reflectors no longer needed; FP32: Q no longer needed
        mbd_inv_sqrt_launch(st, ns_dev, nmax, nmat, X, sc, nmax, M);
        mbd_mirror_launch(st, ns_dev, nmax, nmat, M);
        if (per) {
            const int N = sds[0].N;
            const int nch = per_recip_chunks(prc.ncol);
            double* part = wsT<double>(c, "gpart", (size_t)nq * N * N * PER_PART);
            double* rq = wsT<double>(c, "grq", std::max<size_t>(1, (size_t)nq * nch * N * 4));
            double* rl = wsT<double>(c, "grl", std::max<size_t>(1, (size_t)nq * nch * 10));
            double* latpart = wsT<double>(c, "glat", (size_t)N * 9);
            if (!part || !rq || !rl || !latpart) return (mbd_status)c->err_code;
            mbd_grad_periodic_launch(st, sd_dev, om, cc, qcart, qmult, 0.25 / per->nq_all, nq, img,
                                     (int)per->img.size() / 3, prc, M, part, rq, rl, latpart, N);
        } else {
            mbd_grad_finite_launch(st, sd_dev, nsys, Nmax, om, cc, M);
        }
        HIPCHK(hipGetLastError(), "gradients");
    }
    ph_eg.stop();
    if (capturing) {
        HIPCHK(hipMemcpyAsync(mode->g->h_status, status, sizeof(unsigned) * nsys, hipMemcpyDeviceToHost, st), "status");
        return MBD_OK;
    }
    std::vector<unsigned> sth(nsys);
    HIPCHK(hipMemcpyAsync(sth.data(), status, sizeof(unsigned) * nsys, hipMemcpyDeviceToHost, st), "status");
    HIPCHK(hipStreamSynchronize(st), "synchronize");
    codes.resize(nsys);
    for (int s = 0; s < nsys; s++) codes[s] = status_code(sth[s]);
    return MBD_OK;
}

mbd_status code_message(mbd_ctx* c, int code, const char* origin) {
    if (code == MBD_OK) return MBD_OK;
    if (code == MBD_ERR_INVALID_ARGUMENT)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, origin, "non-finite or non-positive per-atom input, or coincident atoms");
    if (code == MBD_ERR_NEGATIVE_EIGENVALUE)
        return fail(c, MBD_ERR_NEGATIVE_EIGENVALUE, origin, "Q has a non-positive eigenvalue (dipole collapse)");
    if (code == MBD_ERR_NOT_CONVERGED)
        return fail(c, MBD_ERR_NOT_CONVERGED, origin,
                    "FP64 refinement of the FP32 eigenpairs missed its target (FP64 fallback disabled)");
    return fail(c, (mbd_status)code, origin, "evaluation failed");
}

// Re-evaluates, on the FP64 path, the systems of a FP32+refine evaluation
// whose refinement did not converge (codes[s] == MBD_ERR_NOT_CONVERGED),
// unless the fallback is disabled.  Their errors[1..3] then read 0 (no
// refinement step).  per: the periodic setup of a single periodic system.
mbd_status refine_fallback(mbd_ctx* c, std::vector<SysDesc>& sds, unsigned want, std::vector<int>& codes,
                           const PeriodicSetup* per) {
    if (c->prec != MBD_FP32_REFINED || !c->refine_fallback) return MBD_OK;
    std::vector<SysDesc> redo;
    std::vector<int> idx;
    for (size_t s = 0; s < sds.size(); s++)
        if (codes[s] == MBD_ERR_NOT_CONVERGED) { redo.push_back(sds[s]); idx.push_back((int)s); }
    if (redo.empty()) return MBD_OK;
    std::vector<int> c2;
    c->prec = MBD_FP64;
    const mbd_status r = run_core(c, redo, want, c2, per);
    c->prec = MBD_FP32_REFINED;
    if (r != MBD_OK) return r;
    for (size_t k = 0; k < idx.size(); k++) codes[idx[k]] = c2[k];
    return MBD_OK;
}

// Per-device address of the scratch array, resolved once per device (with
// that device current) by the library's init call, mbd_create.
constexpr int MBD_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MBD_MAX_DEVICES] = {};
bool g_scratch_tried[MBD_MAX_DEVICES] = {};

void resolve_scratch(int device) {
    if (device < 0 || device >= MBD_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_tried[device]) return;
    g_scratch_tried[device] = true;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch_ptr[device] = p;
    else (void)hipGetLastError();
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= MBD_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

mbd_status mbd_create(mbd_ctx** ctx, int device, mbd_precision prec, void* hip_stream) {
    if (!ctx) return MBD_ERR_INVALID_ARGUMENT;
    *ctx = nullptr;
    if (prec != MBD_FP64 && prec != MBD_FP32_REFINED) return MBD_ERR_INVALID_ARGUMENT;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return MBD_ERR_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return MBD_ERR_DEVICE;
    resolve_scratch(device);
    mbd_ctx* c = new mbd_ctx();
    c->device = device;
    c->prec = prec;
    c->stream = (hipStream_t)hip_stream;
    const char* lim = std::getenv("MBD_WORKSPACE_LIMIT");
    if (lim) c->limit = (size_t)std::strtoull(lim, nullptr, 10);
    const char* rt = std::getenv("MBD_REFINE_TOL");
    if (rt) c->refine_tol = std::strtod(rt, nullptr);
    const char* fb = std::getenv("MBD_REFINE_FALLBACK");
    if (fb && fb[0] == '0') c->refine_fallback = false;
    *ctx = c;
    return MBD_OK;
}

mbd_status mbd_destroy(mbd_ctx* c) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->gstream) (void)hipStreamSynchronize(c->gstream);
    c->drop_graphs();
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    for (auto& kv : c->bufs) (void)hipFree(kv.second.first);
    delete c;
    return MBD_OK;
}

mbd_status mbd_set_stream(mbd_ctx* c, void* hip_stream) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    (void)hipStreamSynchronize(c->stream);
    c->stream = (hipStream_t)hip_stream;
    return MBD_OK;
}

mbd_status mbd_evaluate(mbd_ctx* c, const mbd_system* s, unsigned want, mbd_result* out) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    mbd_status r = check_system(c, s, want, out, true);
    if (r != MBD_OK) return r;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_evaluate", "hipSetDevice");
    std::vector<SysDesc> sds(1, make_desc(s, want, out));
    std::vector<int> codes;
    if (s->lattice) {
        PeriodicSetup ps;
        // time-reversed pairs evaluated once: on request (MBD_Q_PAIRS=1),
        // and never with eigenvalue output, which is per mesh point
        const char* qp = std::getenv("MBD_Q_PAIRS");
        const bool pair_q = qp && qp[0] == '1' && !(want & MBD_WANT_EIGVALS);
        r = setup_periodic(c, s, sds[0], ps, pair_q);
        if (r != MBD_OK) return r;
        r = run_core(c, sds, want, codes, &ps);
        if (r == MBD_OK) r = refine_fallback(c, sds, want, codes, &ps);
    } else {
        r = run_core(c, sds, want, codes, nullptr);
        if (r == MBD_OK) r = refine_fallback(c, sds, want, codes, nullptr);
    }
    if (r != MBD_OK) return r;
    return code_message(c, codes[0], "mbd_evaluate");
}

mbd_status mbd_evaluate_noalloc(mbd_ctx* c, const mbd_system* s, unsigned want, mbd_result* out) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    mbd_status r = check_system(c, s, want, out, true);
    if (r != MBD_OK) return r;
    if (s->lattice) return fail(c, MBD_ERR_UNSUPPORTED, "mbd_evaluate_noalloc", "finite systems only");
    if (s->n_atoms > MBD_NOALLOC_MAX_ATOMS)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate_noalloc",
                    "n_atoms exceeds MBD_NOALLOC_MAX_ATOMS (" + std::to_string(MBD_NOALLOC_MAX_ATOMS) + ")");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_evaluate_noalloc", "hipSetDevice");
    char* base = (char*)scratch_ptr(c->device);
    if (!base) return fail(c, MBD_ERR_DEVICE, "mbd_evaluate_noalloc", "scratch address not available on this device");
    // no launch timing here: its events would be created on demand
    const bool prof = c->prof.enabled;
    c->prof.enabled = false;
    c->arena = base;
    c->arena_cap = MBD_NOALLOC_SCRATCH_BYTES;
    c->arena_used = 0;
    c->arena_bufs.clear();
    std::vector<SysDesc> sds(1, make_desc(s, want, out));
    std::vector<int> codes;
    r = run_core(c, sds, want, codes, nullptr);
    if (r == MBD_OK) r = refine_fallback(c, sds, want, codes, nullptr);
    c->arena = nullptr;
    c->arena_cap = c->arena_used = 0;
    c->arena_bufs.clear();
    c->prof.enabled = prof;
    if (r != MBD_OK) return r;
    return code_message(c, codes[0], "mbd_evaluate_noalloc");
}

mbd_status mbd_ts_evaluate(mbd_ctx* c, const mbd_system* s, unsigned want, mbd_result* out) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    if (want & (MBD_WANT_GRAD_LATTICE | MBD_WANT_EIGVALS))
        return fail(c, MBD_ERR_UNSUPPORTED, "mbd_ts_evaluate", "grad_lattice and eigvals are not defined here");
    mbd_status r = check_system(c, s, want, out, true);
    if (r != MBD_OK) return r;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_ts_evaluate", "hipSetDevice");
    const hipStream_t st = c->stream;
    SysDesc d = make_desc(s, want, out);
    d.atom_off = 0;
    d.mat0 = 0;
    d.nmat = 0;
    PeriodicSetup ps;
    const bool periodic = s->lattice != nullptr;
    if (periodic) {
        // the pairwise lattice sum has no q mesh: one dummy point for the setup
        mbd_system sq = *s;
        const double q0[3] = {0.0, 0.0, 0.0};
        sq.n_q = 1;
        sq.q_frac = q0;
        r = setup_periodic(c, &sq, d, ps);
        if (r != MBD_OK) return r;
    }
    const int N = s->n_atoms;
    SysDesc* sd_dev = (SysDesc*)ws(c, "sysdesc", sizeof(SysDesc));
    unsigned* status = wsT<unsigned>(c, "status", 1);
    double* om = wsT<double>(c, "om", N);
    double* cc = wsT<double>(c, "cc", N);
    double* eatom = wsT<double>(c, "ts_eatom", N);
    int* img = wsT<int>(c, "img", std::max<size_t>(3, ps.img.size()));
    int* rec = wsT<int>(c, "rec", std::max<size_t>(3, ps.rec.size()));
    if (!sd_dev || !status || !om || !cc || !eatom || !img || !rec) return (mbd_status)c->err_code;
    HIPCHK(hipMemcpyAsync(sd_dev, &d, sizeof(SysDesc), hipMemcpyHostToDevice, st), "upload");
    if (periodic) {
        HIPCHK(hipMemcpyAsync(img, ps.img.data(), sizeof(int) * ps.img.size(), hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(rec, ps.rec.data(), sizeof(int) * ps.rec.size(), hipMemcpyHostToDevice, st), "upload");
    }
    fill_u32_launch(st, status, 1, 0u);
    mbd_prep_launch(st, sd_dev, 1, N, om, cc, status);
    mbd_ts_launch(st, sd_dev, N, om, img, (int)ps.img.size() / 3, rec, (int)ps.rec.size() / 3, periodic ? 1 : 0,
                  eatom, status, &c->prof);
    HIPCHK(hipGetLastError(), "ts");
    unsigned sth = 0;
    HIPCHK(hipMemcpyAsync(&sth, status, sizeof(unsigned), hipMemcpyDeviceToHost, st), "status");
    HIPCHK(hipStreamSynchronize(st), "synchronize");
    return code_message(c, status_code(sth), "mbd_ts_evaluate");
}

}  // extern "C"

namespace {

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n from the
// three-term recurrence, started at the asymptotic estimate of each root
void gauss_legendre_nodes(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < n; k++) {
        double t = std::cos(pi * (k + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = t;
            for (int m = 2; m <= n; m++) {
                const double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int m = 2; m <= n; m++) {
            const double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        dp = n == 1 ? 1.0 : n * (t * p1 - p0) / (t * t - 1.0);
        x[k] = t;
        w[k] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

}  // namespace

extern "C" {

mbd_status mbd_freq_evaluate(mbd_ctx* c, const mbd_system* s, int32_t n_freq, int32_t n_order, double* terms) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    if (n_freq < 1 || n_freq > 512 || n_order < 1 || n_order > 60 || !terms)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_freq_evaluate", "need 1 <= n_freq <= 512, 1 <= n_order <= 60, terms");
    mbd_result dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    mbd_status r = check_system(c, s, 0u, &dummy, true);
    if (r != MBD_OK) return r;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_freq_evaluate", "hipSetDevice");
    const hipStream_t st = c->stream;
    const int N = s->n_atoms;
    const bool periodic = s->lattice != nullptr;
    SysDesc base = make_desc(s, 0u, &dummy);
    PeriodicSetup ps;
    if (periodic) {
        r = setup_periodic(c, s, base, ps);
        if (r != MBD_OK) return r;
    }
    const int nq = periodic ? (int)ps.qcart.size() / 3 : 1;
    if ((long long)n_freq * nq > MBD_MAX_BATCH)
        return fail(c, MBD_ERR_UNSUPPORTED, "mbd_freq_evaluate", "at most 65535 matrices (frequencies x q points)");
    const int nmat = n_freq * nq;
    const int nmax = periodic ? 6 * N : 3 * N;
    const int ld = round_up(nmax, 64);
    const long long stride = (long long)ld * nmax;
    // the frequency grid: Gauss-Legendre on [-1, 1], u = 0.6 (1+x)/(1-x)
    std::vector<double> gx, gw, u(n_freq), wf(n_freq);
    gauss_legendre_nodes(n_freq, gx, gw);
    const double twopi = 6.283185307179586476925;
    for (int f = 0; f < n_freq; f++) {
        u[f] = 0.6 * (1.0 + gx[f]) / (1.0 - gx[f]);
        wf[f] = 1.2 / ((1.0 - gx[f]) * (1.0 - gx[f])) * gw[f] / twopi;
    }
    // descriptor 0: the system; descriptor f + 1: frequency f (its c, omega
    // entries at offset f N)
    std::vector<SysDesc> sds(n_freq + 1, base);
    for (int f = 0; f <= n_freq; f++) {
        sds[f].atom_off = f == 0 ? 0 : (f - 1) * N;
        sds[f].mat0 = f == 0 ? 0 : (f - 1) * nq;
        sds[f].nmat = nq;
        sds[f].embed = periodic ? 1 : 0;
    }
    std::vector<int> nsh(nmat, nmax);
    SysDesc* sd_dev = (SysDesc*)ws(c, "freq_desc", sizeof(SysDesc) * (n_freq + 1));
    int* ns_dev = wsT<int>(c, "freq_ns", nmat);
    unsigned* status = wsT<unsigned>(c, "freq_status", n_freq + 1);
    double* om0 = wsT<double>(c, "om", N);
    double* cc0 = wsT<double>(c, "cc", N);
    double* om_f = wsT<double>(c, "freq_om", (size_t)n_freq * N);
    double* cc_f = wsT<double>(c, "freq_cc", (size_t)n_freq * N);
    double* u_dev = wsT<double>(c, "freq_u", n_freq);
    double* wf_dev = wsT<double>(c, "freq_w", n_freq);
    double* lam = wsT<double>(c, "freq_lam", (size_t)nmax * nmat);
    double* part = wsT<double>(c, "freq_part", (size_t)nmat * (3 + n_order));
    MatBatch<double> K = {wsT<double>(c, "A64", (size_t)stride * nmat), ld, stride};
    if (!sd_dev || !ns_dev || !status || !om0 || !cc0 || !om_f || !cc_f || !u_dev || !wf_dev || !lam || !part || !K.p)
        return (mbd_status)c->err_code;
    HIPCHK(hipMemcpyAsync(sd_dev, sds.data(), sizeof(SysDesc) * (n_freq + 1), hipMemcpyHostToDevice, st), "upload");
    HIPCHK(hipMemcpyAsync(ns_dev, nsh.data(), sizeof(int) * nmat, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(hipMemcpyAsync(u_dev, u.data(), sizeof(double) * n_freq, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(hipMemcpyAsync(wf_dev, wf.data(), sizeof(double) * n_freq, hipMemcpyHostToDevice, st), "upload");
    fill_u32_launch(st, status, n_freq + 1, 0u);
    mbd_prep_launch(st, sd_dev, 1, N, om0, cc0, status);
    mbd_freq_coeff_launch(st, sd_dev, om0, u_dev, n_freq, N, om_f, cc_f);
    if (periodic) {
        int* img = wsT<int>(c, "img", ps.img.size());
        int* rec = wsT<int>(c, "rec", ps.rec.size());
        double* qcart = wsT<double>(c, "qcart", ps.qcart.size());
        if (!img || !rec || !qcart) return (mbd_status)c->err_code;
        HIPCHK(hipMemcpyAsync(qcart, ps.qcart.data(), sizeof(double) * ps.qcart.size(), hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(img, ps.img.data(), sizeof(int) * ps.img.size(), hipMemcpyHostToDevice, st), "upload");
        HIPCHK(hipMemcpyAsync(rec, ps.rec.data(), sizeof(int) * ps.rec.size(), hipMemcpyHostToDevice, st), "upload");
        PerEwald prc = {};
        r = make_per_ewald(c, ps, N, nq, rec, false, prc);
        if (r != MBD_OK) return r;
        // the lattice sums T(q) depend on the geometry only: assembled once,
        // then scaled by c_i c_j per frequency
        const MatBatch<double> Tq = {wsT<double>(c, "freq_T", (size_t)stride * nq), ld, stride};
        if (!Tq.p) return (mbd_status)c->err_code;
        per_recip_basis_launch(st, sd_dev + 1, qcart, nq, img, (int)ps.img.size() / 3, prc);
        mbd_assemble_periodic_launch(st, sd_dev + 1, nullptr, nullptr, qcart, nq, img, (int)ps.img.size() / 3, prc, Tq,
                                     MatBatch<float>{nullptr, ld, stride}, status + 1, N);
        mbd_freq_scale_launch(st, cc_f, N, n_freq, nq, Tq, K);
    } else {
        mbd_assemble_finite_launch(st, sd_dev + 1, n_freq, N, om_f, cc_f, K, MatBatch<float>{nullptr, ld, stride},
                                   status + 1);
    }
    HIPCHK(hipGetLastError(), "freq assemble");
    r = run_eig<double>(c, K, ns_dev, nsh.data(), nmax, nmat, false, lam, nmax, nullptr, nullptr, periodic);
    if (r != MBD_OK) return r;
    mbd_freq_terms_launch(st, ns_dev, nmat, lam, nmax, n_order, part, wf_dev, n_freq, nq, periodic ? 1 : 0, terms);
    HIPCHK(hipGetLastError(), "freq terms");
    std::vector<unsigned> sth(n_freq + 1);
    HIPCHK(hipMemcpyAsync(sth.data(), status, sizeof(unsigned) * (n_freq + 1), hipMemcpyDeviceToHost, st), "status");
    HIPCHK(hipStreamSynchronize(st), "synchronize");
    unsigned all = 0;
    for (unsigned v : sth) all |= v;
    return code_message(c, status_code(all & (MBD_ST_BAD_INPUT | MBD_ST_COINCIDENT)), "mbd_freq_evaluate");
}

mbd_status mbd_rsscs_evaluate(mbd_ctx* c, const mbd_system* s, int32_t n_freq, unsigned want, mbd_result* out,
                              double* scs_params) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    const unsigned allowed = MBD_WANT_ENERGY | MBD_WANT_GRAD_COORDS | MBD_WANT_EIGVALS | MBD_WANT_ERRORS;
    if (want & ~allowed)
        return fail(c, MBD_ERR_UNSUPPORTED, "mbd_rsscs_evaluate", "energy, dE/dR, eigenvalues and errors only");
    if (n_freq < 1 || n_freq > 512) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_rsscs_evaluate", "1 <= n_freq <= 512");
    mbd_status r = check_system(c, s, want, out, true);
    if (r != MBD_OK) return r;
    if (s->lattice) return fail(c, MBD_ERR_UNSUPPORTED, "mbd_rsscs_evaluate", "finite systems only");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_rsscs_evaluate", "hipSetDevice");
    const hipStream_t st = c->stream;
    const int N = s->n_atoms, n = 3 * N, nf = n_freq + 1;
    const int ld = round_up(n, 64);
    const long long stride = (long long)ld * n;
    mbd_result none;
    std::memset(&none, 0, sizeof(none));
    SysDesc base = make_desc(s, 0u, &none);
    // u = 0, then the Gauss-Legendre points; wq = (3/pi) du (Casimir-Polder)
    std::vector<double> gx, gw, u(nf, 0.0), wq(nf, 0.0);
    gauss_legendre_nodes(n_freq, gx, gw);
    const double pi = 3.14159265358979323846;
    for (int f = 1; f < nf; f++) {
        u[f] = 0.6 * (1.0 + gx[f - 1]) / (1.0 - gx[f - 1]);
        wq[f] = 3.0 / pi * 1.2 / ((1.0 - gx[f - 1]) * (1.0 - gx[f - 1])) * gw[f - 1];
    }
    SysDesc* sd_dev = (SysDesc*)ws(c, "scs_desc", sizeof(SysDesc));
    unsigned* status = wsT<unsigned>(c, "scs_status", 1);
    double* om0 = wsT<double>(c, "scs_om", N);
    double* cc0 = wsT<double>(c, "scs_cc", N);
    double* u_dev = wsT<double>(c, "scs_u", nf);
    double* wq_dev = wsT<double>(c, "scs_wq", nf);
    const long long sR = 3LL * n;  // three right-hand sides per matrix, row-major
    double* linv = wsT<double>(c, "scs_linv", (size_t)chol_linv_stride(n) * nf);
    double* rhs = wsT<double>(c, "scs_rhs", (size_t)sR * nf);
    double* ytmp = wsT<double>(c, "scs_y", (size_t)sR * nf);
    double* V = wsT<double>(c, "scs_v", (size_t)sR * nf);
    double* abar = wsT<double>(c, "scs_abar", (size_t)nf * N);
    double* par = wsT<double>(c, "scs_par", (size_t)4 * N);
    MatBatch<double> A = {wsT<double>(c, "scsA", (size_t)stride * nf), ld, stride};
    if (!sd_dev || !status || !om0 || !cc0 || !u_dev || !wq_dev || !linv || !rhs || !ytmp || !V || !abar || !par ||
        !A.p)
        return (mbd_status)c->err_code;
    HIPCHK(hipMemcpyAsync(sd_dev, &base, sizeof(SysDesc), hipMemcpyHostToDevice, st), "upload");
    HIPCHK(hipMemcpyAsync(u_dev, u.data(), sizeof(double) * nf, hipMemcpyHostToDevice, st), "upload");
    HIPCHK(hipMemcpyAsync(wq_dev, wq.data(), sizeof(double) * nf, hipMemcpyHostToDevice, st), "upload");
    fill_u32_launch(st, status, 1, 0u);
    mbd_prep_launch(st, sd_dev, 1, N, om0, cc0, status);
    // screening: A(u) for all u in one batch, its Cholesky factors, and
    // V = A(u)^-1 (1 (x) I_3) from them
    {
        PhaseTimer ph(&c->prof, st, 9);
        scs_assemble_launch(st, sd_dev, N, om0, u_dev, nf, A, status);
        chol_factor_launch(st, A, n, nf, linv, status);
        scs_rhs_launch(st, N, nf, nullptr, rhs);
        chol_solve_launch(st, A, n, nf, linv, rhs, ytmp, V, sR);
        scs_contract_launch(st, N, nf, V, abar);
        scs_params_launch(st, sd_dev, N, abar, wq_dev, nf, par);
    }
    if (scs_params) HIPCHK(hipMemcpyAsync(scs_params, par, sizeof(double) * 4 * N, hipMemcpyDeviceToDevice, st), "copy");
    HIPCHK(hipGetLastError(), "scs");
    unsigned sth = 0;
    HIPCHK(hipMemcpyAsync(&sth, status, sizeof(unsigned), hipMemcpyDeviceToHost, st), "status");
    HIPCHK(hipStreamSynchronize(st), "synchronize");
    if (sth & (MBD_ST_BAD_INPUT | MBD_ST_COINCIDENT)) return code_message(c, MBD_ERR_INVALID_ARGUMENT, "mbd_rsscs_evaluate");
    if (sth & MBD_ST_COLLAPSE)
        return fail(c, MBD_ERR_NEGATIVE_EIGENVALUE, "mbd_rsscs_evaluate",
                    "alpha(iu)^-1 + T^scs is not positive definite (the screening collapses)");
    // MBD with the screened alpha0, omega and R_vdW
    mbd_system ss = *s;
    ss.alpha0 = par;
    ss.omega_or_c6 = par + 2 * N;
    ss.param_kind = MBD_PARAM_OMEGA;
    ss.rvdw = par + 3 * N;
    const bool grads = (want & MBD_WANT_GRAD_COORDS) != 0;
    mbd_result rs = *out;
    unsigned w2 = want;
    double* gpar = nullptr;
    if (grads) {
        gpar = wsT<double>(c, "scs_gpar", (size_t)3 * N);
        if (!gpar) return (mbd_status)c->err_code;
        rs.grad_alpha0 = gpar;
        rs.grad_omega_or_c6 = gpar + N;
        rs.grad_rvdw = gpar + 2 * N;
        w2 |= MBD_WANT_GRAD_ALPHA0 | MBD_WANT_GRAD_OMEGA | MBD_WANT_GRAD_RVDW;
    }
    std::vector<SysDesc> sds(1, make_desc(&ss, w2, &rs));
    std::vector<int> codes;
    r = run_core(c, sds, w2, codes, nullptr);
    if (r == MBD_OK) r = refine_fallback(c, sds, w2, codes, nullptr);
    if (r != MBD_OK) return r;
    if (codes[0] != MBD_OK) return code_message(c, codes[0], "mbd_rsscs_evaluate");
    if (grads) {
        // chain rule through the screened parameters
        // U^T = A(u)^-1 (w (x) I_3) with the gradient weights w_i(u)
        double* w = wsT<double>(c, "scs_w", (size_t)nf * N);
        double* U = wsT<double>(c, "scs_u3", (size_t)sR * nf);
        double* UV = wsT<double>(c, "scs_uv", (size_t)nf * n * 6);
        if (!w || !U || !UV) return (mbd_status)c->err_code;
        PhaseTimer ph(&c->prof, st, 9);
        scs_weights_launch(st, N, nf, par, abar, wq_dev, gpar, gpar + N, gpar + 2 * N, w);
        scs_rhs_launch(st, N, nf, w, rhs);
        chol_solve_launch(st, A, n, nf, linv, rhs, ytmp, U, sR);
        scs_grad_launch(st, sd_dev, N, nf, om0, u_dev, U, V, UV, out->grad_coords);
        HIPCHK(hipGetLastError(), "scs gradient");
        HIPCHK(hipStreamSynchronize(st), "synchronize");
    }
    return MBD_OK;
}

mbd_status mbd_evaluate_batch(mbd_ctx* c, int32_t n_sys, const mbd_system* sys, unsigned want, mbd_result* out,
                              int32_t* status) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    if (n_sys < 1 || !sys || !out || !status)
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_evaluate_batch", "bad batch arguments");
    if (n_sys > MBD_MAX_BATCH)
        return fail(c, MBD_ERR_UNSUPPORTED, "mbd_evaluate_batch", "at most 65535 systems per batch");
    std::vector<SysDesc> sds(n_sys);
    std::string sig = std::to_string((int)c->prec) + ":" + std::to_string(want) + ":";
    for (int i = 0; i < n_sys; i++) {
        mbd_status r = check_system(c, &sys[i], want, &out[i], false);
        if (r != MBD_OK) return r;
        sds[i] = make_desc(&sys[i], want, &out[i]);
        sig += std::to_string(sys[i].n_atoms) + ",";
    }
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_evaluate_batch", "hipSetDevice");
    std::vector<int> codes(n_sys, MBD_OK);
    const char* nograph = std::getenv("MBD_NO_GRAPH");
    const bool use_graph = !(nograph && nograph[0] == '1') && !c->prof.enabled;
    auto it = use_graph ? c->graphs.find(sig) : c->graphs.end();
    if (it != c->graphs.end() && it->second.ok) {
        // replay: refresh the pinned descriptors, run after the caller's stream
        mbd_ctx::Graph& g = it->second;
        int Nt = 0;
        for (int i = 0; i < n_sys; i++) {
            sds[i].atom_off = Nt; Nt += sds[i].N;
            sds[i].mat0 = i; sds[i].nmat = 1; sds[i].weight = 0.5; sds[i].embed = 0;
        }
        HIPCHK(hipStreamSynchronize(c->gstream), "graph");
        std::memcpy(g.h_desc, sds.data(), sizeof(SysDesc) * n_sys);
        HIPCHK(hipEventRecord(c->ev_in, c->stream), "graph");
        HIPCHK(hipStreamWaitEvent(c->gstream, c->ev_in, 0), "graph");
        HIPCHK(hipGraphLaunch(g.exec, c->gstream), "graph launch");
        HIPCHK(hipEventRecord(c->ev_out, c->gstream), "graph");
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_out, 0), "graph");
        HIPCHK(hipStreamSynchronize(c->gstream), "graph");
        for (int i = 0; i < n_sys; i++) codes[i] = status_code(g.h_status[i]);
    } else {
        mbd_status r = run_core(c, sds, want, codes, nullptr);
        if (r != MBD_OK) return r;
        if (use_graph && it == c->graphs.end()) {
            // capture the same launch sequence once for later calls of this signature
            if (!c->gstream) {
                if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
                    hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
                    return fail(c, MBD_ERR_DEVICE, "mbd_evaluate_batch", "stream creation");
            }
            mbd_ctx::Graph g;
            g.nsys = n_sys;
            g.nmat = n_sys;
            bool ok = hipHostMalloc((void**)&g.h_desc, sizeof(SysDesc) * n_sys, 0) == hipSuccess &&
                      hipHostMalloc((void**)&g.h_ns, sizeof(int) * n_sys, 0) == hipSuccess &&
                      hipHostMalloc((void**)&g.h_status, sizeof(unsigned) * n_sys, 0) == hipSuccess;
            if (ok) {
                std::memcpy(g.h_desc, sds.data(), sizeof(SysDesc) * n_sys);
                for (int i = 0; i < n_sys; i++) g.h_ns[i] = 3 * sds[i].N;
                RunMode m;
                m.capturing = true;
                m.g = &g;
                hipStream_t user = c->stream;
                c->stream = c->gstream;
                hipGraph_t graph = nullptr;
                std::vector<int> dummy;
                ok = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    const mbd_status rc = run_core(c, sds, want, dummy, nullptr, &m);
                    const bool end_ok = hipStreamEndCapture(c->gstream, &graph) == hipSuccess;
                    ok = rc == MBD_OK && end_ok && graph &&
                         hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) == hipSuccess;
                    if (graph) (void)hipGraphDestroy(graph);
                }
                c->stream = user;
                (void)hipGetLastError();
            }
            g.ok = ok && g.exec;
            c->graphs[sig] = g;  // a failed capture is remembered: that signature stays eager
        }
    }
    {
        const mbd_status r = refine_fallback(c, sds, want, codes, nullptr);
        if (r != MBD_OK) return r;
    }
    mbd_status first = MBD_OK;
    for (int i = 0; i < n_sys; i++) {
        status[i] = codes[i];
        if (codes[i] != MBD_OK && first == MBD_OK) first = (mbd_status)codes[i];
    }
    if (first != MBD_OK) return code_message(c, first, "mbd_evaluate_batch");
    return MBD_OK;
}

mbd_status mbd_eigh(mbd_ctx* c, int32_t dtype, int32_t n, int32_t nbatch, void* A, int32_t lda, int64_t stride,
                    void* w, void* Z, int32_t ldz, int64_t zstride) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    if (n < 1 || nbatch < 1 || !A || !w || lda < n || stride < (int64_t)lda * n || (dtype != 0 && dtype != 1) ||
        (Z && (ldz < n || zstride < (int64_t)ldz * n)))
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_eigh", "bad sizes or pointers");
    if (nbatch > MBD_MAX_BATCH) return fail(c, MBD_ERR_UNSUPPORTED, "mbd_eigh", "at most 65535 matrices per call");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_eigh", "hipSetDevice");
    std::vector<int> nsh(nbatch, n);
    int* ns_dev = wsT<int>(c, "eigh_ns", nbatch);
    if (!ns_dev) return (mbd_status)c->err_code;
    HIPCHK(hipMemcpyAsync(ns_dev, nsh.data(), sizeof(int) * nbatch, hipMemcpyHostToDevice, c->stream), "upload");
    mbd_status r;
    int* bad = nullptr;
    // the reduction reads the matrices in 16-byte segments of 64-row-aligned
    // columns: stage them into a workspace with a leading dimension that is a
    // multiple of 64 (the caller's A is left unchanged)
    const int lds = round_up(n, 64);
    const long long sts = (long long)lds * n;
    const size_t es = dtype == 0 ? sizeof(double) : sizeof(float);
    void* As = dtype == 0 ? (void*)wsT<double>(c, "eighA", (size_t)sts * nbatch) : (void*)wsT<float>(c, "eighA32", (size_t)sts * nbatch);
    if (!As) return (mbd_status)c->err_code;
    for (int b = 0; b < nbatch; b++)
        HIPCHK(hipMemcpy2DAsync((char*)As + (size_t)b * sts * es, es * lds, (const char*)A + (size_t)b * stride * es,
                                es * lda, es * n, n, hipMemcpyDeviceToDevice, c->stream),
               "stage");
    if (dtype == 0) {
        MatBatch<double> Ab = {(double*)As, lds, sts}, X;
        r = run_eig<double>(c, Ab, ns_dev, nsh.data(), n, nbatch, Z != nullptr, (double*)w, n, &X, &bad);
        if (r == MBD_OK && Z)
            HIPCHK(hipMemcpy2DAsync(Z, sizeof(double) * ldz, X.p, sizeof(double) * X.ld, sizeof(double) * n,
                                    (size_t)n * 1, hipMemcpyDeviceToDevice, c->stream), "copy");
        if (r == MBD_OK && Z && nbatch > 1)
            for (int b = 1; b < nbatch; b++)
                HIPCHK(hipMemcpy2DAsync((double*)Z + (long long)b * zstride, sizeof(double) * ldz, X.p + (long long)b * X.stride,
                                        sizeof(double) * X.ld, sizeof(double) * n, n, hipMemcpyDeviceToDevice, c->stream),
                       "copy");
    } else {
        MatBatch<float> Ab = {(float*)As, lds, sts}, X;
        r = run_eig<float>(c, Ab, ns_dev, nsh.data(), n, nbatch, Z != nullptr, (float*)w, n, &X, &bad);
        if (r == MBD_OK && Z)
            for (int b = 0; b < nbatch; b++)
                HIPCHK(hipMemcpy2DAsync((float*)Z + (long long)b * zstride, sizeof(float) * ldz, X.p + (long long)b * X.stride,
                                        sizeof(float) * X.ld, sizeof(float) * n, n, hipMemcpyDeviceToDevice, c->stream),
                       "copy");
    }
    if (r != MBD_OK) return r;
    std::vector<int> badh(nbatch);
    HIPCHK(hipMemcpyAsync(badh.data(), bad, sizeof(int) * nbatch, hipMemcpyDeviceToHost, c->stream), "read flags");
    HIPCHK(hipStreamSynchronize(c->stream), "mbd_eigh");
    for (int b = 0; b < nbatch; b++)
        if (badh[b]) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_eigh", "non-finite matrix entries");
    return MBD_OK;
}

}  // extern "C"

namespace {

template <typename T>
mbd_status autotune_size(mbd_ctx* c, int n, int* best_target, int* best_lo, double* best_ms) {
    const int ld = round_up(n, 64);
    const long long stride = (long long)ld * n;
    T* A = wsT<T>(c, std::string("tuneA") + tname<T>(), stride);
    T* B = wsT<T>(c, std::string("tuneB") + tname<T>(), stride);
    int* ns_dev = wsT<int>(c, "tune_ns", 1);
    if (!A || !B || !ns_dev) return (mbd_status)c->err_code;
    HIPCHK(hipMemcpyAsync(ns_dev, &n, sizeof(int), hipMemcpyHostToDevice, c->stream), "upload");
    fill_sym_random_launch<T>(c->stream, n, B, ld, 12345u);
    SytrdWs<T> sw;
    MatBatch<T> Ab = {A, ld, stride};
    if (make_sytrd_ws<T>(c, Ab, ns_dev, n, 1, sw) != MBD_OK) return (mbd_status)c->err_code;
    const int cand[] = {256, 512, 768, 1024, 1536, 2048, 3072, 4096};
    int nh = n;
    // Each candidate runs the reduction with a start/stop event pair on every
    // SYMV launch; the kernel times are summed separately over the upper
    // quarter of trailing sizes and below it (the two tuned ranges), and each
    // range keeps its fastest candidate.  Kernel time, not the wall time of
    // an eager reduction, whose host launch rate can hide the differences.
    LaunchProfiler prof;
    prof.enabled = true;
    const int nbk = (n + 63) / 64;
    double best_up = 1e300, best_low = 1e300;
    *best_target = *best_lo = 1536;
    for (int target : cand) {
        double up = 1e300, low = 1e300;
        for (int rep = 0; rep < 2; rep++) {
            HIPCHK(hipMemcpyAsync(A, B, sizeof(T) * stride, hipMemcpyDeviceToDevice, c->stream), "copy");
            sw.chunk_target = target;
            sw.chunk_target_lo = target;
            prof.reset();
            sytrd_launch<T>(sw, 1, n, c->stream, &nh, &prof);
            HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
            double u = 0, l = 0;
            int col = 0;
            for (size_t q = 0; q < prof.kind.size(); q++) {
                if (prof.kind[q] != 0 && prof.kind[q] != 8) continue;  // per-column launches, in order
                float ms = 0;
                (void)hipEventElapsedTime(&ms, prof.pool[2 * q], prof.pool[2 * q + 1]);
                const int nbt = nbk - ((col + 1) >> 6);
                (4 * nbt >= 3 * nbk ? u : l) += ms;
                col++;
            }
            up = std::min(up, u);
            low = std::min(low, l);
        }
        if (up < best_up) { best_up = up; *best_target = target; }
        if (low < best_low) { best_low = low; *best_lo = target; }
    }
    *best_ms = best_up + best_low;
    return MBD_OK;
}

// General-GEMM output tile for order n: C = A B (FP64, n x n x n, the shape
// of the refinement's and the gradients' products) timed with 64 x 64 and
// 128 x 128 tiles, the faster kept.
mbd_status autotune_gemm_tile(mbd_ctx* c, int n, int* ts_out) {
    const int ld = round_up(n, 64);
    const long long stride = (long long)ld * n;
    double* A = wsT<double>(c, "tuneGA", stride);
    double* B = wsT<double>(c, "tuneGB", stride);
    double* C = wsT<double>(c, "tuneGC", stride);
    if (!A || !B || !C) return (mbd_status)c->err_code;
    fill_sym_random_launch<double>(c->stream, n, A, ld, 4321u);
    fill_sym_random_launch<double>(c->stream, n, B, ld, 8765u);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0), "event");
    HIPCHK(hipEventCreate(&e1), "event");
    double best = 1e300;
    *ts_out = 0;
    for (int ts : {64, 128}) {
        GemmTileScope scope(ts);
        float t = 1e30f;
        for (int rep = 0; rep < 3; rep++) {
            (void)hipEventRecord(e0, c->stream);
            gemm_batched<double>(c->stream, false, false, nullptr, n, 1, A, ld, stride, B, ld, stride, C, ld, stride,
                                 1.0, 0.0, false, nullptr);
            (void)hipEventRecord(e1, c->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) t = std::min(t, ms);  // the first launch of a shape is left out
        }
        if (t < best) { best = t; *ts_out = ts; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError(), "autotune gemm");
    return MBD_OK;
}

// Captured batch sequences replay the launch shapes they were recorded with;
// a changed tuning table retires them (after the work queued on both streams)
void drop_graphs_synced(mbd_ctx* c) {
    (void)hipStreamSynchronize(c->stream);
    if (c->gstream) (void)hipStreamSynchronize(c->gstream);
    c->drop_graphs();
}

bool write_tuning(const mbd_ctx* c, const char* path) {
    FILE* f = std::fopen(path, "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    const char* names[2] = {"fp64", "fp32"};
    for (int p = 0; p < 2; p++) {
        std::fprintf(f, "  \"%s\": {", names[p]);
        bool first = true;
        for (const auto& kv : c->tune[p]) {
            std::fprintf(f, "%s\"%d\": [%d, %d, %d]", first ? "" : ", ", kv.first, kv.second.hi, kv.second.lo,
                         kv.second.gemm_ts);
            first = false;
        }
        std::fprintf(f, "}%s\n", p == 0 ? "," : "");
    }
    std::fprintf(f, "}\n");
    return std::fclose(f) == 0;
}

// parses {"fp64": {"n": [upper, lower, gemm_tile], ...}, "fp32": {...}} (the
// format written above); a single number sets both targets, a missing
// (or 0) GEMM tile leaves the choice by order
bool read_tuning(mbd_ctx* c, const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, k);
    std::fclose(f);
    const char* names[2] = {"\"fp64\"", "\"fp32\""};
    for (int p = 0; p < 2; p++) {
        const size_t at = txt.find(names[p]);
        if (at == std::string::npos) continue;
        const size_t lb = txt.find('{', at), rb = txt.find('}', at);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) return false;
        const std::string body = txt.substr(lb + 1, rb - lb - 1);
        size_t pos = 0;
        std::map<int, TuneEntry> tab;
        while ((pos = body.find('"', pos)) != std::string::npos) {
            const size_t q2 = body.find('"', pos + 1);
            const size_t colon = body.find(':', q2);
            if (q2 == std::string::npos || colon == std::string::npos) return false;
            const int key = std::atoi(body.substr(pos + 1, q2 - pos - 1).c_str());
            size_t v = body.find_first_not_of(" \t\n", colon + 1);
            if (v == std::string::npos) return false;
            int hi, lo, ts = 0;
            if (body[v] == '[') {
                const size_t comma = body.find(',', v), rbk = body.find(']', v);
                if (comma == std::string::npos || rbk == std::string::npos || comma > rbk) return false;
                hi = std::atoi(body.c_str() + v + 1);
                lo = std::atoi(body.c_str() + comma + 1);
                const size_t comma2 = body.find(',', comma + 1);
                if (comma2 != std::string::npos && comma2 < rbk) ts = std::atoi(body.c_str() + comma2 + 1);
                pos = body.find(',', rbk);
            } else {
                hi = lo = std::atoi(body.c_str() + v);
                pos = body.find(',', v);
            }
            if (key <= 0 || hi <= 0 || lo <= 0 || (ts != 0 && ts != 64 && ts != 128)) return false;
            TuneEntry e;
            e.hi = hi; e.lo = lo; e.gemm_ts = ts;
            tab[key] = e;
            if (pos == std::string::npos) break;
        }
        c->tune[p] = tab;
    }
    return true;
}

}  // namespace

extern "C" {

mbd_status mbd_autotune(mbd_ctx* c, const int32_t* sizes, int32_t nsizes, const char* path) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    if (!sizes || nsizes < 1) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_autotune", "no sizes");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_autotune", "hipSetDevice");
    const int p = c->prec == MBD_FP32_REFINED ? 1 : 0;
    for (int k = 0; k < nsizes; k++) {
        const int n = sizes[k];
        if (n < 2) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_autotune", "sizes must be >= 2");
        int target = 1536, lo = 1536, ts = 0;
        double ms = 0;
        mbd_status r = p ? autotune_size<float>(c, n, &target, &lo, &ms) : autotune_size<double>(c, n, &target, &lo, &ms);
        if (r != MBD_OK) return r;
        r = autotune_gemm_tile(c, n, &ts);
        if (r != MBD_OK) return r;
        TuneEntry e;
        e.hi = target; e.lo = lo; e.gemm_ts = ts;
        c->tune[p][n] = e;
    }
    drop_graphs_synced(c);  // captured batches were recorded with the old launch shapes
    if (path && !write_tuning(c, path)) return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_autotune", "cannot write table");
    return MBD_OK;
}

mbd_status mbd_load_tuning(mbd_ctx* c, const char* path) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    c->err_code = 0;
    if (!path || !read_tuning(c, path))
        return fail(c, MBD_ERR_INVALID_ARGUMENT, "mbd_load_tuning", "cannot read tuning table");
    drop_graphs_synced(c);  // captured batches were recorded with the old launch shapes
    return MBD_OK;
}

mbd_status mbd_check_dc_buffers(int32_t n_max, int64_t* needed, int64_t* allocated) {
    if (n_max < 1 || !needed || !allocated) return MBD_ERR_INVALID_ARGUMENT;
    const long long ldz = round_up(n_max, 64);
    *allocated = ldz * n_max + 64;
    *needed = 2 * n_max > GEMM_TS128_MIN_ORDER ? stedc_split_extent(n_max, ldz) : 0;
    return *needed <= *allocated ? MBD_OK : MBD_ERR_UNSUPPORTED;
}

mbd_status mbd_set_profiling(mbd_ctx* c, int enable) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    (void)hipStreamSynchronize(c->stream);
    c->prof.enabled = enable != 0;
    c->prof.launches = enable != 2;
    c->prof.reset();
    return MBD_OK;
}

mbd_status mbd_get_profile(mbd_ctx* c, int32_t kind, double* total_ms, int64_t* launches, double* work) {
    if (!c || !total_ms || !launches || !work || kind < 0 || kind >= PROF_KINDS) return MBD_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, MBD_ERR_DEVICE, "mbd_get_profile", "synchronize");
    long long n = 0;
    c->prof.summary(kind, total_ms, &n, work);
    *launches = n;
    return MBD_OK;
}

int mbd_last_error(const mbd_ctx* c, const char** origin, const char** message) {
    if (!c) return MBD_ERR_INVALID_ARGUMENT;
    if (origin) *origin = c->err_origin.c_str();
    if (message) *message = c->err_msg.c_str();
    return c->err_code;
}

}  // extern "C"
