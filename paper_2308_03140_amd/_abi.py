"""ctypes declarations of the C ABI in include/mbd.h (argument marshalling only)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libmbd_hip.so")

MBD_OK = 0
MBD_ERR_INVALID_ARGUMENT = 1
MBD_ERR_NEGATIVE_EIGENVALUE = 2
MBD_ERR_NOT_CONVERGED = 3
MBD_ERR_OUT_OF_MEMORY = 4
MBD_ERR_DEVICE = 5
MBD_ERR_UNSUPPORTED = 6

MBD_FP64 = 0
MBD_FP32_REFINED = 1
MBD_PARAM_OMEGA = 0
MBD_PARAM_C6 = 1

MBD_WANT_ENERGY = 1
MBD_WANT_GRAD_COORDS = 2
MBD_WANT_GRAD_ALPHA0 = 4
MBD_WANT_GRAD_OMEGA = 8
MBD_WANT_GRAD_RVDW = 16
MBD_WANT_GRAD_LATTICE = 32
MBD_WANT_EIGVALS = 64
MBD_WANT_ERRORS = 128

MBD_NOALLOC_MAX_ATOMS = 256
MBD_NOALLOC_SCRATCH_BYTES = 128 << 20

_P = ctypes.c_void_p


class MbdSystem(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32),
        ("coords", _P),
        ("lattice", _P),
        ("n_q", ctypes.c_int32),
        ("q_frac", _P),
        ("kgrid", ctypes.c_int32 * 3),
        ("kshift", ctypes.c_double * 3),
        ("alpha0", _P),
        ("omega_or_c6", _P),
        ("param_kind", ctypes.c_int),
        ("rvdw", _P),
        ("beta", ctypes.c_double),
        ("a", ctypes.c_double),
        ("ewald_gamma", ctypes.c_double),
        ("ewald_rc", ctypes.c_double),
        ("ewald_kc", ctypes.c_double),
    ]


class MbdResult(ctypes.Structure):
    _fields_ = [
        ("energy", _P),
        ("grad_coords", _P),
        ("grad_alpha0", _P),
        ("grad_omega_or_c6", _P),
        ("grad_rvdw", _P),
        ("grad_lattice", _P),
        ("eigvals", _P),
        ("errors", _P),
    ]


_lib = None


def lib():
    """Load libmbd_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError("libmbd_hip.so not built: run `python -m paper_2308_03140_amd.build` "
                               "(or __graft_entry__.build())")
        L = ctypes.CDLL(library_path)
        L.mbd_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int, _P]
        L.mbd_destroy.argtypes = [_P]
        L.mbd_set_stream.argtypes = [_P, _P]
        L.mbd_evaluate.argtypes = [_P, ctypes.POINTER(MbdSystem), ctypes.c_uint, ctypes.POINTER(MbdResult)]
        L.mbd_evaluate_noalloc.argtypes = [_P, ctypes.POINTER(MbdSystem), ctypes.c_uint, ctypes.POINTER(MbdResult)]
        L.mbd_ts_evaluate.argtypes = [_P, ctypes.POINTER(MbdSystem), ctypes.c_uint, ctypes.POINTER(MbdResult)]
        L.mbd_freq_evaluate.argtypes = [_P, ctypes.POINTER(MbdSystem), ctypes.c_int32, ctypes.c_int32, _P]
        L.mbd_rsscs_evaluate.argtypes = [_P, ctypes.POINTER(MbdSystem), ctypes.c_int32, ctypes.c_uint,
                                         ctypes.POINTER(MbdResult), _P]
        L.mbd_evaluate_batch.argtypes = [_P, ctypes.c_int32, ctypes.POINTER(MbdSystem), ctypes.c_uint,
                                         ctypes.POINTER(MbdResult), ctypes.POINTER(ctypes.c_int32)]
        L.mbd_eigh.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                               ctypes.c_int64, _P, _P, ctypes.c_int32, ctypes.c_int64]
        L.mbd_autotune.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_char_p]
        L.mbd_load_tuning.argtypes = [_P, ctypes.c_char_p]
        L.mbd_set_profiling.argtypes = [_P, ctypes.c_int]
        L.mbd_get_profile.argtypes = [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
        L.mbd_last_error.argtypes = [_P, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_char_p)]
        L.mbd_check_dc_buffers.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64)]
        for f in ("mbd_create", "mbd_destroy", "mbd_set_stream", "mbd_evaluate", "mbd_evaluate_noalloc", "mbd_ts_evaluate",
                  "mbd_freq_evaluate", "mbd_rsscs_evaluate",
                  "mbd_evaluate_batch",
                  "mbd_eigh", "mbd_autotune", "mbd_load_tuning", "mbd_last_error", "mbd_set_profiling",
                  "mbd_get_profile", "mbd_check_dc_buffers"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def mbd_create(device=0, precision=MBD_FP64, stream=None):
    """Returns (status, ctx handle)."""
    h = _P()
    st = lib().mbd_create(ctypes.byref(h), int(device), int(precision), _P(stream) if stream else None)
    return st, h


def mbd_destroy(ctx):
    return lib().mbd_destroy(ctx)


def mbd_set_stream(ctx, stream):
    return lib().mbd_set_stream(ctx, _P(stream) if stream else None)


def mbd_evaluate(ctx, system, want, result):
    return lib().mbd_evaluate(ctx, ctypes.byref(system), ctypes.c_uint(want), ctypes.byref(result))


def mbd_evaluate_noalloc(ctx, system, want, result):
    return lib().mbd_evaluate_noalloc(ctx, ctypes.byref(system), ctypes.c_uint(want), ctypes.byref(result))


def mbd_ts_evaluate(ctx, system, want, result):
    return lib().mbd_ts_evaluate(ctx, ctypes.byref(system), ctypes.c_uint(want), ctypes.byref(result))


def mbd_freq_evaluate(ctx, system, n_freq, n_order, terms):
    return lib().mbd_freq_evaluate(ctx, ctypes.byref(system), int(n_freq), int(n_order), _P(terms))


def mbd_rsscs_evaluate(ctx, system, n_freq, want, result, scs_params):
    return lib().mbd_rsscs_evaluate(ctx, ctypes.byref(system), int(n_freq), ctypes.c_uint(want),
                                    ctypes.byref(result), _P(scs_params) if scs_params else None)


def mbd_evaluate_batch(ctx, systems, want, results, status):
    """systems/results: ctypes arrays of MbdSystem/MbdResult; status: ctypes int32 array."""
    return lib().mbd_evaluate_batch(ctx, len(systems), systems, ctypes.c_uint(want), results, status)


def mbd_eigh(ctx, dtype, n, nbatch, A, lda, stride, w, Z, ldz, zstride):
    return lib().mbd_eigh(ctx, dtype, n, nbatch, _P(A), lda, stride, _P(w), _P(Z) if Z else None, ldz, zstride)


def mbd_autotune(ctx, sizes, path=None):
    arr = (ctypes.c_int32 * len(sizes))(*sizes)
    return lib().mbd_autotune(ctx, arr, len(sizes), path.encode() if path else None)


def mbd_load_tuning(ctx, path):
    return lib().mbd_load_tuning(ctx, path.encode())


def mbd_set_profiling(ctx, enable):
    """enable: 0 off, 1 launch and phase events, 2 phases only (host clock)."""
    return lib().mbd_set_profiling(ctx, int(enable))


def mbd_get_profile(ctx, kind):
    """Returns (status, total_ms, launches, work) for one profiling kind: 0 SYMV
    launches, 1 SYR2K launches, 2..7 the evaluation phases, 8 fused per-column
    launches, 9 the screening stage of MBD@rsSCS, 10 the one-workgroup-per-matrix
    reduction of a batch, 11 the pairwise (TS) kernel (see include/mbd.h)."""
    ms = ctypes.c_double(); n = ctypes.c_int64(); w = ctypes.c_double()
    st = lib().mbd_get_profile(ctx, int(kind), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(w))
    return st, ms.value, n.value, w.value


def mbd_check_dc_buffers(n_max):
    """(status, needed, allocated): host-only check of the divide-and-conquer
    gather buffers for matrices of order <= n_max."""
    need = ctypes.c_int64(); have = ctypes.c_int64()
    st = lib().mbd_check_dc_buffers(int(n_max), ctypes.byref(need), ctypes.byref(have))
    return st, need.value, have.value


def mbd_last_error(ctx):
    """Returns (code, origin, message)."""
    o = ctypes.c_char_p()
    m = ctypes.c_char_p()
    code = lib().mbd_last_error(ctx, ctypes.byref(o), ctypes.byref(m))
    return code, (o.value or b"").decode(), (m.value or b"").decode()
