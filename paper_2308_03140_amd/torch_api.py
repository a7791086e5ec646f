"""PyTorch-facing helpers over the C ABI: torch device tensors in, torch
tensors out.  Only argument marshalling happens here; device memory comes from
torch's allocator and work is enqueued on torch's current stream."""
import ctypes

import torch

from . import _abi as A


class MBDError(RuntimeError):
    def __init__(self, code, origin, message):
        super().__init__("MBD error %d in %s: %s" % (code, origin, message))
        self.code = code
        self.origin = origin
        self.message = message


class CollapseError(MBDError):
    """Q is not positive definite (dipole collapse)."""


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _raise(ctx, code):
    c, o, m = A.mbd_last_error(ctx.handle)
    cls = CollapseError if code == A.MBD_ERR_NEGATIVE_EIGENVALUE else MBDError
    raise cls(code, o, m)


class Context:
    """Owns an mbd_ctx bound to a device, a precision and torch's current stream."""

    def __init__(self, device=0, precision="fp64"):
        prec = {"fp64": A.MBD_FP64, "fp32_refined": A.MBD_FP32_REFINED}[precision]
        self.device = torch.device("cuda", device)
        self.precision = precision
        stream = torch.cuda.current_stream(self.device).cuda_stream
        st, h = A.mbd_create(device, prec, stream)
        if st != A.MBD_OK:
            raise MBDError(st, "mbd_create", "could not create context")
        self.handle = h
        self._stream = stream

    def sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            A.mbd_set_stream(self.handle, s)
            self._stream = s

    def autotune(self, sizes, path=None):
        """Time the reduction's launch-shape candidates for these matrix orders
        (mbd_autotune) and keep the fastest in this context."""
        self.sync_stream()
        code = A.mbd_autotune(self.handle, [int(x) for x in sizes], path)
        if code != A.MBD_OK:
            _raise(self, code)

    def load_tuning(self, path):
        code = A.mbd_load_tuning(self.handle, path)
        if code != A.MBD_OK:
            _raise(self, code)

    def close(self):
        if self.handle:
            A.mbd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev(x, device):
    if isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.device == device and x.is_contiguous():
        return x
    return torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()


def make_system(coords, alpha0, omega, rvdw, beta=0.83, a=6.0, lattice=None, q_frac=None,
                kgrid=None, kshift=(0.0, 0.0, 0.0), param="omega", ewald=(0.0, 0.0, 0.0), device=None):
    """Builds (MbdSystem, keep-alive list).  coords/alpha0/omega/rvdw: device tensors
    (or array-likes copied to `device`); lattice and q_frac stay on the host."""
    keep = []
    dev = device if device is not None else coords.device
    c = _dev(coords, dev)
    if c.dim() != 2 or c.shape[1] != 3:
        c = c.reshape(-1, 3)
    a0 = _dev(alpha0, dev); w = _dev(omega, dev); rv = _dev(rvdw, dev)
    keep += [c, a0, w, rv]
    s = A.MbdSystem()
    s.n_atoms = c.shape[0]
    s.coords = c.data_ptr(); s.alpha0 = a0.data_ptr(); s.omega_or_c6 = w.data_ptr(); s.rvdw = rv.data_ptr()
    s.param_kind = A.MBD_PARAM_C6 if param == "c6" else A.MBD_PARAM_OMEGA
    s.beta = float(beta); s.a = float(a)
    if lattice is not None:
        s.ewald_gamma, s.ewald_rc, s.ewald_kc = [float(x) for x in ewald]
    if lattice is not None:
        lat = (ctypes.c_double * 9)(*[float(x) for x in torch.as_tensor(lattice, dtype=torch.float64).reshape(-1).tolist()])
        keep.append(lat)
        s.lattice = ctypes.addressof(lat)
        if q_frac is not None:
            qf = torch.as_tensor(q_frac, dtype=torch.float64).reshape(-1).tolist()
            qarr = (ctypes.c_double * len(qf))(*qf)
            keep.append(qarr)
            s.q_frac = ctypes.addressof(qarr)
            s.n_q = len(qf) // 3
        else:
            s.n_q = 0
            for i in range(3):
                s.kgrid[i] = int(kgrid[i]) if kgrid is not None else 1
                s.kshift[i] = float(kshift[i])
    return s, keep


def evaluate(ctx, coords, alpha0, omega, rvdw, beta=0.83, a=6.0, lattice=None, q_frac=None,
             kgrid=None, kshift=(0.0, 0.0, 0.0), param="omega", gradients=True, eigvals=False, errors=True,
             ewald=(0.0, 0.0, 0.0), noalloc=False):
    """Energy (and gradients) of one system.  Returns a dict of torch tensors.
    Periodic systems take either q_frac or the Monkhorst-Pack mesh kgrid
    (+ kshift) built by the library.  noalloc=True calls
    mbd_evaluate_noalloc (finite systems of at most MBD_NOALLOC_MAX_ATOMS;
    the outputs are still allocated here, by torch)."""
    ctx.sync_stream()
    dev = ctx.device
    s, keep = make_system(coords, alpha0, omega, rvdw, beta, a, lattice, q_frac, kgrid, kshift,
                          param=param, ewald=ewald, device=dev)
    N = s.n_atoms
    periodic = lattice is not None
    nq = s.n_q if (periodic and s.n_q) else (int(torch.tensor(kgrid).prod()) if periodic else 1)
    out = {"energy": torch.empty(1, dtype=torch.float64, device=dev)}
    want = A.MBD_WANT_ENERGY
    r = A.MbdResult()
    r.energy = out["energy"].data_ptr()
    if gradients:
        out["grad_coords"] = torch.empty(N, 3, dtype=torch.float64, device=dev)
        out["grad_alpha0"] = torch.empty(N, dtype=torch.float64, device=dev)
        r.grad_coords = out["grad_coords"].data_ptr()
        r.grad_alpha0 = out["grad_alpha0"].data_ptr()
        want |= A.MBD_WANT_GRAD_COORDS | A.MBD_WANT_GRAD_ALPHA0
        if periodic:
            out["grad_lattice"] = torch.empty(3, 3, dtype=torch.float64, device=dev)
            r.grad_lattice = out["grad_lattice"].data_ptr()
            want |= A.MBD_WANT_GRAD_LATTICE
        out["grad_omega"] = torch.empty(N, dtype=torch.float64, device=dev)
        out["grad_rvdw"] = torch.empty(N, dtype=torch.float64, device=dev)
        r.grad_omega_or_c6 = out["grad_omega"].data_ptr()
        r.grad_rvdw = out["grad_rvdw"].data_ptr()
        want |= A.MBD_WANT_GRAD_OMEGA | A.MBD_WANT_GRAD_RVDW
    if eigvals:
        out["eigvals"] = torch.empty(nq, 3 * N, dtype=torch.float64, device=dev)
        r.eigvals = out["eigvals"].data_ptr()
        want |= A.MBD_WANT_EIGVALS
    if errors:
        out["errors"] = torch.zeros(4, dtype=torch.float64, device=dev)
        r.errors = out["errors"].data_ptr()
        want |= A.MBD_WANT_ERRORS
    code = (A.mbd_evaluate_noalloc if noalloc else A.mbd_evaluate)(ctx.handle, s, want, r)
    if code != A.MBD_OK:
        _raise(ctx, code)
    return out


def ts_evaluate(ctx, coords, alpha0, omega, rvdw, sR, a=20.0, lattice=None, param="omega", gradients=True,
                ewald=(0.0, 0.0, 0.0)):
    """Pairwise (TS) dispersion energy (and gradients) of one finite or
    periodic system (mbd_ts_evaluate): s_R and the damping steepness a
    (TS: 20) take the places of beta and a of the MBD damping."""
    ctx.sync_stream()
    dev = ctx.device
    s, keep = make_system(coords, alpha0, omega, rvdw, sR, a, lattice, [[0.0, 0.0, 0.0]] if lattice is not None
                          else None, param=param, ewald=ewald, device=dev)
    N = s.n_atoms
    out = {"energy": torch.empty(1, dtype=torch.float64, device=dev)}
    r = A.MbdResult()
    r.energy = out["energy"].data_ptr()
    want = A.MBD_WANT_ENERGY
    if gradients:
        for name, field, shape, bit in (("grad_coords", "grad_coords", (N, 3), A.MBD_WANT_GRAD_COORDS),
                                        ("grad_alpha0", "grad_alpha0", (N,), A.MBD_WANT_GRAD_ALPHA0),
                                        ("grad_omega", "grad_omega_or_c6", (N,), A.MBD_WANT_GRAD_OMEGA),
                                        ("grad_rvdw", "grad_rvdw", (N,), A.MBD_WANT_GRAD_RVDW)):
            out[name] = torch.empty(*shape, dtype=torch.float64, device=dev)
            setattr(r, field, out[name].data_ptr())
            want |= bit
    code = A.mbd_ts_evaluate(ctx.handle, s, want, r)
    if code != A.MBD_OK:
        _raise(ctx, code)
    return out


def freq_evaluate(ctx, coords, alpha0, omega, rvdw, beta=0.83, a=6.0, lattice=None, q_frac=None, kgrid=None,
                  kshift=(0.0, 0.0, 0.0), n_freq=15, n_order=6, param="omega", ewald=(0.0, 0.0, 0.0)):
    """Frequency-route energies (mbd_freq_evaluate): returns a dict with the
    log-formula energy, the renormalised energy, min(1 + x_k) and the
    many-body orders E^(1..n_order) (a tensor)."""
    ctx.sync_stream()
    dev = ctx.device
    s, keep = make_system(coords, alpha0, omega, rvdw, beta, a, lattice, q_frac, kgrid, kshift, param=param,
                          ewald=ewald, device=dev)
    t = torch.empty(3 + n_order, dtype=torch.float64, device=dev)
    code = A.mbd_freq_evaluate(ctx.handle, s, n_freq, n_order, t.data_ptr())
    if code != A.MBD_OK:
        _raise(ctx, code)
    return {"energy": t[0], "energy_gould": t[1], "min_one_plus_x": t[2], "orders": t[3:]}


def rsscs_evaluate(ctx, coords, alpha0, omega, rvdw, beta=0.83, a=6.0, n_freq=15, param="omega", gradients=True,
                   errors=True):
    """MBD@rsSCS energy (and dE/dR) of a finite system (mbd_rsscs_evaluate);
    also returns the screened parameters (alpha0, C6, omega, R_vdW)."""
    ctx.sync_stream()
    dev = ctx.device
    s, keep = make_system(coords, alpha0, omega, rvdw, beta, a, param=param, device=dev)
    N = s.n_atoms
    out = {"energy": torch.empty(1, dtype=torch.float64, device=dev),
           "scs": torch.empty(4, N, dtype=torch.float64, device=dev)}
    r = A.MbdResult()
    r.energy = out["energy"].data_ptr()
    want = A.MBD_WANT_ENERGY
    if gradients:
        out["grad_coords"] = torch.empty(N, 3, dtype=torch.float64, device=dev)
        r.grad_coords = out["grad_coords"].data_ptr()
        want |= A.MBD_WANT_GRAD_COORDS
    if errors:
        out["errors"] = torch.zeros(4, dtype=torch.float64, device=dev)
        r.errors = out["errors"].data_ptr()
        want |= A.MBD_WANT_ERRORS
    code = A.mbd_rsscs_evaluate(ctx.handle, s, n_freq, want, r, out["scs"].data_ptr())
    if code != A.MBD_OK:
        _raise(ctx, code)
    return out


def evaluate_batch(ctx, systems, gradients=True, errors=True):
    """systems: list of dicts with coords, alpha0, omega, rvdw (, beta, a).  Finite only."""
    ctx.sync_stream()
    dev = ctx.device
    n = len(systems)
    sarr = (A.MbdSystem * n)()
    rarr = (A.MbdResult * n)()
    stat = (ctypes.c_int32 * n)()
    keep, outs = [], []
    want = A.MBD_WANT_ENERGY
    if gradients:
        want |= A.MBD_WANT_GRAD_COORDS | A.MBD_WANT_GRAD_ALPHA0 | A.MBD_WANT_GRAD_OMEGA
    if errors:
        want |= A.MBD_WANT_ERRORS
    for i, sy in enumerate(systems):
        s, k = make_system(sy["coords"], sy["alpha0"], sy["omega"], sy["rvdw"], sy.get("beta", 0.83),
                           sy.get("a", 6.0), device=dev)
        keep.append(k)
        sarr[i] = s
    # one allocation per output kind for the whole batch; each system gets views
    sizes = [sarr[i].n_atoms for i in range(n)]
    tot = sum(sizes)
    energy_all = torch.empty(n, dtype=torch.float64, device=dev)
    if gradients:
        gc_all = torch.empty(tot, 3, dtype=torch.float64, device=dev)
        ga_all = torch.empty(tot, dtype=torch.float64, device=dev)
        gw_all = torch.empty(tot, dtype=torch.float64, device=dev)
    if errors:
        err_all = torch.zeros(n, 4, dtype=torch.float64, device=dev)
    off = 0
    for i in range(n):
        N = sizes[i]
        o = {"energy": energy_all[i:i + 1]}
        rarr[i].energy = o["energy"].data_ptr()
        if gradients:
            o["grad_coords"] = gc_all[off:off + N]
            o["grad_alpha0"] = ga_all[off:off + N]
            o["grad_omega"] = gw_all[off:off + N]
            rarr[i].grad_coords = o["grad_coords"].data_ptr()
            rarr[i].grad_alpha0 = o["grad_alpha0"].data_ptr()
            rarr[i].grad_omega_or_c6 = o["grad_omega"].data_ptr()
        if errors:
            o["errors"] = err_all[i]
            rarr[i].errors = o["errors"].data_ptr()
        outs.append(o)
        off += N
    code = A.mbd_evaluate_batch(ctx.handle, sarr, want, rarr, stat)
    for i in range(n):
        outs[i]["status"] = int(stat[i])
    if code not in (A.MBD_OK, A.MBD_ERR_NEGATIVE_EIGENVALUE):
        _raise(ctx, code)
    return outs


def eigh(ctx, A_mat, vectors=True):
    """Symmetric eigendecomposition of a (batch of) square device matrices
    (float64 or float32).  Returns (w ascending, Z with eigenvectors as columns)."""
    ctx.sync_stream()
    M = A_mat
    squeeze = M.dim() == 2
    if squeeze:
        M = M.unsqueeze(0)
    M = M.contiguous().clone()
    nb, n, _ = M.shape
    dtype = 0 if M.dtype == torch.float64 else 1
    w = torch.empty(nb, n, dtype=M.dtype, device=M.device)
    Z = torch.empty(nb, n, n, dtype=M.dtype, device=M.device) if vectors else None
    code = A.mbd_eigh(ctx.handle, dtype, n, nb, M.data_ptr(), n, n * n, w.data_ptr(),
                      Z.data_ptr() if vectors else None, n, n * n)
    if code != A.MBD_OK:
        _raise(ctx, code)
    if vectors:
        Z = Z.transpose(1, 2)  # column-major result: Z[b][:, k] is eigenvector k
    if squeeze:
        return w[0], (Z[0] if vectors else None)
    return w, Z
