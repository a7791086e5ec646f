"""Benchmark: MBD energy + forces on one MI355X.

Headline (one step = one full evaluation of the hot path on the N=2000 finite
cluster, n = 6000 real symmetric Q): assembly, Householder reduction, divide
and conquer, back-transform, refinement, energy, adjoint gradients.  Inputs
are resident in HBM before timing starts.  The value is the FP32 +
Ogita-Aishima refinement path (seconds per evaluation, lower is better); the
plain FP64 GPU path is timed the same way beside it, with the error of every
result against FP64.

Secondary legs, reported in the same JSON line:
  batch     512 molecules, N ~ U{10..300}, energies + forces per molecule, one
            captured launch graph per call (systems/s, FP32+refine and FP64,
            per-molecule error of FP32+refine against FP64)
  periodic  64-atom triclinic cell, 4x4x4 Monkhorst-Pack mesh (64 Hermitian
            192x192 matrices in one batch), energy + dE/dR + dE/dlattice
  ts        pairwise (TS) energy + gradients: N=2000 cluster and the 64-atom
            crystal (Ewald), errors against the oracle
  freq      frequency route on the 64-atom crystal (15 frequencies x 64 q)
  rsscs     MBD@rsSCS on the N=2000 cluster (screening + MBD energy/forces)

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--legs c2,batch,periodic,ts,freq,rsscs] [--tuning-dir DIR]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3
SYMV_SOURCE = os.path.join(ROOT, "paper_2308_03140_amd", "csrc", "k_sytrd.hip")
# The per-column launches of the FP32 reduction: a SYMV launch (plus a finish
# launch) per column while the trailing order exceeds FUSED_MAX_ORDER, one
# fused launch per column below it.  Profiling kind, kernel, counter file.
COLUMN_KERNELS = {
    0: ("sytrd_symv_kernel<float", os.path.join(ROOT, "profiles", "sytrd_symv_fp32_n6000_pmc.txt")),
    8: ("sytrd_col_kernel<float", os.path.join(ROOT, "profiles", "sytrd_col_fp32_n6000_pmc.txt")),
}
FUSED_MAX_ORDER = 4000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_info():
    """CPU model and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None and core is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return model, (len(cores) or None)


def cpu_baseline(sizes=(500, 700), n_full=2000):
    """The oracle as it stands (Jacobi eigensolver, energy + gradients) on a
    bounded sample: the first n atoms of the N=2000 cluster for two sample
    sizes.  The cost exponent p is fitted from the two times (Jacobi's sweep
    count grows with n, so it is not exactly 3) and the larger sample is
    extrapolated to N=2000 with it."""
    import math

    import gen
    import oracle
    c = gen.cluster_n2000()
    oracle.mbd_finite(c["coords"][:20], c["alpha0"][:20], c["omega"][:20], c["rvdw"][:20])  # warm
    t = {}
    for n in sizes:
        sl = slice(0, n)
        t0 = time.perf_counter()
        oracle.mbd_finite(c["coords"][sl], c["alpha0"][sl], c["omega"][sl], c["rvdw"][sl], c["beta"], c["a"])
        t[n] = time.perf_counter() - t0
    a, b = sizes
    p = math.log(t[b] / t[a]) / math.log(b / a)
    value = t[b] * (n_full / b) ** p
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model, phys = _cpu_info()
    return {"value": value, "unit": "s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "physical_cores": phys, "fitted_exponent": p,
            "sample": "oracle energy+gradients (cyclic Jacobi) on the first %d and %d atoms of the N=2000 cluster "
                      "(%.2f s and %.2f s measured); cost exponent fitted from the two, %.2f; the %d-atom time "
                      "extrapolated with it to one N=%d evaluation" % (a, b, t[a], t[b], p, b, n_full)}


def column_traffic(kind):
    """HBM bytes per launch of one per-column kernel from the committed
    rocprofv3 counter runs (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when the kernel source has changed since the
    counters were taken."""
    path = COLUMN_KERNELS[kind][1]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    with open(SYMV_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if kv.get("kernel_source_sha256_16") != sha or "hbm_bytes_per_launch" not in kv:
        return None
    return float(kv["hbm_bytes_per_launch"])


def timed(fn, steps, warmup, torch):
    out = None
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def leg_c2(args, torch, T, A):
    import gen
    dev = torch.device("cuda", 0)
    c = gen.cluster_n2000()
    N = len(c["omega"])
    coords = torch.tensor(c["coords"], device=dev)
    a0 = torch.tensor(c["alpha0"], device=dev)
    om = torch.tensor(c["omega"], device=dev)
    rv = torch.tensor(c["rvdw"], device=dev)
    torch.cuda.synchronize()
    res = {}
    for prec in ("fp64", "fp32_refined"):
        ctx = T.Context(0, prec)
        log("[bench] c2 %s autotune n=%d" % (prec, 3 * N))
        t0 = time.perf_counter()
        ctx.autotune([3 * N], os.path.join(args.tuning_dir, "tuning_%s.json" % prec) if args.tuning_dir else None)
        tune_s = time.perf_counter() - t0

        def step():
            return T.evaluate(ctx, coords, a0, om, rv, beta=c["beta"], a=c["a"], gradients=True, errors=True)

        log("[bench] c2 %s warmup x%d, timed x%d" % (prec, args.warmup, args.steps))
        dt, out = timed(step, args.steps, args.warmup, torch)
        log("[bench] c2 %s %.4f s/step" % (prec, dt))
        # each phase on the host clock (no timing events: once the stream has
        # recorded timing events every later dispatch is timestamped, which
        # slows the launch-bound reduction), then launch-level timing of the
        # reduction kernels in a separate, profiled evaluation
        prof = {}
        A.mbd_set_profiling(ctx.handle, 2)
        step()
        for kind in range(2, 8):
            st, ms, nl, work = A.mbd_get_profile(ctx.handle, kind)
            prof[kind] = (ms, nl, work)
        A.mbd_set_profiling(ctx.handle, 1)
        step()
        for kind in (0, 1, 8):
            st, ms, nl, work = A.mbd_get_profile(ctx.handle, kind)
            prof[kind] = (ms, nl, work)
        A.mbd_set_profiling(ctx.handle, 0)
        res[prec] = {"s": dt, "tune_s": tune_s, "prof": prof,
                     "out": {k: v.detach().cpu().numpy() for k, v in out.items()}}
        ctx.close()
    res["N"] = N
    res["alpha_scale"] = c["alpha_scale"]
    return res


PHASES = {2: "assembly", 3: "reduction", 4: "divide_and_conquer", 5: "back_transform", 6: "refinement",
          7: "energy_and_gradients"}


def phase_rooflines(prof, n, fp32, eval_s):
    """Per-phase time of one profiled evaluation against the time the phase's
    algorithmic work takes at the MI355X peaks (HBM 8 TB/s; FP32 and FP64
    matrix cores 157.3 and 78.6 TFLOP/s): assembly writes Q (8 n^2 B, and
    4 n^2 B for the FP32 copy); the reduction reads the lower trailing triangle
    once per column (n^3/6 elements) and does (2/3) n^3 rank-2k flops; divide
    and conquer at most (4/3) n^3 merge flops; the back-transform 2 n^3; one
    refinement step 6 n^3 FP64; Q^{-1/2} n^3 FP64 plus one pass over it.
    The phases are timed on the host clock with the stream synchronised at
    their boundaries (no timing events); the reduction is also given as the
    timed step minus the other phases ("in_evaluation"), a check that the
    synchronisation does not distort it."""
    es = 4 if fp32 else 8
    peak = FP32_PEAK_TFS if fp32 else FP64_PEAK_TFS
    tmin = {2: (8 + (4 if fp32 else 0)) * n * n / (HBM_PEAK_GBS * 1e9),
            3: n ** 3 / 6 * es / (HBM_PEAK_GBS * 1e9) + (2.0 / 3.0) * n ** 3 / (peak * 1e12),
            4: (4.0 / 3.0) * n ** 3 / (peak * 1e12),
            5: 2.0 * n ** 3 / (peak * 1e12),
            6: 6.0 * n ** 3 / (FP64_PEAK_TFS * 1e12) if fp32 else 0.0,
            7: n ** 3 / (FP64_PEAK_TFS * 1e12) + 8 * n * n / (HBM_PEAK_GBS * 1e9)}
    out, tot_ms, tot_min = {}, 0.0, 0.0
    for k, name in PHASES.items():
        ms = prof[k][0]
        if prof[k][1] == 0:
            continue
        t = tmin[k] * 1e3
        out[name] = {"ms": ms, "t_min_ms": t, "frac": t / ms if ms > 0 else None}
        tot_ms += ms
        tot_min += t
    out["sum"] = {"ms": tot_ms, "t_min_ms": tot_min, "frac": tot_min / tot_ms if tot_ms > 0 else None}
    if "reduction" in out:
        red = eval_s * 1e3 - sum(v["ms"] for k, v in out.items() if k not in ("reduction", "sum"))
        out["reduction"]["ms_in_evaluation"] = red
        out["reduction"]["frac_in_evaluation"] = out["reduction"]["t_min_ms"] / red if red > 0 else None
    out["evaluation"] = {"ms": eval_s * 1e3, "t_min_ms": tot_min, "frac": tot_min / (eval_s * 1e3)}
    return out


def leg_batch(args, torch, T):
    import numpy as np

    import gen
    dev = torch.device("cuda", 0)
    mols = gen.molecule_batch()
    systems = [{"coords": torch.tensor(m["coords"], device=dev), "alpha0": torch.tensor(m["alpha0"], device=dev),
                "omega": torch.tensor(m["omega"], device=dev), "rvdw": torch.tensor(m["rvdw"], device=dev),
                "beta": m["beta"], "a": m["a"]} for m in mols]
    torch.cuda.synchronize()
    nmax = max(3 * len(m["omega"]) for m in mols)
    res = {}
    for prec in ("fp32_refined", "fp64"):
        ctx = T.Context(0, prec)
        ctx.autotune([nmax])
        log("[bench] batch %s warmup x%d, timed x%d" % (prec, args.warmup, args.steps))
        dt, outs = timed(lambda: T.evaluate_batch(ctx, systems), args.steps, args.warmup, torch)
        log("[bench] batch %s %.4f s/batch" % (prec, dt))
        res[prec] = {"s": dt, "outs": [{k: (v.detach().cpu().numpy() if hasattr(v, "detach") else v)
                                        for k, v in o.items()} for o in outs]}
        ctx.close()
    dE, dG, dA, dW, steps2, rem = [], [], [], [], 0, 0.0
    for m, o32, o64 in zip(mols, res["fp32_refined"]["outs"], res["fp64"]["outs"]):
        N = len(m["omega"])
        dE.append(abs(float(o32["energy"][0]) - float(o64["energy"][0])) / N)
        dG.append(float(np.abs(o32["grad_coords"] - o64["grad_coords"]).max()))
        dA.append(float(np.abs(o32["grad_alpha0"] - o64["grad_alpha0"]).max()))
        dW.append(float(np.abs(o32["grad_omega"] - o64["grad_omega"]).max()))
        steps2 += int(o32["errors"][2] >= 2.0)
        rem = max(rem, float(o32["errors"][3]))
    sizes = [len(m["omega"]) for m in mols]
    status = [o["status"] for o in res["fp32_refined"]["outs"]]
    return {"workload": "512 molecules, N ~ U{10..300} (matrices 30..900), seed 4, one captured graph per call",
            "n_systems": len(mols), "atoms_total": int(sum(sizes)),
            "systems_per_s": len(mols) / res["fp32_refined"]["s"], "s_per_batch": res["fp32_refined"]["s"],
            "fp64_systems_per_s": len(mols) / res["fp64"]["s"], "fp64_s_per_batch": res["fp64"]["s"],
            "nonzero_status": int(sum(1 for s in status if s != 0)),
            "molecules_with_second_refinement_step": steps2,
            "max_refine_remainder_estimate": rem,
            "errors_vs_fp64_per_molecule": {
                "energy_per_atom_Ha": {"max": max(dE), "median": float(np.median(dE))},
                "grad_coords_Ha_per_bohr": {"max": max(dG), "median": float(np.median(dG))},
                "grad_alpha0": {"max": max(dA), "median": float(np.median(dA))},
                "grad_omega": {"max": max(dW), "median": float(np.median(dW))}}}


def leg_periodic(args, torch, T):
    import numpy as np

    import gen
    dev = torch.device("cuda", 0)
    c = gen.crystal_n64()
    coords = torch.tensor(c["coords"], device=dev)
    a0 = torch.tensor(c["alpha0"], device=dev)
    om = torch.tensor(c["omega"], device=dev)
    rv = torch.tensor(c["rvdw"], device=dev)
    torch.cuda.synchronize()
    res = {}
    for prec in ("fp32_refined", "fp64"):
        ctx = T.Context(0, prec)
        ctx.autotune([6 * 64])

        def step():
            return T.evaluate(ctx, coords, a0, om, rv, beta=c["beta"], a=c["a"], lattice=c["lattice"],
                              q_frac=c["q_frac"], gradients=True, errors=True)

        log("[bench] periodic %s warmup x%d, timed x%d" % (prec, args.warmup, args.steps))
        dt, out = timed(step, args.steps, args.warmup, torch)
        log("[bench] periodic %s %.4f s/step" % (prec, dt))
        # the same with time-reversed q points folded (32 of the 64 matrices)
        os.environ["MBD_Q_PAIRS"] = "1"
        try:
            dtp, _ = timed(step, args.steps, args.warmup, torch)
        finally:
            del os.environ["MBD_Q_PAIRS"]
        log("[bench] periodic %s, q pairs folded: %.4f s/step" % (prec, dtp))
        res[prec] = {"s": dt, "s_pairs": dtp, "out": {k: v.detach().cpu().numpy() for k, v in out.items()}}
        ctx.close()
    o32, o64 = res["fp32_refined"]["out"], res["fp64"]["out"]
    return {"workload": "64-atom triclinic cell, 4x4x4 Monkhorst-Pack (64 Hermitian 192x192 = real 384x384), "
                        "Ewald defaults, seed 3, alpha0 x %.4f" % c["alpha_scale"],
            "s_per_eval": res["fp32_refined"]["s"], "fp64_s_per_eval": res["fp64"]["s"],
            "q_pairs_folded": {"s_per_eval": res["fp32_refined"]["s_pairs"],
                               "fp64_s_per_eval": res["fp64"]["s_pairs"]},
            "errors_vs_fp64": {
                "energy_per_atom_Ha": abs(float(o32["energy"][0]) - float(o64["energy"][0])) / 64,
                "grad_coords_Ha_per_bohr": float(np.abs(o32["grad_coords"] - o64["grad_coords"]).max()),
                "grad_alpha0": float(np.abs(o32["grad_alpha0"] - o64["grad_alpha0"]).max()),
                "grad_lattice_Ha_per_bohr": float(np.abs(o32["grad_lattice"] - o64["grad_lattice"]).max())}}


TS_SR, TS_A = 0.94, 20.0
# FP64 operations of one finite pair term of the pairwise kernel, counted from
# its source: distance (3 sub, 3 fma, sqrt ~ 10, reciprocal ~ 10, 3 mul), C6
# and its omega factor (reciprocal ~ 10, 8 mul), Fermi factor (2 reciprocals
# ~ 20, exp ~ 20, ~ 10), energy, gradient and parameter terms (~ 25)
TS_OPS_PER_PAIR = 120


def leg_ts(args, torch, T, A):
    """Pairwise (TS) dispersion: N=2000 cluster (finite, all ordered pairs) and
    the 64-atom crystal (periodic, Ewald split), energy + all gradients, FP64;
    error of every result against the oracle.  Per call: the wall time of the
    whole call (setup, launches, status read-back) and the pair kernel's own
    time from its launch events (profiling kind 11)."""
    import numpy as np

    import gen
    import oracle
    dev = torch.device("cuda", 0)
    ctx = T.Context(0, "fp64")
    out = {}
    for name, c in (("finite_n2000", gen.cluster_n2000()), ("crystal_n64", gen.crystal_n64())):
        lat = c["lattice"] if name.startswith("crystal") else None
        coords = torch.tensor(c["coords"], device=dev)
        a0 = torch.tensor(c["alpha0"], device=dev)
        om = torch.tensor(c["omega"], device=dev)
        rv = torch.tensor(c["rvdw"], device=dev)

        def step():
            return T.ts_evaluate(ctx, coords, a0, om, rv, TS_SR, TS_A, lattice=lat)

        log("[bench] ts %s warmup x%d, timed x%d" % (name, args.warmup, 4 * args.steps))
        dt, o = timed(step, 4 * args.steps, args.warmup, torch)
        A.mbd_set_profiling(ctx.handle, 1)
        for _ in range(4 * args.steps):
            step()
        _, kms, kn, kterms = A.mbd_get_profile(ctx.handle, 11)
        A.mbd_set_profiling(ctx.handle, 0)
        kt = kms * 1e-3 / max(kn, 1)
        ref = oracle.ts(c["coords"], c["alpha0"], c["omega"], c["rvdw"], sR=TS_SR, a=TS_A, lattice=lat)
        N = len(c["omega"])
        res = {"s_per_eval": dt, "kernel_s": kt, "pair_terms": kterms / max(kn, 1),
               "errors_vs_oracle": {
                   "energy_per_atom_Ha": abs(o["energy"].item() - ref["energy"]) / N,
                   "grad_coords_Ha_per_bohr": float(np.abs(o["grad_coords"].cpu().numpy() - ref["grad_R"]).max())}}
        if lat is None:
            pairs = N * (N - 1)
            res["pairs_per_s"] = pairs / dt
            res["alu_roofline"] = {"bound": "alu", "ops_per_pair": TS_OPS_PER_PAIR, "time": "pair kernel",
                                   "achieved_TFs": pairs * TS_OPS_PER_PAIR / kt / 1e12, "peak": FP64_PEAK_TFS,
                                   "frac": pairs * TS_OPS_PER_PAIR / kt / 1e12 / FP64_PEAK_TFS}
        out[name] = res
    ctx.close()
    out["workload"] = ("pairwise (TS) energy + dE/dR, dE/dalpha0, dE/domega, dE/dRv; s_R = %.2f, a = %g; N=2000 "
                       "cluster (finite) and 64-atom crystal (periodic, Ewald defaults)" % (TS_SR, TS_A))
    return out


def leg_freq(args, torch, T, A):
    """Frequency route on the 64-atom crystal: 15 frequencies x 64 q points =
    960 embedded matrices of order 384 in one batch (eigenvalues only), with
    the log-formula energy against the eigenvalue-route energy (their
    difference is the 15-point quadrature error) and the renormalised energy
    and many-body orders."""
    import gen
    dev = torch.device("cuda", 0)
    c = gen.crystal_n64()
    ctx = T.Context(0, "fp64")
    coords = torch.tensor(c["coords"], device=dev)

    def step():
        return T.freq_evaluate(ctx, coords, c["alpha0"], c["omega"], c["rvdw"], beta=c["beta"], a=c["a"],
                               lattice=c["lattice"], q_frac=c["q_frac"], n_freq=15, n_order=6)

    log("[bench] freq warmup x%d, timed x%d" % (args.warmup, args.steps))
    dt, o = timed(step, args.steps, args.warmup, torch)
    e = T.evaluate(ctx, coords, c["alpha0"], c["omega"], c["rvdw"], beta=c["beta"], a=c["a"], lattice=c["lattice"],
                   q_frac=c["q_frac"], gradients=False)["energy"].item()
    A.mbd_set_profiling(ctx.handle, 2)
    step()
    ph = {k: A.mbd_get_profile(ctx.handle, k)[1] for k in (3, 4)}
    A.mbd_set_profiling(ctx.handle, 0)
    ctx.close()
    n, nm = 384, 960
    return {"workload": "64-atom crystal, 4x4x4 mesh, 15 frequencies: 960 matrices of order 384, eigenvalues only",
            "s_per_eval": dt, "energy_log_formula": o["energy"].item(), "energy_eigen_route": e,
            "quadrature_error_rel": abs(o["energy"].item() - e) / abs(e),
            "energy_gould": o["energy_gould"].item(), "min_one_plus_x": o["min_one_plus_x"].item(),
            "orders": [float(x) for x in o["orders"].cpu().numpy()],
            "phases_ms": {"reduction": ph[3], "eigenvalues": ph[4]},
            "reduction_t_min_ms": nm * n ** 3 / 6 * 8 / (HBM_PEAK_GBS * 1e9) * 1e3}


def leg_rsscs(args, torch, T, A):
    """MBD@rsSCS on the N=2000 cluster: the screening stage (16 FP64
    Cholesky factorisations of order 6000, u = 0 and 15 frequencies, and
    three-column solves) and the MBD energy + forces (FP32+refine) with the
    screened parameters; phase times (screening: profiling kind 9)."""
    import gen
    dev = torch.device("cuda", 0)
    c = gen.cluster_n2000()
    ctx = T.Context(0, "fp32_refined")
    coords = torch.tensor(c["coords"], device=dev)

    def step():
        return T.rsscs_evaluate(ctx, coords, c["alpha0"], c["omega"], c["rvdw"], beta=c["beta"], a=c["a"],
                                n_freq=15)

    steps = max(1, args.steps // 2)
    log("[bench] rsscs warmup x1, timed x%d" % steps)
    dt, o = timed(step, steps, 1, torch)
    A.mbd_set_profiling(ctx.handle, 2)
    step()
    ph = {PHASES[k]: A.mbd_get_profile(ctx.handle, k)[1] for k in range(2, 8)}
    scr = A.mbd_get_profile(ctx.handle, 9)[1]
    A.mbd_set_profiling(ctx.handle, 0)
    ctx.close()
    n = 6000
    # screening bound: the 16 factorisations' n^3/3 flops at the FP64 matrix
    # peak and one write and read of the 16 matrices at the HBM peak
    t_min = (16 * n ** 3 / 3 / (FP64_PEAK_TFS * 1e12) + 2 * 16 * n * n * 8 / (HBM_PEAK_GBS * 1e9)) * 1e3
    return {"workload": "N=2000 cluster, 15 frequencies + u = 0 (16 FP64 Cholesky factorisations of order 6000 "
                        "and three-column solves), then MBD energy + forces FP32+refine",
            "s_per_eval": dt, "energy": o["energy"].item(),
            "screening_ms": scr, "screening_t_min_ms": t_min, "screening_frac": t_min / scr if scr > 0 else None,
            "mbd_stage_phases_ms": ph}


def pmc_pass(torch, T):
    """Runs under rocprofv3 --pmc: one FP32+refine N=2000 evaluation with every
    kernel dispatched individually (no launch graph, default launch shapes, so
    the counter collection sees each dispatch), then one device-to-device copy
    of 2^28 floats (1 GiB read + 1 GiB written) whose counters calibrate
    FETCH_SIZE and WRITE_SIZE.  (A second evaluation, about 25k counted
    dispatches in all, ended in a host-side crash inside the profiler.)"""
    import gen
    os.environ["MBD_NO_GRAPH"] = "1"
    dev = torch.device("cuda", 0)
    c = gen.cluster_n2000()
    args = [torch.tensor(c[k], device=dev) for k in ("coords", "alpha0", "omega", "rvdw")]
    ctx = T.Context(0, "fp32_refined")
    log("[bench] pmc pass: evaluation")
    T.evaluate(ctx, *args, beta=c["beta"], a=c["a"])
    torch.cuda.synchronize()
    x = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    log("[bench] pmc pass: 1 GiB copy")
    y.copy_(x)
    torch.cuda.synchronize()
    ctx.close()


def column_launches(n, tail=256, panel=32, fused_max=FUSED_MAX_ORDER):
    """Per-column launches of one FP32 reduction of a single matrix of order
    n, as {profiling kind: count}: one per column up to the panel boundary
    where the last columns (at most `tail`) are reduced in LDS; a panel
    starting at column k0 runs fused launches (kind 8) when n - k0 - 1 <=
    fused_max (and its work items are short, which holds for one matrix at
    the default targets)."""
    start = 0 if n <= tail else -(-(n - tail) // panel) * panel
    start = min(n - 1, start)
    out = {0: 0, 8: 0}
    for k0 in range(0, start, panel):
        out[8 if n - k0 - 1 <= fused_max else 0] += min(panel, start - k0)
    return out


def _pmc_dispatches(d):
    """(kernel name, summed counter value) per dispatch, in dispatch order, from
    a rocprofv3 --pmc CSV directory (one counter per run)."""
    import csv
    files = [os.path.join(r, f) for r, _, fs in os.walk(d) for f in fs if f.endswith("counter_collection.csv")]
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    per = {}
    for fn in files:
        with open(fn) as f:
            for row in csv.DictReader(f):
                key = int(row.get("Dispatch_Id") or row.get("Correlation_Id"))
                name = row.get("Kernel_Name", "")
                val = float(row.get("Counter_Value", 0.0))
                if key in per:
                    per[key][1] += val
                else:
                    per[key] = [name, val]
    return [tuple(per[k]) for k in sorted(per)]


def pmc_summary(fetch_dir, write_dir):
    """Turns the FETCH_SIZE and WRITE_SIZE runs of --pmc-pass into the HBM bytes
    per launch of each per-column kernel (the files named in COLUMN_KERNELS):
    counters are in KiB per dispatch; each is scaled by bytes/counter measured
    on the 1 GiB copy of the same run."""
    with open(SYMV_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    total = sum(column_launches(6000).values())
    disp = {name: _pmc_dispatches(d) for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir))}
    for name, dl in disp.items():
        got = sum(1 for k, _ in dl if any(kn in k for kn, _ in COLUMN_KERNELS.values()))
        if got != total:
            raise SystemExit("%s: %d per-column dispatches, expected the %d of one evaluation" % (name, got, total))
    for kind, (kname, path) in COLUMN_KERNELS.items():
        out = {}
        for name, dl in disp.items():
            vals = [v for k, v in dl if kname in k]
            if not vals:
                raise SystemExit("%s: no dispatch of %s" % (name, kname))
            copies = [v for k, v in dl if "copy" in k.lower()]
            if not copies:
                raise SystemExit("%s: no copy dispatch for the calibration" % name)
            cal = float(1 << 30) / max(copies)  # bytes per counter unit on the 1 GiB copy
            out[name] = (sum(vals) / len(vals), max(copies), cal)
        fetch, wr = out["FETCH_SIZE"], out["WRITE_SIZE"]
        hbm = fetch[0] * fetch[2] + wr[0] * wr[2]
        lines = [
            "# rocprofv3 counters of %s> at N=2000 (n=6000), FP32+refine path" % kname,
            "# commands (repository root, MI355X):",
            "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d %s -o f -- python3 bench.py --pmc-pass" % fetch_dir,
            "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d %s -o w -- python3 bench.py --pmc-pass" % write_dir,
            "#   python3 bench.py --pmc-summary %s %s" % (fetch_dir, write_dir),
            "# averages over the %d dispatches of one evaluation; calibration on the 1 GiB copy" % len(vals),
            "fetch_counter_avg = %.3f" % fetch[0],
            "write_counter_avg = %.3f" % wr[0],
            "copy_fetch_counter = %.3f" % fetch[1],
            "copy_write_counter = %.3f" % wr[1],
            "bytes_per_fetch_unit = %.6f" % fetch[2],
            "bytes_per_write_unit = %.6f" % wr[2],
            "hbm_bytes_per_launch = %.1f" % hbm,
            "kernel_source_sha256_16 = %s" % sha,
        ]
        with open(path, "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))


MFMA_PMC = os.path.join(ROOT, "profiles", "gemm_mfma_fp32_n6000_mfma.md")
MFMA_REGEX = "gemm_mfma_kernel|gemm_f16x3_kernel|xf_small_f16_kernel"


def _short(name):
    name = name.replace("void ", "")
    return name if len(name) <= 110 else name[:107] + "..."


def mfma_summary(pmc_dir, trace_dir):
    """Matrix-core utilisation of the GEMM kernels of one FP32+refine N=2000
    evaluation (--pmc-pass), per kernel instantiation: MFMA flops from the
    MfmaFlopsF16/F32/F64 counters (MOPS x 512), kernel time from a kernel-trace
    run of the same pass, and the MfmaUtil counter (MFMA busy cycles over
    active cycles of all SIMDs)."""
    import csv
    pfiles = [os.path.join(r, f) for r, _, fs in os.walk(pmc_dir) for f in fs if f.endswith("counter_collection.csv")]
    tfiles = [os.path.join(r, f) for r, _, fs in os.walk(trace_dir) for f in fs if f.endswith("kernel_trace.csv")]
    if not pfiles or not tfiles:
        raise SystemExit("need counter_collection.csv under %s and kernel_trace.csv under %s" % (pmc_dir, trace_dir))
    disp = {}
    for fn in pfiles:
        with open(fn) as f:
            for row in csv.DictReader(f):
                key = int(row.get("Dispatch_Id") or row.get("Correlation_Id"))
                d = disp.setdefault(key, {"name": row.get("Kernel_Name", "")})
                d[row["Counter_Name"]] = d.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    counted = [disp[k] for k in sorted(disp)]
    traced = []
    for fn in tfiles:
        with open(fn) as f:
            traced += [r for r in csv.DictReader(f)]
    traced.sort(key=lambda r: int(r["Start_Timestamp"]))
    traced = [r for r in traced if any(x in r["Kernel_Name"] for x in MFMA_REGEX.split("|"))]
    if len(traced) != len(counted):
        raise SystemExit("%d traced vs %d counted GEMM dispatches" % (len(traced), len(counted)))
    groups = {}
    for c, t in zip(counted, traced):
        if c["name"] != t["Kernel_Name"]:
            raise SystemExit("dispatch order differs between the runs: %s / %s" % (c["name"], t["Kernel_Name"]))
        g = groups.setdefault(c["name"], {"n": 0, "ms": 0.0, "f16": 0.0, "f32": 0.0, "f64": 0.0, "util_ms": 0.0})
        ms = (int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) * 1e-6
        g["n"] += 1
        g["ms"] += ms
        g["f16"] += c.get("MfmaFlopsF16", 0.0)
        g["f32"] += c.get("MfmaFlopsF32", 0.0)
        g["f64"] += c.get("MfmaFlopsF64", 0.0)
        g["util_ms"] += c.get("MfmaUtil", 0.0) * ms
    peaks = {"f16": 2500.0, "f32": FP32_PEAK_TFS, "f64": FP64_PEAK_TFS}
    lines = ["# Matrix-core utilisation of the GEMM kernels, one FP32+refine evaluation at N=2000 (n=6000)", "",
             "Commands (repository root, MI355X):", "",
             "    rocprofv3 --pmc MfmaUtil MfmaFlopsF16 MfmaFlopsF32 MfmaFlopsF64 --kernel-include-regex "
             "'%s' --output-format csv -d %s -o m -- python3 bench.py --pmc-pass" % (MFMA_REGEX, pmc_dir),
             "    rocprofv3 --kernel-trace --stats --kernel-include-regex '%s' --output-format csv "
             "-d %s -o t -- python3 bench.py --pmc-pass" % (MFMA_REGEX, trace_dir),
             "    python3 bench.py --mfma-summary %s %s" % (pmc_dir, trace_dir), "",
             "Flops = MFMA MOPS x 512 (counter); time = traced kernel duration; TF/s and fraction of the dense "
             "peak of the kernel's MFMA type (FP64 78.6, FP32 157.3, FP16 2500 TFLOP/s); MfmaUtil = MFMA-busy "
             "cycles over active cycles of all SIMDs, time-weighted.", "",
             "| kernel | dispatches | total ms | MFMA type | TFLOP/s | frac of peak | MfmaUtil % |",
             "|---|---|---|---|---|---|---|"]
    tot = {"f16": [0.0, 0.0], "f32": [0.0, 0.0], "f64": [0.0, 0.0]}
    for name, g in sorted(groups.items(), key=lambda kv: -kv[1]["ms"]):
        typ = max(("f16", "f32", "f64"), key=lambda k: g[k])
        fl = g[typ]
        tfs = fl / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
        tot[typ][0] += fl
        tot[typ][1] += g["ms"]
        lines.append("| `%s` | %d | %.3f | %s | %.1f | %.3f | %.1f |" % (
            _short(name), g["n"], g["ms"], typ.upper(), tfs, tfs / peaks[typ], g["util_ms"] / g["ms"] if g["ms"] else 0))
    lines += ["", "| MFMA type | total ms | TFLOP/s | frac of peak |", "|---|---|---|---|"]
    for typ, (fl, ms) in tot.items():
        if ms > 0:
            tfs = fl / (ms * 1e-3) / 1e12
            lines.append("| %s | %.3f | %.1f | %.3f |" % (typ.upper(), ms, tfs, tfs / peaks[typ]))
    with open(MFMA_PMC, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(trace_dir, steps, warmup):
    """Average duration of each FP32 per-column kernel over the evaluations of
    a `--legs c2` run traced by rocprofv3 --kernel-trace (its kernel_trace.csv
    under trace_dir).  Every FP32 reduction ends with one LDS tail launch, so
    the trace is cut there: the per-column launches of the last warmup +
    steps + 1 reductions (warm-up, timed, profiled) are kept and the
    autotuner's candidate reductions before them left out."""
    import csv
    files = [os.path.join(r, f) for r, _, fs in os.walk(trace_dir) for f in fs if f.endswith("kernel_trace.csv")]
    if not files:
        raise SystemExit("no kernel_trace.csv under %s" % trace_dir)
    rows = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                if name.startswith("void sytrd_tail_kernel<float") or any(
                        name.startswith("void " + k) for k, _ in COLUMN_KERNELS.values()):
                    rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), name))
    rows.sort()
    segs, cur = [], []
    for s0, e0, name in rows:
        if name.startswith("void sytrd_tail_kernel"):
            segs.append(cur)
            cur = []
        else:
            cur.append((name, (e0 - s0) * 1e-3))
    n_eval = warmup + steps + 1  # warm-up, timed (captured graphs), one profiled eager evaluation
    if len(segs) < n_eval:
        raise SystemExit("%d FP32 reductions in the trace, fewer than %d" % (len(segs), n_eval))
    ev = segs[-n_eval:]
    for kind, (kname, _) in sorted(COLUMN_KERNELS.items()):
        per = [[d for nm, d in sg if nm.startswith("void " + kname)] for sg in ev]
        if not per[-1]:
            print("%s>: no launches" % kname)
            continue
        allv = [d for sg in per for d in sg]
        timed = [d for sg in per[warmup:warmup + steps] for d in sg]
        prof = per[-1]
        print("%s>: %d launches per reduction" % (kname, len(prof)))
        print("  the %d launches of the %d evaluations: %.2f us" % (len(allv), n_eval, sum(allv) / len(allv)))
        print("  the %d launches of the %d timed (captured-graph) evaluations: %.2f us"
              % (len(timed), steps, sum(timed) / len(timed)))
        print("  the %d launches of the profiled evaluation: %.2f us" % (len(prof), sum(prof) / len(prof)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="c2,batch,periodic,ts,freq,rsscs",
                    help="legs to run; without c2 the named legs run alone and print their results only")
    ap.add_argument("--tuning-dir", default=None, help="write the autotuner tables (JSON) here")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="write the SYMV HBM-traffic file under profiles/ from two --pmc-pass counter runs")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR", default=None,
                    help="average SYMV kernel duration per evaluation from a rocprofv3 --kernel-trace run of "
                         "--legs c2 with the same --steps/--warmup")
    ap.add_argument("--mfma-summary", nargs=2, metavar=("PMC_DIR", "TRACE_DIR"), default=None,
                    help="write the matrix-core utilisation table of the GEMM kernels under profiles/ from a "
                         "--pmc-pass counter run (MfmaUtil, MfmaFlops*) and a kernel-trace run of the same pass")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="counter-collection pass: one FP32+refine N=2000 evaluation, then a plain device copy "
                         "of 1 GiB (the calibration kernel of known traffic); prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(q-point/molecule sharding is design-only); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.steps, args.warmup)
        return
    if args.mfma_summary:
        mfma_summary(*args.mfma_summary)
        return

    import numpy as np
    import torch

    from paper_2308_03140_amd import _abi as A
    from paper_2308_03140_amd import torch_api as T

    if args.pmc_pass:
        pmc_pass(torch, T)
        return
    if "c2" not in legs:
        # secondary legs on their own (profiling runs): their results only,
        # not the benchmark line
        out = {}
        for name, fn in (("batch", lambda: leg_batch(args, torch, T)), ("periodic", lambda: leg_periodic(args, torch, T)),
                         ("ts", lambda: leg_ts(args, torch, T, A)), ("freq", lambda: leg_freq(args, torch, T, A)),
                         ("rsscs", lambda: leg_rsscs(args, torch, T, A))):
            if name in legs:
                out[name] = fn()
        print(json.dumps(out), flush=True)
        return
    r = leg_c2(args, torch, T, A)
    e64, e32 = r["fp64"]["out"], r["fp32_refined"]["out"]
    N = r["N"]
    dE = abs(float(e32["energy"][0]) - float(e64["energy"][0])) / N
    dG = float(np.abs(e32["grad_coords"] - e64["grad_coords"]).max())
    dA = float(np.abs(e32["grad_alpha0"] - e64["grad_alpha0"]).max())
    dW = float(np.abs(e32["grad_omega"] - e64["grad_omega"]).max())

    # roofline of the dominant kernel: the per-column kernel of the FP32
    # reduction (SYMV or fused) with the larger total time
    col = {}
    for kind, (kname, _) in COLUMN_KERNELS.items():
        kms, knl, kb = r["fp32_refined"]["prof"][kind]
        if knl == 0:
            continue
        avg = kms * 1e-3 / knl
        col[kind] = {"kernel": kname + ">", "launches": knl, "total_ms": kms, "avg_launch_us": avg * 1e6,
                     "algorithmic_bytes_per_launch": kb / knl, "achieved_GBs": kb / knl / avg / 1e9,
                     "traffic": column_traffic(kind)}
    dom = max(col, key=lambda k: col[k]["total_ms"])
    ms, nl = col[dom]["total_ms"], col[dom]["launches"]
    avg_s = col[dom]["avg_launch_us"] * 1e-6
    bytes_per_launch = col[dom]["algorithmic_bytes_per_launch"]
    achieved = col[dom]["achieved_GBs"]
    traffic = col[dom]["traffic"]
    ms3, nl3, fl3 = r["fp32_refined"]["prof"][1]
    ms64, nl64, b64 = r["fp64"]["prof"][0]
    ms364, nl364, fl364 = r["fp64"]["prof"][1]

    line = {
        "metric": "N=2000 MBD energy+force time (s), FP32+refine vs FP64",
        "value": r["fp32_refined"]["s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["fp32_refined"]["s"] * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "finite cluster N=2000 atoms (Q 6000x6000 real symmetric), energy + forces; "
                               "seed 2, 0.1 atoms/A^3, alpha0 x %.4f (collapse rule)" % r["alpha_scale"],
                   "path": "FP32 reduction/D&C/back-transform on matrix cores + FP64 Ogita-Aishima refinement "
                           "(second step only where the first leaves a large remainder)"},
        "fp64_s": r["fp64"]["s"],
        "autotune_s": {p: r[p]["tune_s"] for p in ("fp64", "fp32_refined")},
        "speedup_fp32_refined_vs_fp64": r["fp64"]["s"] / r["fp32_refined"]["s"],
        "errors_vs_fp64": {"energy_per_atom_Ha": dE, "max_grad_coords_Ha_per_bohr": dG,
                           "max_grad_alpha0": dA, "max_grad_omega": dW,
                           "refine_orth_residual_before": float(e32["errors"][1]),
                           "refine_steps": float(e32["errors"][2]),
                           "refine_remainder_estimate": float(e32["errors"][3]),
                           "lambda_min": float(e64["errors"][0])},
        "roofline": {"bound": "hbm", "kernel": col[dom]["kernel"] + " (per-column reduction launch)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launches": nl, "avg_launch_us": avg_s * 1e6,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "per_column_kernels": list(col.values())},
        "phase_rooflines": {"fp32_refined": phase_rooflines(r["fp32_refined"]["prof"], 3 * N, True,
                                                            r["fp32_refined"]["s"]),
                            "fp64": phase_rooflines(r["fp64"]["prof"], 3 * N, False, r["fp64"]["s"])},
        "phases": {
            "fp32_column_GBs": achieved, "fp32_column_total_ms": sum(v["total_ms"] for v in col.values()),
            "fp32_syr2k_TFs": fl3 / (ms3 * 1e-3) / 1e12 if ms3 > 0 else None, "fp32_syr2k_total_ms": ms3,
            "fp64_symv_GBs": (b64 / max(nl64, 1)) / (ms64 * 1e-3 / max(nl64, 1)) / 1e9 if ms64 > 0 else None,
            "fp64_symv_total_ms": ms64,
            "fp64_syr2k_TFs": fl364 / (ms364 * 1e-3) / 1e12 if ms364 > 0 else None, "fp64_syr2k_total_ms": ms364,
        },
    }
    if "batch" in legs:
        line["batch"] = leg_batch(args, torch, T)
    if "periodic" in legs:
        line["periodic"] = leg_periodic(args, torch, T)
    if "ts" in legs:
        line["ts"] = leg_ts(args, torch, T, A)
    if "freq" in legs:
        line["freq"] = leg_freq(args, torch, T, A)
    if "rsscs" in legs:
        line["rsscs"] = leg_rsscs(args, torch, T, A)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
