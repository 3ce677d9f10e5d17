#!/usr/bin/env python
"""Benchmark of the Poisson-Fermi hot path on one MI355X.

A step is one batched solve of the 64 linearised Poisson-Boltzmann systems
(sizes 33^3 to 129^3, 49,173,256 unknowns, each the PF2 operator at
phi_0 = 0 with its own charge set and bath), every member Jacobi-BiCGSTAB
(Sec. 4, Table 3) in FP64 from x = 0 to true relative residual 1e-10, all
members' iterations in shared launches (one launch per BiCGSTAB step kernel
per iteration covering every member still iterating).  This is the largest
single-GPU workload of the benchmark set.  All inputs are resident in device
memory before the timed region starts.

The JSON line also carries:
  roofline      the batched BiCGSTAB step-A stencil kernel (the previous
                iteration's x, r update, the p update and v = A p^ in one
                pass over every iterating member), timed with HIP events on
                the library's stream over every launch of the timed steps
                (one chunk of iterations out of --sample, default 1: all of
                them, whose graph launches then become direct launches with
                dispatch-stamped events); algorithmic bytes per launch
                = 77 B per node of every member still iterating (reads s^,
                p^, v^, t^, x in FP64, the coefficient's one-byte palette
                index, which also selects the member's shift from its
                per-class table, and the FP32 shadow; writes x, r^, p^, v^);
  cpu_baseline  the serial FP64 oracle, pinned to one core, on a bounded
                sample of the members, extrapolated to the whole batch by
                node-iterations;
  forms         batched mixed precision and sequential FP64 on the same
                batch; FP64 vs mixed on the 193^3 Poisson problem with the
                per-iteration fraction of the HBM roofline; the isolated
                Jacobi-scaled product at 193^3 with cold operands; the
                device's streaming ceiling from the library's own probe; the
                97^3 full PF solve (cache-resident); the singular-charge
                decomposition; the 16-bias PF sweep at 129^3 with a stated
                outer-iteration cap.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "time to 1e-10 rel residual & HBM GB/s: FP64 vs mixed-precision vs batched"
# Bytes of one BiCGSTAB iteration per node: the method's own count for the
# fused schedule, 20 vectors of the working precision (operator from eps
# alone; reads r, p, v, eps, shadow / r, v, eps / x, p, s, t, shadow, eps;
# writes p, v / s, t / x, r), and this build's two kernels on a Poisson
# system: step A reads s^, p^, v^, t^, x, the coefficient and the FP32 shadow
# and writes x, r^, p^, v^ (9 elements + coefficient + 4 B); step B reads r^,
# v^, the coefficient and the shadow and writes s^, t^ (4 elements +
# coefficient + 4 B).  The coefficient is a one-byte palette index when the
# field has at most 128 distinct values (the sphere has two).
ITER_VECTORS_METHOD = 20.0


def iter_bytes_build(elem, palette=True):
    coef = 1 if (palette and os.environ.get("PF_PALETTE") != "0") else elem
    return 13 * elem + 2 * coef + 8
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector peak
# Coulomb kernel, per (point, charge) pair: 3 differences, 5 for r^2, 1 for the
# reciprocal square root, 2 for the potential term and its sum, 5 for the
# component along the derivative direction, 4 for the derivative term and sum
COULOMB_FLOP_PER_PAIR = 20.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the device source: traffic counters stay valid while it is unchanged."""
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_1711_04060_amd", "csrc", "pf_kernels.h"), "rb").read())
    return h.hexdigest()[:16]


PMC_BATCH_FILE = os.path.join(ROOT, "profiles", "pmc_batch64_step_a.json")


def traffic_from_profiles(bytes_per_launch):
    """HBM bytes per launch of the batched FP64 step A: the committed
    rocprofv3 counter ratio (counter bytes / algorithmic bytes over the
    counted launches) times this run's algorithmic bytes per launch, if the
    counters were taken on the current kernel source; else None."""
    if not os.path.exists(PMC_BATCH_FILE):
        return None
    try:
        d = json.load(open(PMC_BATCH_FILE))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash() or not d.get("counter_over_algorithmic"):
        return None
    return d["counter_over_algorithmic"] * bytes_per_launch


def forms_linear(pf, torch, inputs, timing_sample):
    """FP64 vs mixed precision on the 193^3 sphere Poisson problem."""
    import numpy as np
    prob = inputs.sphere_poisson(193)
    g = pf.grid_from_problem(prob)
    b = torch.as_tensor(prob.b, device="cuda")
    out = {}
    xs = {}
    for name, prec in (("fp64", pf.PF_FP64), ("mixed", pf.PF_MIXED)):
        x = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
        pf.pf_linear_solve(g, None, b, x, pf.pf_lin_opts_default(precision=prec))   # warm-up
        pf.pf_timing_enable(1, timing_sample)
        times = []
        for _ in range(3):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = pf.pf_linear_solve(g, None, b, x, pf.pf_lin_opts_default(precision=prec))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tm = pf.pf_timing_read(prec)
        pf.pf_timing_enable(0, 1)
        t = sorted(times)[1]
        rel = pf.pf_residual(g, None, b, x)
        xs[name] = x.cpu().numpy()
        elem = 8 if prec == pf.PF_FP64 else 4
        t_iter = t / info["iters"]      # whole solve (residuals, refinement, host checks included)
        out[name] = dict(seconds=t, iters=info["iters"], refinements=info["refinements"],
                         rel_res=rel, iters_per_s=info["iters"] / t, us_per_iter=t_iter * 1e6,
                         iter_frac_method_bytes=ITER_VECTORS_METHOD * prob.N * elem / t_iter / 1e9 / PEAK_HBM_GBS,
                         iter_frac_build_bytes=iter_bytes_build(elem) * prob.N / t_iter / 1e9 / PEAK_HBM_GBS,
                         step_a_mean_us=tm["mean_ms"] * 1e3,
                         step_a_gbs=(tm["bytes"] / tm["launches"] / (tm["mean_ms"] * 1e-3) / 1e9)
                         if tm["launches"] else None)
    d = xs["mixed"] - xs["fp64"]
    out["mixed_vs_fp64_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(xs["fp64"]))
    out["mixed_speedup"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    out["workload"] = "sphere_poisson 193^3 (7,189,057 unknowns), rel res 1e-10"
    return out


def forms_spmv_cold(pf, torch, inputs, n=193, sets=3, reps=10):
    """Isolated Jacobi-scaled stencil product M^-1 A x on the n^3 sphere
    problem, FP64 and FP32, cycling through `sets` independent grids and
    (x, y) pairs so that the 256 MB Infinity Cache cannot hold the operands
    between launches (each FP64 set reads and writes 3 vectors of 57.5 MB at
    193^3: x, eps in, y out).  Kernel time from HIP events around each
    launch."""
    prob = inputs.sphere_poisson(n)
    grids = [pf.grid_from_problem(prob) for _ in range(sets)]
    out = {"workload": f"sphere_poisson {n}^3, {sets} operand sets cycled, {reps} launches each"}
    for name, dt, fn, kind in (("fp64", torch.float64, pf.pf_spmv, pf.TIMING_SPMV_FP64),
                               ("fp32", torch.float32, pf.pf_spmv_f32, pf.TIMING_SPMV_FP32)):
        xs = [torch.randn(prob.N, dtype=dt, device="cuda") for _ in range(sets)]
        ys = [torch.empty(prob.N, dtype=dt, device="cuda") for _ in range(sets)]
        for i in range(sets):
            fn(grids[i], None, xs[i], ys[i], 1)   # untimed first launch per set
        pf.pf_timing_enable(1, 1)
        for _ in range(reps):
            for i in range(sets):
                fn(grids[i], None, xs[i], ys[i], 1)
        tm = pf.pf_timing_read(kind)
        pf.pf_timing_enable(0, 1)
        bpl = tm["bytes"] / max(1, tm["launches"])
        out[name] = dict(launches=tm["launches"], mean_us=tm["mean_ms"] * 1e3, bytes_per_launch=bpl,
                         gbs=bpl / (tm["mean_ms"] * 1e-3) / 1e9 if tm["mean_ms"] > 0 else None)
        out[name]["frac_of_8tbs"] = out[name]["gbs"] / PEAK_HBM_GBS if out[name]["gbs"] else None
    return out


class Batch:
    """The 64-system batch resident on the device: grids, right-hand sides,
    shifts and solution vectors."""

    def __init__(self, pf, torch, inputs):
        self.probs = inputs.batch_systems()
        self.grids = [pf.grid_from_problem(p) for p in self.probs]
        self.bs = [torch.as_tensor(p.b, device="cuda") for p in self.probs]
        self.sg = [torch.as_tensor(p.sigma, device="cuda") for p in self.probs]
        self.xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in self.probs]
        self.unknowns = sum(p.N for p in self.probs)

    def solve(self, pf, torch, prec, batched):
        for x in self.xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        opts = pf.pf_lin_opts_default(precision=prec)
        if batched:
            infos = pf.pf_linear_solve_batch(self.grids, self.sg, self.bs, self.xs, opts)
        else:
            infos = [pf.pf_linear_solve(g, s, b, x, opts) for g, s, b, x in zip(self.grids, self.sg, self.bs, self.xs)]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos

    def max_rel_res(self, pf):
        return max(pf.pf_residual(g, s, b, x) for g, s, b, x in zip(self.grids, self.sg, self.bs, self.xs))


def forms_batch(pf, torch, batch, value_s, reps=3):
    """Batched mixed precision (FP32 inner BiCGSTAB, FP64 refinement) and 64
    sequential FP64 solves on the headline batch, each to 1e-10; the median
    of `reps` runs after one untimed run.  The batched FP32 step A is timed
    as the headline's FP64 one."""
    res = {}
    for name, prec, batched in (("batched_mixed", pf.PF_MIXED, True), ("sequential_fp64", pf.PF_FP64, False)):
        batch.solve(pf, torch, prec, batched)          # first use: FP32 workspaces and tuning
        times = []
        if name == "batched_mixed":
            pf.pf_timing_enable(1, 4)
        for _ in range(reps):
            t, infos = batch.solve(pf, torch, prec, batched)
            times.append(t)
        row = dict(seconds=sorted(times)[len(times) // 2], total_iters=sum(i["iters"] for i in infos),
                   max_rel_res=batch.max_rel_res(pf), fp64_fallbacks=sum(i["fp64_fallback"] for i in infos))
        if name == "batched_mixed":
            tm = pf.pf_timing_read(pf.TIMING_BATCH_FP32)
            pf.pf_timing_enable(0, 1)
            row["step_a_fp32"] = dict(launches=tm["launches"], mean_us=tm["mean_ms"] * 1e3,
                                      gbs=tm["bytes"] / tm["launches"] / (tm["mean_ms"] * 1e-3) / 1e9
                                      if tm["launches"] else None)
        res[name] = row
    res["batched_fp64_seconds"] = value_s
    res["batched_fp64_speedup_vs_sequential"] = res["sequential_fp64"]["seconds"] / value_s
    res["batched_mixed_speedup_vs_sequential"] = res["sequential_fp64"]["seconds"] / res["batched_mixed"]["seconds"]
    res["batched_mixed_speedup_vs_batched_fp64"] = value_s / res["batched_mixed"]["seconds"]
    return res


def forms_ceiling(pf, torch, n=193 ** 3 + 1, reps=30):
    """The device's streaming ceiling from the library's probe kernel (FP64,
    three operand sets of n doubles cycled so that the Infinity Cache cannot
    hold them; 64- and 128-bit lane accesses)."""
    out = []
    for kind in (0, 1, 2):
        r, w = pf.STREAM_MIX[kind]
        sets = [[torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(r + w)] for _ in range(3)]
        for width in (8, 16):
            us = pf.pf_stream_probe(kind, width, sets, reps=reps)
            out.append(dict(reads=r, writes=w, bytes_per_access=width, mean_us=us,
                            tbs=(r + w) * n * 8 / us * 1e-6))
        del sets
        torch.cuda.empty_cache()
    return {"arrays_of_doubles": n, "runs": out, "best_tbs": max(x["tbs"] for x in out)}


def forms_pf97(pf, torch, inputs):
    """Configuration 2: the full PF nonlinear solve on the 97^3 membrane
    (outer 1e-8, BiCGSTAB 1e-10), FP64 and with mixed-precision linear
    solves.  Its ~100 MB working set stays in the 256 MB Infinity Cache, so
    the step-A rate is an effective (cache-resident) GB/s, not an HBM
    fraction."""
    prob = inputs.membrane_pore(97)
    g = pf.grid_from_problem(prob)
    out = {"workload": "membrane_pore 97^3 (912,673 nodes): full PF solve, outer 1e-8, BiCGSTAB 1e-10"}
    phis = {}
    for name, prec in (("fp64", pf.PF_FP64), ("mixed", pf.PF_MIXED)):
        prm = pf.params_for(prob, outer_tol=1e-8, lin={"rel_tol": 1e-10, "precision": prec})
        phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
        pf.pf_nonlinear_solve(g, prm, phi)              # tuning, workspaces
        phi.zero_()
        pf.pf_timing_enable(1, 16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = pf.pf_nonlinear_solve(g, prm, phi)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        tm = pf.pf_timing_read(prec)
        pf.pf_timing_enable(0, 1)
        phis[name] = phi
        out[name] = dict(seconds=sec, outer_iters=info["outer_iters"], lin_iters=info["total_lin_iters"],
                         step_a_mean_us=tm["mean_ms"] * 1e3,
                         step_a_effective_gbs_cache_resident=tm["bytes"] / tm["launches"] / (tm["mean_ms"] * 1e-3)
                         / 1e9 if tm["launches"] else None)
    out["mixed_vs_fp64_rel_l2"] = float(torch.linalg.vector_norm(phis["mixed"] - phis["fp64"])
                                        / torch.linalg.vector_norm(phis["fp64"]))
    out["mixed_speedup"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    return out


def forms_interface(pf, torch, inputs, n=97, reps=5):
    """Singular-charge decomposition (Sec. 3) on the n^3 membrane with its
    2000 charges: time of pf_interface_setup (Coulomb sums, Laplace solve on
    Omega_m, SMIB terms); the Coulomb kernel alone over every Omega_m node
    (potential and one derivative per point, FLOP count per pair below,
    against the FP64 vector peak); and the PF solve with the interface terms
    as the extra PF2 right-hand side instead of charges spread to nodes."""
    import dataclasses
    prob = dataclasses.replace(inputs.membrane_pore(n), fixed_charge=None)
    g = pf.grid_from_problem(prob)
    ch = torch.as_tensor(inputs.point_charges(prob), device="cuda")
    M = ch.shape[0]
    lam = inputs.lambda_length_A()
    em, es = inputs.TABLE1["eps_m"], inputs.TABLE1["eps_s"]
    b = torch.empty(prob.N, dtype=torch.float64, device="cuda")
    reg = torch.empty_like(b)
    pf.pf_interface_setup(g, ch, lam, em, es, b, reg)            # first call: tuning of the Laplace grid
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = pf.pf_interface_setup(g, ch, lam, em, es, b, reg)
    setup_s = time.perf_counter() - t0
    # Coulomb kernel over every Omega_m node, timed with events on its stream
    solute = np.flatnonzero(prob.node_type == inputs.SOLUTE)
    k, j, i = np.unravel_index(solute, prob.shape)
    pts = torch.as_tensor(np.column_stack([i, j, k]) * prob.h, device="cuda")
    dirs = torch.full((len(solute),), 1, dtype=torch.int8, device="cuda")
    out = torch.empty(len(solute), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    pf.pf_coulomb(pts, ch, 1.0, out, dirs=dirs, stream=st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        pf.pf_coulomb(pts, ch, 1.0, out, dirs=dirs, stream=st)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pairs = float(len(solute)) * M
    flops = COULOMB_FLOP_PER_PAIR * pairs
    # PF solve with the decomposition
    prm = pf.params_for(prob, outer_tol=1e-8, lin={"rel_tol": 1e-10}, rhs_extra=b)
    phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nl = pf.pf_nonlinear_solve(g, prm, phi)
    solve_s = time.perf_counter() - t0
    return {"workload": f"membrane_pore {n}^3, {M} charges, Omega_m = {len(solute)} nodes",
            "setup_seconds": setup_s, "laplace_iters": info["iters"],
            "coulomb_kernel": {"points": len(solute), "charges": M, "mean_us": ms * 1e3,
                               "pairs_per_s": pairs / (ms * 1e-3),
                               "tflops": flops / (ms * 1e-3) / 1e12,
                               "frac_of_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                               "flop_per_pair": COULOMB_FLOP_PER_PAIR},
            "pf_solve": {"seconds": solve_s, "outer_iters": nl["outer_iters"],
                         "lin_iters": nl["total_lin_iters"], "status": nl["status"]}}


def forms_tps(pf, torch, inputs, n=97, outer_tol=1e-3):
    """The five states of the exchange cycle on the n^3 membrane: atomic model
    of the eight sites (Eqs. (19)-(20)), filter-region fill, then the five PF
    solves one after another and as one batch.  The outer loop stops at the
    paper's ErrTol of Table 2 (1e-3 on the max-norm update): the occupied
    sites hold phi-hat values of 50-100 as Dirichlet data, and the relaxed
    fixed-point iteration approaches 1e-8 only after many thousands of outer
    iterations there.  BiCGSTAB to relative residual 1e-10."""
    states = inputs.tps_states(n)
    prm = pf.params_for(states[0]["problem"], outer_tol=outer_tol, lin={"rel_tol": 1e-10})
    grids, site_rows = [], []
    t0 = time.perf_counter()
    for st in states:
        prob, s = st["problem"], st["sites"]
        sites = pf.Sites(s["xyz"], s["radius"], s["valence"], s["occupied"],
                         torch.as_tensor(st["atoms"], device="cuda"), s["eps_p"], s["eps_b"], s["V_sites"])
        phi_b, S_b, psi_b, _ = pf.pf_site_model(prm, sites)
        typ = torch.as_tensor(prob.node_type, device="cuda")
        fv = torch.as_tensor(prob.fixed_value, device="cuda")
        marked = pf.pf_site_fill(prob.nx, prob.ny, prob.nz, prob.h, sites, phi_b, typ, fv)
        grids.append(pf.pf_grid_create(prob.nx, prob.ny, prob.nz, prob.h, torch.as_tensor(prob.eps, device="cuda"),
                                       typ, torch.as_tensor(prob.fixed_charge, device="cuda"), fv,
                                       prob.bc_phi, prob.bc_value, prob.bc_psi))
        site_rows.append(dict(state=st["name"], facing=st["facing"], filter_nodes=marked,
                              psi_b=dict(zip(inputs.SITE_NAMES, np.round(psi_b, 4).tolist()))))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    res = dict(workload=f"membrane_pore {n}^3, 5 states x 8 sites", outer_tol=outer_tol, setup_seconds=setup_s,
               sites=site_rows)
    prm_mixed = pf.params_for(states[0]["problem"], outer_tol=outer_tol,
                              lin={"rel_tol": 1e-10, "precision": pf.PF_MIXED})
    for name, batched, p in (("sequential", False, prm), ("batched", True, prm), ("batched_mixed", True, prm_mixed)):
        phis = [torch.zeros(n ** 3, dtype=torch.float64, device="cuda") for _ in states]
        if name == "batched_mixed":   # first use of the FP32 workspaces (tuning) outside the timing
            pf.pf_nonlinear_solve(grids[0], p, phis[0])
            phis[0].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if batched:
            infos = pf.pf_nonlinear_solve_batch(grids, [p] * len(grids), phis)
        else:
            infos = [pf.pf_nonlinear_solve(g, p, x) for g, x in zip(grids, phis)]
        torch.cuda.synchronize()
        res[name] = dict(seconds=time.perf_counter() - t0, outer_iters=[i["outer_iters"] for i in infos],
                         status=[i["status"] for i in infos])
    res["batched_speedup"] = res["sequential"]["seconds"] / res["batched"]["seconds"]
    res["batched_mixed_speedup"] = res["sequential"]["seconds"] / res["batched_mixed"]["seconds"]
    return res


def forms_loop_settings(pf, torch, inputs, n=49):
    """Outer-loop settings on the n^3 membrane: relaxation weight omega and
    outer tolerance ErrTol swept with BiCGSTAB to relative residual 1e-10,
    plus the paper's own settings (Table 2: omega 0.3, ErrTol 1e-3; Table 3:
    absolute max-norm residual 1e-6 for every linear solve)."""
    prob = inputs.membrane_pore(n)
    g = pf.grid_from_problem(prob)
    runs = []
    cases = [(w, t, pf.PF_STOP_REL2, 1e-10) for t in (1e-3, 1e-8) for w in (0.1, 0.3, 0.5, 0.7)]
    cases.append((0.3, 1e-3, pf.PF_STOP_ABS_INF, 1e-6))
    for omega, tol, rule, ltol in cases:
        prm = pf.params_for(prob, omega=omega, outer_tol=tol, max_outer=20000,
                            lin={"rel_tol": ltol, "stop_rule": rule})
        phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = pf.pf_nonlinear_solve(g, prm, phi, check=False)
        torch.cuda.synchronize()
        runs.append(dict(omega=omega, outer_tol=tol, linear_stop="abs_inf" if rule else "rel2", linear_tol=ltol,
                         seconds=time.perf_counter() - t0, outer_iters=info["outer_iters"],
                         lin_iters=info["total_lin_iters"], status=info["status"]))
    return dict(workload=f"membrane_pore {n}^3", runs=runs)


BIAS_MODES = ("batched_mixed", "sequential_fp64")


def forms_bias_sweep(pf, torch, inputs, n=129, chunk=400, outer_cap=0, modes=BIAS_MODES, members=None):
    """Configuration 5: 16 bias voltages on the membrane workload, full PF
    nonlinear solves, batched (shared launches, mixed-precision linear
    solves) vs 16 sequential FP64 solves.  Each run is driven in chunks of
    `chunk` outer iterations (warm-started from the last iterate; the PF1
    initial guess restarts from zero) so that progress is printed.
    outer_cap > 0 stops every bias after that many outer iterations (equal
    work in both modes: a throughput comparison instead of time to
    convergence).  modes and members (indices into the 16 biases) select
    part of the sweep, for runs split over several invocations."""
    vt = inputs.thermal_voltage_mV()
    sweep = inputs.bias_sweep_mV()
    members = list(range(len(sweep))) if members is None else list(members)
    probs = [inputs.membrane_pore(n, bias_phi=sweep[m] / vt) for m in members]
    grids = [pf.grid_from_problem(p) for p in probs]
    res = {"members": members, "bias_mV": [sweep[m] for m in members]}
    for name, prec, batched in (("batched_mixed", pf.PF_MIXED, True), ("sequential_fp64", pf.PF_FP64, False)):
        if name not in modes:
            continue
        step = min(chunk, outer_cap) if outer_cap else chunk
        prms = [pf.params_for(p, outer_tol=1e-8, max_outer=step, lin={"rel_tol": 1e-10, "precision": prec})
                for p in probs]
        phis = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in probs]
        outer = [0] * len(probs)
        lin = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        groups = [list(range(len(probs)))] if batched else [[i] for i in range(len(probs))]
        for grp in groups:
            todo = list(grp)
            while todo:
                if len(todo) > 1 or batched:
                    infos = pf.pf_nonlinear_solve_batch([grids[i] for i in todo], [prms[i] for i in todo],
                                                        [phis[i] for i in todo], check=False)
                else:
                    infos = [pf.pf_nonlinear_solve(grids[todo[0]], prms[todo[0]], phis[todo[0]], check=False)]
                nxt = []
                for i, info in zip(todo, infos):
                    outer[i] += info["outer_iters"]
                    lin += info["total_lin_iters"]
                    prms[i].c.warm_start = 1
                    cap = outer_cap if outer_cap else 20000
                    if info["status"] == pf.PF_ERR_NOCONV and outer[i] < cap:
                        nxt.append(i)
                    elif info["status"] == pf.PF_ERR_NOCONV and outer_cap:
                        pass   # stopped at the cap on purpose
                    elif info["status"] != 0:
                        raise RuntimeError(f"bias {i}: status {info['status']}")
                todo = nxt
                log(f"[bench]   {name}: {len(todo)} of {len(grp)} still running, "
                    f"{time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        res[name] = dict(seconds=time.perf_counter() - t0, outer_iters=outer, total_lin_iters=lin,
                         converged=not outer_cap)
        log(f"[bench] bias sweep {name}: {res[name]['seconds']:.1f} s")
    if all(m in res for m in BIAS_MODES):
        res["speedup"] = res["sequential_fp64"]["seconds"] / res["batched_mixed"]["seconds"]
    res["workload"] = (f"membrane_pore {n}^3, {len(members)} of the 16 biases -150..+150 mV on -z, outer 1e-8, "
                       "BiCGSTAB 1e-10"
                       + (f", every bias stopped after {outer_cap} outer iterations" if outer_cap else ", converged"))
    return res


def trace_summary(paths, top=12):
    """Busy and idle time of the GPU from rocprofv3 kernel (and memory-copy)
    trace CSVs: the union of activity intervals, the idle gaps between
    consecutive activities by size and by the pair of activities around them,
    and the busy time per kernel."""
    import csv
    import re
    from collections import Counter

    def short(name):
        name = name.replace("void ", "")
        m = re.match(r"(pfk::\w+)(<[^>]*>)?", name)
        return (m.group(1) + (m.group(2) or "")) if m else name[:40]

    ev = []
    for path in paths:
        for r in csv.DictReader(open(path)):
            nm = r.get("Kernel_Name") or ("copy " + r.get("Direction", "?"))
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(nm)))
    ev.sort()
    if not ev:
        return {}
    busy, end, prev = 0, ev[0][0], "start"
    gaps, gapn, kern, kn, hist = Counter(), Counter(), Counter(), Counter(), Counter()
    durs = {}
    for s0, e0, nm in ev:
        kern[nm] += e0 - s0
        kn[nm] += 1
        durs.setdefault(nm, []).append(e0 - s0)
        if s0 > end:
            g = s0 - end
            gaps[f"{prev} -> {nm}"] += g
            gapn[f"{prev} -> {nm}"] += 1
            b = 1
            while b * 2 <= g / 1000:
                b *= 2
            hist[b] += g
        busy += max(0, e0 - max(s0, end))
        if e0 > end:
            end, prev = e0, nm
    span = ev[-1][1] - ev[0][0]
    return {"events": len(ev), "span_s": span * 1e-9, "busy_s": busy * 1e-9, "idle_s": (span - busy) * 1e-9,
            "idle_by_gap_us_at_least": {str(b): v * 1e-9 for b, v in sorted(hist.items())},
            "top_gaps": [{"pair": k, "seconds": v * 1e-9, "count": gapn[k], "mean_us": v / gapn[k] * 1e-3}
                         for k, v in gaps.most_common(top)],
            "busy_by_kernel": [dict({"kernel": k, "seconds": v * 1e-9, "count": kn[k], "mean_us": v / kn[k] * 1e-3},
                                    **_full_launches(durs[k])) for k, v in kern.most_common(top)]}


def _full_launches(d):
    """Mean duration of the launches that did their work: those of at least a
    quarter of the median (BiCGSTAB launches queued after convergence exit
    at once and take a few percent of a full one)."""
    d = sorted(d)
    cut = 0.25 * d[len(d) // 2]
    full = [x for x in d if x >= cut]
    return {"count_full": len(full), "mean_us_full": sum(full) / len(full) * 1e-3}


def copy_ceiling(torch):
    """Achievable device bandwidth of this part for plain streaming kernels
    (torch's own elementwise kernels, FP64): a copy (1 read, 1 write) and a
    three-operand product (3 reads, 1 write) per buffer size, timed with
    events over 20 launches after 3 warm-up launches; the smaller sizes stay
    in the Infinity Cache between launches."""
    out = []
    for mib in (32, 96, 512, 2048):
        n = mib * (1 << 20) // 8
        a = torch.rand(n, dtype=torch.float64, device="cuda")
        b, c, d = torch.rand_like(a), torch.rand_like(a), torch.empty_like(a)
        row = {"mib_per_buffer": mib}
        for name, fn, nbuf in (("copy", lambda: d.copy_(a), 2), ("addcmul", lambda: torch.addcmul(a, b, c, out=d), 4)):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn()
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / 20
            row[name + "_tbs"] = nbuf * n * 8 / sec / 1e12
        out.append(row)
        del a, b, c, d
    torch.cuda.empty_cache()
    return out


def copy_reference(torch, mib=512):
    """A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE give the
    counters' scale (bytes per reported KiB) for the traffic figure."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return n * 8


PMC_BATCH_KERNEL = "k_zmarch_batch<3, double, false, 2, true"   # batched step A, FP64, shift per class


def _counter_rows(path, counter):
    """Counter values (bytes) per kernel name, in dispatch order."""
    import csv
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals.setdefault(r["Kernel_Name"], []).append((int(r.get("Dispatch_Id") or 0),
                                                          float(r["Counter_Value"]) * 1024.0))
    return {k: [v for _, v in sorted(xs, key=lambda t: t[0])] for k, xs in vals.items()}


# The 193^3 Poisson steps in the pinned launch shapes (SHAPE_193) and their
# algorithmic bytes per node (palette form, no shift): step A reads s^, p^,
# v^, t^, x, the palette byte and the FP32 shadow and writes x, r^, p^, v^;
# step B reads r^, v^, the palette byte and the shadow and writes s^, t^.
PMC_193_KERNELS = {
    "step_a_fp64": ("k_zmarch<3, double, false, 0, true, 512, 1, false, 1>", 9 * 8 + 1 + 4),
    "step_b_fp64": ("k_zmarch<4, double, false, 0, true, 512, 1, false, 1>", 4 * 8 + 1 + 4),
    "step_a_fp32": ("k_zmarch<3, float, false, 0, true, 1024, 2, false, 1>", 9 * 4 + 1 + 4),
    "step_b_fp32": ("k_zmarch<4, float, false, 0, true, 1024, 2, false, 1>", 4 * 4 + 1 + 4),
}


def pmc_summary_193(fetch_csv, write_csv, copy_bytes, n=193):
    """Counter traffic of the 193^3 BiCGSTAB steps from two rocprofv3 --pmc
    runs of `bench.py --linear193-only 1 --copy-ref 1`: per kernel, the
    dispatches that did a whole step (those queued after convergence exit at
    once and fetch almost nothing: counted are the ones fetching at least a
    fifth of the algorithmic bytes, the same dispatches in both runs), the
    counters scaled by their reading on the copy kernel of known size, and
    their ratio to the algorithmic bytes."""
    N = n ** 3
    rows = {c: _counter_rows(p, c) for c, p in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv))}
    scale = {}
    for c, r in rows.items():
        copy = [x for k, xs in r.items() if "copy" in k.lower() for x in xs]
        scale[c] = copy_bytes / max(copy) if copy else None
    out = {"workload": f"sphere_poisson_{n}", "source_hash": kernel_source_hash(), "copy_bytes": copy_bytes,
           "FETCH_SIZE_scale": scale["FETCH_SIZE"], "WRITE_SIZE_scale": scale["WRITE_SIZE"], "kernels": {}}
    if not all(scale.values()):
        return out
    for key, (name, per_node) in PMC_193_KERNELS.items():
        alg = per_node * N
        f = [x * scale["FETCH_SIZE"] for k, xs in rows["FETCH_SIZE"].items() if name in k for x in xs]
        w = [x * scale["WRITE_SIZE"] for k, xs in rows["WRITE_SIZE"].items() if name in k for x in xs]
        e = {"kernel": name, "algorithmic_bytes": alg, "dispatches": len(f), "runs_aligned": len(f) == len(w)}
        if f and len(f) == len(w):
            full = [i for i, x in enumerate(f) if x >= 0.2 * alg]
            e["dispatches_counted"] = len(full)
            if full:
                e["FETCH_SIZE"] = sum(f[i] for i in full) / len(full)
                e["WRITE_SIZE"] = sum(w[i] for i in full) / len(full)
                e["counter_bytes"] = e["FETCH_SIZE"] + e["WRITE_SIZE"]
                e["counter_over_algorithmic"] = e["counter_bytes"] / alg
        out["kernels"][key] = e
    return out


def pmc_summary_batch(fetch_csv, write_csv, copy_bytes, fetch_log, write_log):
    """Counter traffic of the batched FP64 step A from two rocprofv3 --pmc
    runs (CSV) of `bench.py --pmc-run 1`: FETCH_SIZE and WRITE_SIZE summed
    over every dispatch of that kernel (the run times every chunk, so each
    dispatch is also in the algorithmic count the run printed to its log),
    each counter scaled by its reading on the copy kernel of known size and
    divided by its own run's algorithmic bytes (the two runs can differ by a
    chunk: the true-residual checks between Krylov runs use autotuned shapes,
    whose reduction order decides a restart near the tolerance)."""
    def alg_of(path):
        alg = None
        for line in open(path):
            if line.startswith("{") and "pmc_run" in line:
                alg = json.loads(line)["pmc_run"]
        return alg

    out = {"kernel": PMC_BATCH_KERNEL, "source_hash": kernel_source_hash(), "copy_bytes": copy_bytes}
    ratio = {}
    for counter, path, log_path in (("FETCH_SIZE", fetch_csv, fetch_log), ("WRITE_SIZE", write_csv, write_log)):
        alg = alg_of(log_path)
        rows = _counter_rows(path, counter)
        copy = [x for k, xs in rows.items() if "copy" in k.lower() for x in xs]
        scale = copy_bytes / max(copy) if copy else None
        mine = [x for k, xs in rows.items() if PMC_BATCH_KERNEL in k for x in xs]
        out[counter + "_run"] = alg
        out[counter + "_dispatches"] = len(mine)
        out[counter + "_scale"] = scale
        if mine and scale and alg and alg["launches_timed"] == len(mine) and alg["bytes_timed"] > 0:
            out[counter + "_bytes_per_launch"] = sum(mine) * scale / len(mine)
            ratio[counter] = sum(mine) * scale / alg["bytes_timed"]
    if len(ratio) == 2:
        out["counter_over_algorithmic"] = ratio["FETCH_SIZE"] + ratio["WRITE_SIZE"]
    return out


# Step-A launch shapes the autotuner picks for the 193^3 grid in an
# uninstrumented run (threads, points per strip, z-planes, pipeline depth):
# counters serialise the launches and distort the tuner's timings, so the
# profiling mode pins these for both steps instead of tuning.
SHAPE_193 = {"fp64": (512, 512, 32, 1), "fp32": (1024, 2048, 16, 1)}


def linear193_only(pf, torch, inputs):
    """The 193^3 sphere Poisson solves alone, FP64 then mixed, once each with
    the launch shape pinned (SHAPE_193), so that two profiler runs launch the
    same kernels in the same order; for kernel traces and counters."""
    p = inputs.sphere_poisson(193)
    b = torch.as_tensor(p.b, device="cuda")
    res = []
    for prec, key in ((pf.PF_FP64, "fp64"), (pf.PF_MIXED, "fp32")):
        nt, strip, kz, depth = SHAPE_193[key]
        pf.pf_set_launch(strip, kz, nt, depth)
        g = pf.grid_from_problem(p)
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        info = pf.pf_linear_solve(g, None, b, x, pf.pf_lin_opts_default(precision=prec))
        res.append({k: info[k] for k in ("iters", "refinements", "rel_res")})
        del g
    pf.pf_set_launch(0, 0, 0, 0)
    return res


CPU_SAMPLE_SIZES = (33, 65, 97, 129)   # one member of each of these sizes


def _cpu_sample_job(indices):
    """Child process body: the oracle's solves of the listed batch members,
    pinned to core 0; prints one JSON line per member."""
    os.sched_setaffinity(0, {0})
    import oracle
    from paper_1711_04060_amd import inputs
    probs = inputs.batch_systems()
    for i in indices:
        p = probs[i]
        t0 = time.perf_counter()
        _, info = oracle.linear_solve(p, p.sigma, p.b, tol=1e-10)
        print(json.dumps(dict(member=i, n=p.nx, N=p.N, iters=info["iters"], seconds=time.perf_counter() - t0)),
              flush=True)


def cpu_baseline(batch, infos_fp64):
    """The serial FP64 oracle (Table 3 BiCGSTAB on the seven-diagonal matrix)
    on one member of each size in CPU_SAMPLE_SIZES, in a child process pinned
    to one core, extrapolated to the whole batch by node-iterations (the GPU
    FP64 run's iteration count of every member times its size)."""
    import subprocess
    sizes = {}
    for i, p in enumerate(batch.probs):
        sizes.setdefault(p.nx, i)
    pick = [sizes[n] for n in CPU_SAMPLE_SIZES if n in sizes]
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample-job", ",".join(map(str, pick))]
    out = subprocess.run(cmd, capture_output=True, text=True, check=True).stdout
    rows = [json.loads(line) for line in out.splitlines() if line.startswith("{")]
    t = sum(r["seconds"] for r in rows)
    node_iters = sum(r["iters"] * r["N"] for r in rows)
    total_node_iters = sum(info["iters"] * p.N for info, p in zip(infos_fp64, batch.probs))
    model, nproc = "unknown", os.cpu_count()
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except (OSError, ValueError):
        pass
    return dict(value=t / node_iters * total_node_iters, unit="s", cores=1, kind="oracle",
                sample=(f"serial FP64 oracle (BiCGSTAB of Table 3 on the seven-diagonal matrix), pinned to core 0, "
                        f"on members of sizes {[r['n'] for r in rows]}: {t:.1f} s for "
                        f"{node_iters / 1e6:.1f} M node-iterations, extrapolated to the batch's "
                        f"{total_node_iters / 1e9:.2f} G node-iterations"),
                extrapolated=True, cpu_model=model, nproc=nproc, pinned="core 0 (sched_setaffinity)",
                members=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sample", type=int, default=1,
                    help="time step A in one chunk of iterations out of this many (1: every launch of the timed "
                         "steps, the set a profiler's mean over them covers)")
    ap.add_argument("--forms", type=int, default=1)
    ap.add_argument("--cpu", type=int, default=1)
    ap.add_argument("--bias-outer", type=int, default=100,
                    help="configuration 5: stop every bias after this many outer iterations (0: converge)")
    ap.add_argument("--bias-sweep", type=int, default=1, help="run configuration 5 (16 biases, 129^3)")
    ap.add_argument("--bias-n", type=int, default=129)
    ap.add_argument("--bias-modes", type=str, default=",".join(BIAS_MODES),
                    help="bias sweep modes to run (comma list of batched_mixed, sequential_fp64)")
    ap.add_argument("--bias-members", type=str, default="",
                    help="first:last (exclusive) of the 16 biases; default all")
    ap.add_argument("--tps", type=int, default=0, help="also run the five exchange-cycle states at 97^3")
    ap.add_argument("--loop-settings", type=int, default=0, help="also sweep omega and ErrTol at 49^3")
    ap.add_argument("--copy-ref", type=int, default=0, help="run the copy reference kernel (counter scale)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "FETCH_LOG", "WRITE_LOG"),
                    help="summarise the rocprofv3 --pmc CSVs of two --pmc-run invocations (and the algorithmic "
                         "bytes each printed) into the traffic file and exit")
    ap.add_argument("--pmc-run", type=int, default=0,
                    help="counter run: the headline steps only, every chunk timed (--sample 1), and the "
                         "algorithmic bytes of the timed launches printed (run it with PF_BATCH_POLICY set "
                         "to the policy an uninstrumented run keeps, and --warmup 0)")
    ap.add_argument("--trace-summary", nargs="+", metavar="CSV",
                    help="summarise rocprofv3 kernel / memory-copy trace CSVs (busy, idle gaps) and exit")
    ap.add_argument("--copy-ceiling", type=int, default=0,
                    help="measure plain streaming bandwidth (copy, 3-operand product) at several sizes and exit")
    ap.add_argument("--pin-shape", type=str, default="",
                    help="threads,strip,zplanes,depth: launch shape of every stencil kernel instead of the "
                         "autotuner's (for counter runs, whose serialised launches distort the tuner)")
    ap.add_argument("--pmc-summary-193", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs of --linear193-only 1 --copy-ref 1 and exit")
    ap.add_argument("--spmv-only", type=int, default=0,
                    help="run only the isolated cold 193^3 product (for counters) and exit")
    ap.add_argument("--linear193-only", type=int, default=0,
                    help="run only the 193^3 FP64 and mixed linear solves (for traces and counters) and exit")
    ap.add_argument("--cpu-sample-job", type=str, default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_sample_job:
        _cpu_sample_job([int(v) for v in args.cpu_sample_job.split(",")])
        return
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary), indent=1))
        return
    if args.pmc_summary:
        f_csv, w_csv, f_log, w_log = args.pmc_summary
        print(json.dumps(pmc_summary_batch(f_csv, w_csv, 512 * (1 << 20), f_log, w_log), indent=1))
        return
    if args.pmc_summary_193:
        print(json.dumps(pmc_summary_193(args.pmc_summary_193[0], args.pmc_summary_193[1], 512 * (1 << 20)),
                         indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path "
              "is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_04060_amd import inputs, pf
    pf.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.copy_ceiling:
        print(json.dumps({"copy_ceiling": copy_ceiling(torch)}), flush=True)
        return
    if args.copy_ref:
        copy_reference(torch)
    if args.pin_shape:
        nt, strip, kz, depth = (int(v) for v in args.pin_shape.split(","))
        pf.pf_set_launch(strip, kz, nt, depth)
    if args.linear193_only:
        print(json.dumps({"linear_193": linear193_only(pf, torch, inputs)}), flush=True)
        return
    if args.spmv_only:
        print(json.dumps({"spmv_cold_193": forms_spmv_cold(pf, torch, inputs)}), flush=True)
        return
    if args.pmc_run:
        args.sample, args.forms, args.cpu, args.bias_sweep = 1, 0, 0, 0

    batch = Batch(pf, torch, inputs)
    log(f"[bench] workload batch_64: {len(batch.probs)} systems, {batch.unknowns} unknowns, "
        f"warmup {args.warmup}, steps {args.steps}")
    for w in range(args.warmup):
        t, infos = batch.solve(pf, torch, pf.PF_FP64, True)
        log(f"[bench] warmup {w}: {t:.3f} s, {sum(i['iters'] for i in infos)} iterations")
    pf.pf_timing_enable(1, args.sample)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        t, infos = batch.solve(pf, torch, pf.PF_FP64, True)
        log(f"[bench] step {s_}: {t:.3f} s, {sum(i['iters'] for i in infos)} iterations, "
            f"max rel res {max(i['rel_res'] for i in infos):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = pf.pf_timing_read(pf.TIMING_BATCH_FP64)
    pf.pf_timing_enable(0, 1)
    sec_per_step = elapsed / args.steps
    total_iters = sum(i["iters"] for i in infos)
    node_iters = sum(i["iters"] * p.N for i, p in zip(infos, batch.probs))
    bpl = tm["bytes"] / tm["launches"] if tm["launches"] else 0.0
    achieved = bpl / (tm["mean_ms"] * 1e-3) / 1e9 if tm["launches"] else 0.0
    if args.pmc_run:
        print(json.dumps({"pmc_run": {"launches_timed": tm["launches"], "bytes_timed": tm["bytes"],
                                      "mean_us": tm["mean_ms"] * 1e3}}), flush=True)
        return
    max_res = batch.max_rel_res(pf)
    traffic = traffic_from_profiles(bpl)
    result = {
        "metric": METRIC,
        "value": sec_per_step,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"batch_64: 64 linearised-PB systems 33^3..129^3 ({batch.unknowns:,} unknowns), each "
                         "Jacobi-BiCGSTAB FP64 from x = 0 to true rel. residual 1e-10, batched (one launch per "
                         "step kernel per iteration over all iterating members)"),
            "members": len(batch.probs),
            "unknowns": batch.unknowns,
            "bicgstab_iters_total": total_iters,
            "bicgstab_iters_max_member": max(i["iters"] for i in infos),
            "node_iters_per_s": node_iters / sec_per_step,
            "bicgstab_iters_per_s": total_iters / sec_per_step,
            "max_true_rel_res": max_res,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("batched BiCGSTAB step A, FP64, palette form with the shift per class (previous x, "
                       "r^ update + p^ update + v^ = D^-1 A p^ + 2 dots over every iterating member)"),
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "traffic_gbs": traffic / (tm["mean_ms"] * 1e-3) / 1e9 if (traffic and tm["launches"]) else None,
            "launches_timed": tm["launches"],
            "mean_us": tm["mean_ms"] * 1e3,
            "bytes_per_launch": bpl,
            "bytes_rule": ("77 B per node of every member still iterating at that launch: s^, p^, v^, t^, x "
                           "(8 B each) read, 1-byte coefficient palette index (it also selects the shift from "
                           "the member's per-class table), 4-byte shadow; x, r^, p^, v^ written"),
        },
    }
    if args.forms:
        log("[bench] forms: batch_64 mixed and sequential")
        result["forms"] = {"batch_64": forms_batch(pf, torch, batch, sec_per_step)}
        log("[bench] forms: streaming ceiling")
        result["forms"]["ceiling"] = forms_ceiling(pf, torch)
        log("[bench] forms: 193^3 FP64 vs mixed")
        result["forms"]["linear_193"] = forms_linear(pf, torch, inputs, args.sample)
        log("[bench] forms: isolated cold stencil product at 193^3")
        result["forms"]["spmv_cold_193"] = forms_spmv_cold(pf, torch, inputs)
        log("[bench] forms: 97^3 PF solve")
        result["forms"]["pf_97"] = forms_pf97(pf, torch, inputs)
        log("[bench] forms: singular-charge decomposition at 97^3")
        result["forms"]["interface_97"] = forms_interface(pf, torch, inputs)
    if args.bias_sweep:
        log(f"[bench] forms: 16-bias sweep at {args.bias_n}^3")
        sel = [int(v) for v in args.bias_members.split(":")] if args.bias_members else None
        result.setdefault("forms", {})["bias_sweep"] = forms_bias_sweep(
            pf, torch, inputs, n=args.bias_n, outer_cap=args.bias_outer,
            modes=tuple(args.bias_modes.split(",")), members=range(sel[0], sel[1]) if sel else None)
    if args.loop_settings:
        log("[bench] forms: outer-loop settings at 49^3")
        result.setdefault("forms", {})["loop_settings_49"] = forms_loop_settings(pf, torch, inputs)
    if args.tps:
        log("[bench] forms: five exchange-cycle states at 97^3")
        result.setdefault("forms", {})["tps_97"] = forms_tps(pf, torch, inputs)
    if args.cpu:
        log("[bench] cpu baseline (oracle sample)")
        result["cpu_baseline"] = cpu_baseline(batch, infos)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
