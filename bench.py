#!/usr/bin/env python
"""Benchmark of the Poisson-Fermi hot path on one MI355X.

A step is one full nonlinear Poisson-Fermi solve (Sec. 4, Tables 2 and 4) of
the 97^3 membrane workload from phi = 0: initial PF2 solve, then Fermi update,
PF1 solve, PF2 solve and relaxation until the max-norm update is below 1e-8,
every linear solve Jacobi-BiCGSTAB to relative residual 1e-10.  All inputs are
resident in device memory before the timed region starts.

The JSON line also carries:
  roofline      the BiCGSTAB step-A stencil kernel (the previous iteration's
                x, r update, the p update and v = A M^-1 p in one pass),
                timed with HIP events on the library's stream during the
                timed steps; algorithmic bytes = 12 vectors of N doubles per
                launch (reads s, t, x, p, v, shadow, dinv, eps; writes x, r,
                p, v);
  cpu_baseline  the serial FP64 oracle on a bounded sample of the same solve
                (its first outer iterations), scaled to a whole solve by the
                number of BiCGSTAB iterations the solve needs;
  forms         FP64 vs mixed precision on the 193^3 Poisson problem and the
                64-system batch, each to relative residual 1e-10; the isolated
                Jacobi-scaled stencil product at 193^3 with operands cycled
                through three sets (cold in the Infinity Cache).
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
STEP_A_VECTORS = 12.0   # N-vectors step A reads and writes
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


def traffic_from_profiles(workload):
    """HBM bytes per step-A launch from committed rocprofv3 PMC summaries, if
    they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_bicg_step_a.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash() or d.get("workload") != workload:
        return None
    return d.get("hbm_bytes_per_launch")


def run_nonlinear(pf, torch, prob, prm):
    phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
    info = pf.pf_nonlinear_solve(g_cache[prob.name], prm, phi, check=prm.c.max_outer >= 5000)
    return info, phi


g_cache = {}


def forms_pf_mixed(pf, torch, prob, phi64):
    """The benchmark's own 97^3 PF solve with every linear solve in mixed
    precision (FP32 BiCGSTAB inside FP64 refinement to the same 1e-10 true
    relative residual), against the FP64 solve's potential phi64."""
    prm = pf.params_for(prob, outer_tol=1e-8, lin={"rel_tol": 1e-10, "precision": pf.PF_MIXED})
    phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
    g = g_cache[prob.name]
    pf.pf_nonlinear_solve(g, prm, phi)             # first use of the FP32 workspace: tuning
    phi.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = pf.pf_nonlinear_solve(g, prm, phi)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    rel = float(torch.linalg.vector_norm(phi - phi64) / torch.linalg.vector_norm(phi64))
    return dict(seconds=sec, outer_iters=info["outer_iters"], lin_iters=info["total_lin_iters"],
                rel_l2_vs_fp64=rel)


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
        bpl = STEP_A_VECTORS * prob.N * (8 if prec == pf.PF_FP64 else 4)
        out[name] = dict(seconds=t, iters=info["iters"], refinements=info["refinements"],
                         rel_res=rel, iters_per_s=info["iters"] / t,
                         step_a_mean_us=tm["mean_ms"] * 1e3,
                         step_a_gbs=(bpl / (tm["mean_ms"] * 1e-3) / 1e9) if tm["launches"] else None)
    d = xs["mixed"] - xs["fp64"]
    out["mixed_vs_fp64_rel_l2"] = float(np.linalg.norm(d) / np.linalg.norm(xs["fp64"]))
    out["mixed_speedup"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    out["workload"] = "sphere_poisson 193^3 (7,189,057 unknowns), rel res 1e-10"
    return out


def forms_spmv_cold(pf, torch, inputs, n=193, sets=3, reps=10):
    """Isolated Jacobi-scaled stencil product A M^-1 x on the n^3 sphere
    problem, FP64 and FP32, cycling through `sets` independent grids and
    (x, y) pairs so that the 256 MB Infinity Cache cannot hold the operands
    between launches (each FP64 set reads and writes 4 vectors of 57.5 MB at
    193^3).  Kernel time from HIP events around each launch."""
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


def forms_batch(pf, torch, inputs):
    """64 linearised-PB systems (33^3..129^3), each to rel. res. 1e-10:
    sequential FP64 solves vs one batched launch sequence (FP64 and mixed)."""
    probs = inputs.batch_systems()
    grids = [pf.grid_from_problem(p) for p in probs]
    bs = [torch.as_tensor(p.b, device="cuda") for p in probs]
    sg = [torch.as_tensor(p.sigma, device="cuda") for p in probs]
    xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in probs]
    res = {}
    for name, prec, batched in (("sequential_fp64", pf.PF_FP64, False), ("batched_fp64", pf.PF_FP64, True),
                                ("batched_mixed", pf.PF_MIXED, True)):
        opts = pf.pf_lin_opts_default(precision=prec)
        times = []
        for rep in range(2):                       # first pass: tuning, workspaces
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if batched:
                infos = pf.pf_linear_solve_batch(grids, sg, bs, xs, opts)
            else:
                infos = [pf.pf_linear_solve(gr, s, b, x, opts) for gr, s, b, x in zip(grids, sg, bs, xs)]
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        res[name] = dict(seconds=times[-1], total_iters=sum(i["iters"] for i in infos),
                         max_rel_res=max(pf.pf_residual(gr, s, b, x) for gr, s, b, x in zip(grids, sg, bs, xs)))
    res["unknowns"] = sum(p.N for p in probs)
    res["batched_fp64_speedup"] = res["sequential_fp64"]["seconds"] / res["batched_fp64"]["seconds"]
    res["batched_mixed_speedup"] = res["sequential_fp64"]["seconds"] / res["batched_mixed"]["seconds"]
    return res


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


def forms_bias_sweep(pf, torch, inputs, n=129, chunk=400, outer_cap=0):
    """Configuration 5: 16 bias voltages on the membrane workload, full PF
    nonlinear solves, batched (shared launches, mixed-precision linear
    solves) vs 16 sequential FP64 solves.  Each run is driven in chunks of
    `chunk` outer iterations (warm-started from the last iterate, which is the
    whole state of the outer loop) so that progress is printed.  outer_cap > 0
    stops every bias after that many outer iterations (equal work in both
    modes: a throughput comparison instead of time to convergence)."""
    vt = inputs.thermal_voltage_mV()
    probs = [inputs.membrane_pore(n, bias_phi=v / vt) for v in inputs.bias_sweep_mV()]
    grids = [pf.grid_from_problem(p) for p in probs]
    res = {}
    for name, prec, batched in (("batched_mixed", pf.PF_MIXED, True), ("sequential_fp64", pf.PF_FP64, False)):
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
        res[name] = dict(seconds=time.perf_counter() - t0, outer_iters=outer, total_lin_iters=lin)
        log(f"[bench] bias sweep {name}: {res[name]['seconds']:.1f} s")
    res["speedup"] = res["sequential_fp64"]["seconds"] / res["batched_mixed"]["seconds"]
    res["workload"] = (f"membrane_pore {n}^3, 16 biases -150..+150 mV on -z, outer 1e-8, BiCGSTAB 1e-10"
                       + (f", every bias stopped after {outer_cap} outer iterations" if outer_cap else ""))
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


PMC_FAMILIES = {"step_a_fp64": "k_zmarch<3, double, false", "step_b_fp64": "k_zmarch<4, double, false",
                    "step_a_fp32": "k_zmarch<3, float, false", "step_b_fp32": "k_zmarch<4, float, false"}
VECTORS = {"step_a": 12, "step_b": 7}


def pmc_summary_families(fetch_csv, write_csv, workload, copy_bytes, n_nodes):
    """Per-launch counter traffic of the BiCGSTAB step kernels (variable-
    coefficient form; FP64, and FP32 where the run has it) from two
    rocprofv3 --pmc runs (CSV): for each family the most frequent instance
    (the pinned shape), averaged over
    its dispatches that read at least half the algorithmic bytes (launches
    queued after convergence exit early and are left out), each counter
    scaled by its reading on the copy kernel of known size."""
    import csv
    from collections import Counter

    out = {"workload": workload, "source_hash": kernel_source_hash(), "copy_bytes": copy_bytes, "kernels": {}}
    raw = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        raw[counter] = vals
    for fam, pat in PMC_FAMILIES.items():
        names = Counter()
        for k, xs in raw["FETCH_SIZE"].items():
            if pat in k:
                names[k] += len(xs)
        if not names:
            continue
        name = names.most_common(1)[0][0]
        elem = 8 if "double" in pat else 4
        alg = VECTORS[fam[:6]] * n_nodes * elem
        row = {"kernel": name.split("(")[0].replace("void ", ""), "algorithmic_bytes": alg}
        scales = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            copy = [x for k, xs in raw[counter].items() if "copy" in k.lower() for x in xs]
            scales[counter] = copy_bytes / max(copy) if copy else None
        fetch = raw["FETCH_SIZE"].get(name, [])
        write = raw["WRITE_SIZE"].get(name, [])
        keep = [i for i, x in enumerate(fetch) if scales["FETCH_SIZE"] and x * scales["FETCH_SIZE"] >= 0.5 * alg]
        row["dispatches"] = len(fetch)
        row["dispatches_counted"] = len(keep)
        row["runs_aligned"] = len(fetch) == len(write)   # same launches in both runs (pinned shapes)
        for counter, xs in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
            sel = [xs[i] for i in keep if i < len(xs)]
            sc = scales[counter]
            row[counter] = sum(sel) / len(sel) * sc if (sel and sc) else None
            row[counter + "_scale"] = sc
        if row["FETCH_SIZE"] is not None and row["WRITE_SIZE"] is not None:
            row["counter_bytes"] = row["FETCH_SIZE"] + row["WRITE_SIZE"]
            row["counter_over_algorithmic"] = row["counter_bytes"] / alg
        out["kernels"][fam] = row
    a = out["kernels"].get("step_a_fp64", {})
    out["hbm_bytes_per_launch"] = a.get("counter_bytes")   # the roofline's `traffic`
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


def cpu_baseline(prob, lin_iters_full, budget_outer=2, with_interface=False):
    """Oracle on the first outer iterations of the same solve, scaled by the
    BiCGSTAB iteration count of the whole solve."""
    import oracle
    ms = prob.meta["species"]
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
    t0 = time.perf_counter()
    phi, info, _, _ = oracle.nonlinear_solve(prob, prob.fixed_charge, sp, 78.45, prob.meta["lc_A"],
                                            outer_tol=1e-8, lin_tol=1e-10, max_outer=budget_outer,
                                            check=False)
    t = time.perf_counter() - t0
    per_iter = t / max(1, info["total_lin_iters"])
    out = dict(value=per_iter * lin_iters_full, unit="s", cores=1, kind="oracle",
               sample=(f"oracle (serial FP64, 1 thread) on the initial PF2 solve plus {info['outer_iters']} "
                       f"outer iterations of the same 97^3 solve: {t:.1f} s for {info['total_lin_iters']} "
                       f"BiCGSTAB iterations, scaled to the {lin_iters_full} iterations of the full solve"))
    if with_interface:
        # the decomposition's interface setup on the same membrane (compare forms.interface_97.setup_seconds)
        import dataclasses
        import numpy as np
        from paper_1711_04060_amd import inputs
        p2 = dataclasses.replace(prob, fixed_charge=np.zeros(prob.N))
        t0 = time.perf_counter()
        oracle.interface(p2, inputs.point_charges(prob), inputs.lambda_length_A(), inputs.TABLE1["eps_m"],
                         inputs.TABLE1["eps_s"], tol=1e-12)
        out["interface_setup_seconds"] = time.perf_counter() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sample", type=int, default=16, help="time step A in one batch of chunks out of this many")
    ap.add_argument("--forms", type=int, default=1)
    ap.add_argument("--cpu", type=int, default=1)
    ap.add_argument("--n", type=int, default=97)
    ap.add_argument("--bias-sweep", type=int, default=0, help="also run configuration 5 (16 biases, 129^3)")
    ap.add_argument("--tps", type=int, default=0, help="also run the five exchange-cycle states at 97^3")
    ap.add_argument("--loop-settings", type=int, default=0, help="also sweep omega and ErrTol at 49^3")
    ap.add_argument("--bias-outer", type=int, default=0,
                    help="configuration 5: stop every bias after this many outer iterations (0: converge)")
    ap.add_argument("--max-outer", type=int, default=0, help="bounded outer loop (profiler runs only)")
    ap.add_argument("--copy-ref", type=int, default=0, help="run the copy reference kernel (counter scale)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc CSVs into the traffic file and exit")
    ap.add_argument("--trace-summary", nargs="+", metavar="CSV",
                    help="summarise rocprofv3 kernel / memory-copy trace CSVs (busy, idle gaps) and exit")
    ap.add_argument("--copy-ceiling", type=int, default=0,
                    help="measure plain streaming bandwidth (copy, 3-operand product) at several sizes and exit")
    ap.add_argument("--pin-shape", type=str, default="",
                    help="threads,strip,zplanes,depth: launch shape of every stencil kernel instead of the "
                         "autotuner's (for counter runs, whose serialised launches distort the tuner)")
    ap.add_argument("--linear193-only", type=int, default=0,
                    help="run only the 193^3 FP64 and mixed linear solves (for traces and counters) and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary), indent=1))
        return
    if args.pmc_summary:
        if args.linear193_only:
            print(json.dumps(pmc_summary_families(args.pmc_summary[0], args.pmc_summary[1], "sphere_poisson_193",
                                                  512 * (1 << 20), 193 ** 3), indent=1))
        else:
            print(json.dumps(pmc_summary_families(args.pmc_summary[0], args.pmc_summary[1], f"membrane_pore_{args.n}",
                                                  512 * (1 << 20), args.n ** 3), indent=1))
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
    prob = inputs.membrane_pore(args.n)
    g_cache[prob.name] = pf.grid_from_problem(prob)
    extra = {"max_outer": args.max_outer} if args.max_outer else {}
    prm = pf.params_for(prob, outer_tol=1e-8, lin={"rel_tol": 1e-10}, **extra)
    log(f"[bench] workload {prob.name}: N={prob.N}, warmup {args.warmup}, steps {args.steps}")
    for w in range(args.warmup):
        info, _ = run_nonlinear(pf, torch, prob, prm)
        log(f"[bench] warmup {w}: outer {info['outer_iters']} lin {info['total_lin_iters']} "
            f"{info['seconds']:.2f} s")
    pf.pf_timing_enable(1, args.sample)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for s in range(args.steps):
        info, phi = run_nonlinear(pf, torch, prob, prm)
        infos.append(info)
        log(f"[bench] step {s}: outer {info['outer_iters']} lin {info['total_lin_iters']} "
            f"delta {info['last_delta']:.2e} {info['seconds']:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = pf.pf_timing_read(pf.PF_FP64)
    pf.pf_timing_enable(0, 1)
    sec_per_step = elapsed / args.steps
    bytes_per_launch = STEP_A_VECTORS * prob.N * 8
    achieved = bytes_per_launch / (tm["mean_ms"] * 1e-3) / 1e9 if tm["launches"] else 0.0
    traffic = traffic_from_profiles(prob.name)
    lin_iters = infos[-1]["total_lin_iters"]

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
            "workload": (f"membrane_pore {args.n}^3 ({prob.N} nodes, 40 A box, slab+pore+2000-charge shell, "
                         "Na/Ca/Cl/water, steric on, lc 1.9 A): full PF nonlinear solve, outer 1e-8, "
                         "BiCGSTAB 1e-10"),
            "outer_iters": infos[-1]["outer_iters"],
            "bicgstab_iters": lin_iters,
            "bicgstab_iters_per_s": lin_iters / sec_per_step,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "BiCGSTAB step A (previous x, r update + p update + v = A M^-1 p + 2 dots), FP64",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "launches_timed": tm["launches"],
            "mean_us": tm["mean_ms"] * 1e3,
            "bytes_per_launch": bytes_per_launch,
        },
    }
    if args.forms:
        log("[bench] forms: 97^3 PF solve with mixed-precision linear solves")
        result["forms"] = {"pf_solve_97_mixed": forms_pf_mixed(pf, torch, prob, phi)}
        log("[bench] forms: 193^3 FP64 vs mixed")
        result["forms"]["linear_193"] = forms_linear(pf, torch, inputs, args.sample)
        log("[bench] forms: 64-system batch")
        result["forms"]["batch_64"] = forms_batch(pf, torch, inputs)
        log("[bench] forms: isolated cold stencil product at 193^3")
        result["forms"]["spmv_cold_193"] = forms_spmv_cold(pf, torch, inputs)
        log("[bench] forms: singular-charge decomposition at 97^3")
        result["forms"]["interface_97"] = forms_interface(pf, torch, inputs)
    if args.loop_settings:
        log("[bench] forms: outer-loop settings at 49^3")
        result.setdefault("forms", {})["loop_settings_49"] = forms_loop_settings(pf, torch, inputs)
    if args.tps:
        log("[bench] forms: five exchange-cycle states at 97^3")
        result.setdefault("forms", {})["tps_97"] = forms_tps(pf, torch, inputs)
    if args.bias_sweep:
        log("[bench] forms: 16-bias sweep at 129^3")
        result.setdefault("forms", {})["bias_sweep_129"] = forms_bias_sweep(pf, torch, inputs,
                                                                           outer_cap=args.bias_outer)
    if args.cpu:
        log("[bench] cpu baseline (oracle sample)")
        result["cpu_baseline"] = cpu_baseline(prob, lin_iters, with_interface=bool(args.forms))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
