#!/usr/bin/env python3
"""Benchmark: decoupled Bidomain time stepping on one MI355X, AMG-PCG for both systems.

Workload (default): the 384 x 384 x 96-element slab (14,377,825 nodes, 384 M nonzeros; elements
of aspect 2, rotating axisymmetric fibers, eight seeded plateau ellipsoids), the paper's
per-GPU scale (Sec. 6).  Each step is one Aliev-Panfilov membrane update, one parabolic solve
and one elliptic solve (eqs. (4)-(7)), both AMG-preconditioned to rtol 1e-8 with the
hierarchies built once and reused.  The headline path runs the V-cycles in float32 inside
float64 flexible CG; the plain float64 path runs the same steps on the same GPU beside it.

Metric: elliptic PCG-AMG DOF*iters/s = n * (elliptic iterations) / (elliptic solve time), summed
over the timed steps; solve times come from HIP events on the solve stream, inputs resident in
HBM.  The JSON line also carries the roofline of the fine-level outer CG product q = A p (HIP
events around each launch that did the product), the whole-iteration byte rate, the CPU oracle
timed on a bounded sample of the same workload (one core and all cores), and the p50/p99
latencies of a bounded stream of served cases.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
PMC_FILES = [os.path.join(ROOT, "profiles", "pmc_outer_spmv_c5.json")]
# the kernels and their block -> tile mapping; a counter summary stays valid while these are unchanged
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2311_13914_amd", "csrc", "kernels.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def spmv_bytes(n: int, nnz: int, s: int = 8, col_bytes: int = 4, tiles: int = 0, diags: int = 0) -> int:
    """Algorithmic bytes of y = A x in CSR: values + column indices (4 bytes, 3-byte packed
    indices, 2-byte offsets from a per-tile base, or 1-byte offset-dictionary indices) + row
    offsets, x read once, y
    written once, the tile table (and the per-tile column bases with 2-byte offsets); in the
    symmetric diagonal form the `diags` stored diagonals of n values, x once and y once.  The
    p^T q partials are negligible."""
    if diags:
        return diags * n * s + 2 * n * s
    b = nnz * (s + col_bytes) + n * (4 + 2 * s)
    if tiles:
        b += 4 * (tiles + 1) + (4 * tiles if col_bytes == 2 else 0)
    return b


def iteration_bytes(info: dict, s: int) -> int:
    """Algorithmic bytes of one PCG iteration by the cost model of the solve phase: the outer
    float64 product, then per level k below the coarsest 4 products with A_k (pre-smoothing,
    residual, two post-smoothing steps), one with R_k and one with P_k, about 6 level vectors
    streamed by their epilogues, plus about 10 fine float64 vector streams of the CG updates and
    the dense coarsest GEMV.  s: bytes per V-cycle value (8, or 4 for the float32 V-cycle)."""
    n, nnz, L = info["n"], info["nnz"], info["nlevels"]
    d = info.get("diags", [0] * L)
    b = spmv_bytes(n[0], nnz[0], 8, info["col_bytes"][0], info["tiles"][0], d[0])
    for k in range(L - 1):
        b += 4 * spmv_bytes(n[k], nnz[k], s, info["col_bytes"][k], info["tiles"][k], d[k])
        pn = info["p_nnz"][k]
        b += pn * (s + info["col_bytes_r"][k]) + n[k + 1] * (4 + s) + n[k] * s  # R_k: n_{k+1} rows
        b += pn * (s + info["col_bytes_p"][k]) + n[k] * (4 + 2 * s) + n[k + 1] * s  # P_k: y += P e
        b += 6 * n[k] * s
    b += 10 * n[0] * 8 + n[L - 1] * n[L - 1] * 8
    return b


def traffic_from_profile(n, nnz):
    """Measured HBM bytes per launch of the outer product, from the committed rocprofv3 counter
    summary of this workload -- only while the kernel sources are the ones that were profiled."""
    for path in PMC_FILES:
        if not os.path.exists(path):
            continue
        rec = json.load(open(path))
        if rec.get("kernel_source_hash") == kernel_source_hash() and rec.get("n") == n and rec.get("nnz") == nnz:
            return rec.get("bytes_per_launch")
    return None


# ---- CPU oracle baseline ----------------------------------------------------------------
def _oracle_sample_worker(case, reps, barrier, out):
    """One oracle process: assemble and set up (untimed), then `reps` elliptic solves from a zero
    guess to rtol 1e-8, each started together with the other processes' (barrier)."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, fem, krylov
    import bidomain_cases as bc

    with threadpool_limits(limits=1):
        ops = fem.assemble_operators(case)
        A = ops["Aell"]
        f = -(ops["Ai"] @ bc.nodal_v0(case))
        t = time.perf_counter()
        h = amg.setup(A, amg.AMGOptions(nullspace=True))
        t_setup = time.perf_counter() - t
        runs = []
        for _ in range(reps):
            if barrier is not None:
                barrier.wait()
            t = time.perf_counter()
            res = krylov.amg_pcg(A, f, h, rtol=1e-8, maxit=500, m=ops["m"])
            runs.append((res.iterations, time.perf_counter() - t))
    out.put((t_setup, runs))


def cpu_baseline(case, block, reps: int = 3):
    """The oracle (plain float64 numpy/scipy, as it stands) on a bounded sample of the workload:
    the block of `block` elements around the first stimulus ellipsoid, with the workload's element
    sizes, fiber field and stimulus.  One process on one core, then one process per core of the
    host's CPU share solving concurrently (whole-job rate: all processes' DOF*iters over the
    slowest one's time); the median of `reps` solves each."""
    import multiprocessing as mp

    import bidomain_cases as bc

    sample = bc.block_of(case, *block) if (case.nx, case.ny, case.nz) != tuple(block) else case
    ctx = mp.get_context("spawn")

    def run(procs):
        q = ctx.Queue()
        bar = ctx.Barrier(procs) if procs > 1 else None
        ps = [ctx.Process(target=_oracle_sample_worker, args=(sample, reps, bar, q)) for _ in range(procs)]
        for p in ps:
            p.start()
        res = [q.get() for _ in ps]
        for p in ps:
            p.join()
        rates = []
        for r in range(reps):
            its = sum(x[1][r][0] for x in res)
            slowest = max(x[1][r][1] for x in res)
            rates.append(sample.n * its / slowest)
        return float(np.median(rates)), res[0][0], res[0][1][0][0]

    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    procs = max(1, min(16, share))
    one, t_setup, its = run(1)
    allc, _, _ = run(procs) if procs > 1 else (one, None, None)
    desc = (f"{sample.nx}x{sample.ny}x{sample.nz}-element block of the {case.nx}x{case.ny}x{case.nz} slab "
            f"(n = {sample.n}, same element sizes, fibers and stimulus); elliptic AMG-PCG solve from a zero "
            f"guess to rtol 1e-8 ({its} iterations), median of {reps}; oracle assembly and setup untimed "
            f"({t_setup:.1f} s); all-core figure: {procs} concurrent single-threaded processes")
    return dict(value=allc, unit="DOF*iters/s", cores=procs, kind="oracle", sample=desc,
                one_core=dict(value=one, cores=1))


def bench_solve(args):
    """Single elliptic solves (f = -A_i v0, zero guess) with the float64 V-cycle as reference."""
    import torch

    import bidomain_cases as bc
    import paper_2311_13914_amd as lib

    case = bc.config_case(args.workload)
    n = case.n
    rp, ci, vi, m = lib.bidomain_slab_assemble(case, lib.BD_MAT_AI)
    rpe, cie, ve, _ = lib.bidomain_slab_assemble(case, lib.BD_MAT_AELL)
    v0 = bc.nodal_v0(case)
    import scipy.sparse as sp
    Ai = sp.csr_matrix((vi, ci, rp), shape=(n, n))
    f = torch.tensor(-(Ai @ v0), dtype=torch.float64, device="cuda")
    del Ai, vi
    coarsening = lib.BD_RS if args.coarsening == "rs" else lib.BD_SA
    thr = 0.5 if args.coarsening == "rs" else 0.06
    results = {}
    for prec in ([lib.BD_F64, lib.BD_F32] if args.mixed else [lib.BD_F64]):
        t = time.perf_counter()
        h = lib.bidomain_amg_setup((rpe, cie, ve), lib.bidomain_default_opts(
            nullspace=1, vcycle_precision=prec, coarsening=coarsening, threshold=thr), m)
        setup_s = time.perf_counter() - t
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            lib.bidomain_pcg_solve(h, f, x, False, args.rtol, 500)
        its, secs = 0, 0.0
        for _ in range(args.steps):
            rc, info = lib.bidomain_pcg_solve(h, f, x, False, args.rtol, 500)
            assert rc == lib.BD_OK, info
            its += info["iterations"]
            secs += info["seconds"]
        hinfo = lib.bidomain_amg_info(h)
        lib.bidomain_amg_destroy(h)
        results[prec] = dict(x=x, its=its, secs=secs, setup_s=setup_s, levels=hinfo["n"],
                             opc=hinfo["operator_complexity"], res=info["rel_residual_true"],
                             bytes=hinfo["device_bytes"],
                             hierarchy={k: hinfo[k] for k in ("n", "nnz", "p_nnz", "tiles", "col_bytes",
                                                              "col_bytes_p", "col_bytes_r", "diags")})
        print(f"[bench] {'f32' if prec else 'f64'} {args.coarsening}: setup {setup_s:.1f} s, levels "
              f"{hinfo['n']}, {its / args.steps:.1f} it/solve, {secs / args.steps * 1e3:.2f} ms/solve",
              file=sys.stderr, flush=True)
    key = lib.BD_F32 if args.mixed else lib.BD_F64
    r = results[key]
    err = None
    if args.mixed:
        x64 = results[lib.BD_F64]["x"]
        err = float(torch.linalg.norm(r["x"] - x64) / torch.linalg.norm(x64))
    out = {
        "metric": "elliptic PCG-AMG DOF*iters/s", "value": n * r["its"] / r["secs"], "unit": "DOF*iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["secs"] * 1e3 / args.steps, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32-vcycle/f64" if args.mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: single elliptic solve on the {case.nx}x{case.ny}x{case.nz} "
                               f"slab, n={n}, {args.coarsening.upper()} hierarchy, rtol {args.rtol:g}",
                   "levels": r["levels"], "operator_complexity": round(r["opc"], 3),
                   "device_bytes": r["bytes"]},
        "hierarchy": r["hierarchy"],
        "iters_per_solve": r["its"] / args.steps, "rel_residual_true": r["res"],
        "rel_error_vs_f64": err, "setup_s": round(r["setup_s"], 1),
    }
    if args.mixed:
        r64 = results[lib.BD_F64]
        out["f64_reference"] = {"value": n * r64["its"] / r64["secs"], "iters_per_solve": r64["its"] / args.steps,
                                "ms_per_solve": r64["secs"] * 1e3 / args.steps}
    print(json.dumps(out), flush=True)


def serve_stream(args, n_cases, nsteps, rate):
    """A seeded stream of slab cases (log-uniform sizes, Poisson arrivals) through the server:
    float32 V-cycles inside float64 CG, hierarchies and states resident in HBM, admission by
    device budget and slots, all running solves batched per round.  Returns the latency and
    throughput summary."""
    import bidomain_cases as bc
    import paper_2311_13914_amd as lib

    reqs = bc.serving_stream(n_cases=n_cases, nsteps=nsteps, rate_per_s=rate, seed=4)
    v0s = {r.ticket: bc.nodal_v0(r.case) for r in reqs}
    prec = lib.BD_F64 if args.no_mixed_serve else lib.BD_F32
    oe = lib.bidomain_default_opts(vcycle_precision=prec)
    op = lib.bidomain_default_opts(vcycle_precision=prec, threshold=0.0)  # parabolic default
    budget = int(args.budget_gb * (1 << 30))
    srv = lib.bidomain_serve_create(budget, args.slots, oe, op, args.rtol)
    done, ticket_of, peak = {}, {}, dict(running=0, bytes=0)
    t0 = time.perf_counter()
    nxt = 0
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt].arrival_s <= now:
            r = reqs[nxt]
            ticket_of[lib.bidomain_serve_submit(srv, r.case, v0s[r.ticket], r.nsteps)] = r
            nxt += 1
        for res in lib.bidomain_serve_poll(srv):
            done[res["ticket"]] = res
        st = lib.bidomain_serve_stats(srv)
        peak["running"] = max(peak["running"], st["running"])
        peak["bytes"] = max(peak["bytes"], st["bytes_in_use"])
        if nxt < len(reqs) and st["running"] + st["setting_up"] + st["queued"] == 0:
            time.sleep(max(0.0, min(0.01, reqs[nxt].arrival_s - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    lat = lib.bidomain_serve_solve_latencies(srv)
    st = lib.bidomain_serve_stats(srv)
    lib.bidomain_serve_destroy(srv)
    bad = [r for r in done.values() if r["status"] != lib.BD_OK]
    assert not bad, bad[:3]
    case_lat = np.array([r["t_done"] - r["t_submit"] for r in done.values()])
    queue_wait = np.array([r["t_admit"] - r["t_submit"] for r in done.values()])
    setup_s = np.array([r["t_ready"] - r["t_admit"] for r in done.values()])
    dof_its = sum(ticket_of[t].case.n * (r["it_par"] + r["it_ell"]) for t, r in done.items())
    return {
        "workload": f"C4 stream: {n_cases} slab cases, elements log-uniform 32x32x16..160x160x64, {nsteps} IMEX "
                    f"steps each, Poisson arrivals {rate:g}/s, budget {args.budget_gb:g} GB, {args.slots} slots, "
                    f"{'float64' if args.no_mixed_serve else 'float32'} V-cycles, rtol {args.rtol:g}",
        "solves": int(len(lat)), "p50_solve_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_solve_ms": float(np.percentile(lat, 99) * 1e3),
        "p50_case_s": float(np.percentile(case_lat, 50)), "p99_case_s": float(np.percentile(case_lat, 99)),
        "max_case_s": float(case_lat.max()), "mean_queue_wait_s": float(queue_wait.mean()),
        "mean_setup_s": float(setup_s.mean()), "makespan_s": wall,
        "throughput_dof_iters_per_s": dof_its / wall, "rounds": st["rounds"],
        "max_solves_per_round": st["max_batched"], "peak_running_cases": peak["running"],
        "peak_bytes": peak["bytes"], "host_enqueue_s": round(st["host_enqueue_s"], 2),
        "host_wait_s": round(st["host_wait_s"], 2), "host_exit_s": round(st["host_exit_s"], 2),
        "note": f"with {n_cases} cases the case p99 is close to the maximum",
    }


def bench_serve(args):
    out = serve_stream(args, args.serve_cases, args.serve_steps, args.rate)
    line = {
        "metric": "p50/p99 served solve latency", "value": out["p50_solve_ms"], "unit": "ms",
        "n_gpus": 1, "steps": args.serve_steps, "warmup": 0, "ms_per_step": None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.no_mixed_serve else "f32-vcycle/f64", "data": "synthetic",
        "config": {"workload": out["workload"]}, "serving": out,
    }
    print(json.dumps(line), flush=True)


def run_steps(args, case, mixed: bool, profile: bool):
    """Build the simulation (setup untimed), run the warm-up steps, then time `args.steps` steps.
    Returns the step statistics, the hierarchy statistics and the final v and u_e (device)."""
    import torch

    import bidomain_cases as bc
    import paper_2311_13914_amd as lib

    prec = lib.BD_F32 if mixed else lib.BD_F64
    opts_e = lib.bidomain_default_opts(vcycle_precision=prec)
    opts_p = lib.bidomain_default_opts(vcycle_precision=prec, threshold=0.0)  # parabolic default
    opts_p.preconditioner = {"amg": lib.BD_PC_AMG, "jacobi": lib.BD_PC_JACOBI, "none": lib.BD_PC_NONE}[args.par_precond]
    if opts_p.preconditioner != lib.BD_PC_AMG:
        opts_p.vcycle_precision = lib.BD_F64
    v0 = torch.tensor(bc.nodal_v0(case), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    t = time.perf_counter()
    sim = lib.bidomain_sim_create(case, v0, rtol=args.rtol, ell_opts=opts_e, par_opts=opts_p, stream=stream)
    setup_s = time.perf_counter() - t
    del v0
    info_e = lib.bidomain_amg_info(lib.bidomain_sim_hierarchy(sim, 0))
    info_p = lib.bidomain_amg_info(lib.bidomain_sim_hierarchy(sim, 1))
    tag = "float32 V-cycles" if mixed else "float64"
    print(f"[bench] {tag}: n={case.n} setup {setup_s:.1f} s; elliptic levels {info_e['n']}; "
          f"parabolic levels {info_p['n']}", file=sys.stderr, flush=True)
    if args.warmup:
        rc, _ = lib.bidomain_step(sim, args.warmup, args.rtol, stream=stream)
        assert rc == lib.BD_OK, rc
    lib.bidomain_profile_read(reset=True)
    lib.bidomain_profile_enable(profile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, info = lib.bidomain_step(sim, args.steps, args.rtol, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lib.bidomain_profile_enable(False)
    prof_ms, prof_launches = lib.bidomain_profile_read(reset=True)
    assert rc == lib.BD_OK, (rc, info)
    v = torch.empty(case.n, dtype=torch.float64, device="cuda")
    ue = torch.empty(case.n, dtype=torch.float64, device="cuda")
    lib.bidomain_sim_get(sim, lib.BD_V, v)
    lib.bidomain_sim_get(sim, lib.BD_UE, ue)
    lib.bidomain_sim_destroy(sim)
    torch.cuda.synchronize()
    print(f"[bench] {tag}: {args.steps} steps in {wall:.3f} s; it_ell {info['it_ell']} it_par {info['it_par']}",
          file=sys.stderr, flush=True)
    return dict(info=info, info_e=info_e, info_p=info_p, wall=wall, setup_s=setup_s, prof_ms=prof_ms,
                prof_launches=prof_launches, v=v, ue=ue)


def step_summary(args, case, r):
    info = r["info"]
    return {"value": case.n * info["it_ell"] / (info["ms_ell"] * 1e-3),
            "ms_per_step": r["wall"] * 1e3 / args.steps,
            "phases_ms_per_step": {"memb": info["ms_memb"] / args.steps, "par": info["ms_par"] / args.steps,
                                   "ell": info["ms_ell"] / args.steps},
            "iters_per_step": {"par": info["it_par"] / args.steps, "ell": info["it_ell"] / args.steps},
            "rel_residual_last": {"par": info["rel_res_par"], "ell": info["rel_res_ell"]},
            "setup_s": round(r["setup_s"], 2)}


SWEEP = {"sa": (0.0, 0.01, 0.02, 0.03, 0.04, 0.05, 0.06, 0.07),
         "pmis": (0.25, 0.3, 0.4, 0.5, 0.6, 0.7),
         "rs": (0.25, 0.3, 0.4, 0.5, 0.6, 0.7)}


def bench_sweep(args):
    """Threshold calibration on the truncated ellipsoid (Sec. 6 Test 1): for each coarsening and
    threshold of the paper's ranges (SA: the aggregation threshold of its GAMG table; PMIS and the
    classical first pass: the strong threshold of its BoomerAMG tables), a simulation of
    args.sweep_steps IMEX steps from the apical stimulus; reports the mean elliptic iterations and
    device time per step and the hierarchy.  One JSON line on stdout, a table on stderr."""
    import torch

    import bidomain_cases as bc
    import paper_2311_13914_amd as lib

    case = bc.ellipsoid_case(args.sweep_mesh)
    prec = lib.BD_F64 if args.f64 else lib.BD_F32
    v0 = torch.tensor(bc.ellipsoid_v0(case), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for coarsening, ths in SWEEP.items():
        code = {"sa": lib.BD_SA, "rs": lib.BD_RS, "pmis": lib.BD_PMIS}[coarsening]
        for th in ths:
            opts_e = lib.bidomain_default_opts(coarsening=code, threshold=th, vcycle_precision=prec)
            opts_p = lib.bidomain_default_opts(vcycle_precision=prec, threshold=0.0)
            t = time.perf_counter()
            sim = lib.bidomain_sim_create(case, v0, rtol=args.rtol, ell_opts=opts_e, par_opts=opts_p, stream=stream)
            setup_s = time.perf_counter() - t
            info_e = lib.bidomain_amg_info(lib.bidomain_sim_hierarchy(sim, 0))
            rc, info = lib.bidomain_step(sim, args.sweep_steps, args.rtol, stream=stream)
            lib.bidomain_sim_destroy(sim)
            assert rc == lib.BD_OK, (coarsening, th, rc, info)
            row = dict(coarsening=coarsening, threshold=th, levels=info_e["n"],
                       operator_complexity=round(info_e["operator_complexity"], 3),
                       it_ell_mean=round(info["it_ell"] / args.sweep_steps, 2),
                       ms_ell_mean=round(info["ms_ell"] / args.sweep_steps, 3),
                       it_par_mean=round(info["it_par"] / args.sweep_steps, 2), setup_s=round(setup_s, 3))
            rows.append(row)
            print(f"[sweep] {coarsening:4s} {th:5.2f}: it_ell {row['it_ell_mean']:6.2f}  ms_ell "
                  f"{row['ms_ell_mean']:7.3f}  levels {row['levels']}  complexity {row['operator_complexity']}",
                  file=sys.stderr, flush=True)
    print(json.dumps({"metric": "elliptic_iterations_per_step", "mode": "threshold_sweep",
                      "workload": f"truncated ellipsoid {case.n_theta}x{case.n_phi}x{case.n_r} ({case.n} nodes)",
                      "steps": args.sweep_steps, "dt_ms": case.dt, "rtol": args.rtol,
                      "vcycle": "f64" if args.f64 else "f32", "rows": rows}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--f64", action="store_true", help="headline path with float64 V-cycles (default: float32 "
                                                       "V-cycles inside float64 flexible CG)")
    ap.add_argument("--mixed", action="store_true", help="(solve mode) float32 V-cycle beside the float64 one")
    ap.add_argument("--no-f64-path", action="store_true", help="skip the float64 path run beside the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-block", default="128,128,32", help="elements of the oracle's sample block")
    ap.add_argument("--no-serve", action="store_true", help="skip the bounded serving stream")
    ap.add_argument("--workload", default="C5", choices=["C1", "C2", "C3", "C5"])
    ap.add_argument("--mode", default="step", choices=["step", "solve", "serve", "sweep"],
                    help="step: Bidomain time steps (default); solve: repeated single elliptic solves; "
                         "serve: a stream of cases through the batching server; sweep: AMG threshold "
                         "calibration on the truncated ellipsoid")
    ap.add_argument("--sweep-mesh", default="E1", choices=["E1", "E2"])
    ap.add_argument("--sweep-steps", type=int, default=100, help="sweep: IMEX steps per threshold (5 ms)")
    ap.add_argument("--serve-cases", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=20)
    ap.add_argument("--rate", type=float, default=1.0, help="serve: Poisson arrival rate (cases/s)")
    ap.add_argument("--bounded-serve", default="16,5,2", help="cases,steps,rate of the serving stream in the "
                                                              "step-mode line")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--no-mixed-serve", action="store_true", help="serve: float64 V-cycles")
    ap.add_argument("--coarsening", default="sa", choices=["sa", "rs"])
    ap.add_argument("--par-precond", default="amg", choices=["amg", "jacobi", "none"],
                    help="step: preconditioner of the parabolic CG (none = the paper's GPU runs, Sec. 5)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed region, copy 1 GiB once (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import bidomain_cases as bc
    import paper_2311_13914_amd as lib

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.mode == "solve":
        return bench_solve(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "sweep":
        return bench_sweep(args)
    case = bc.config_case(args.workload)
    n, nnz = case.n, case.nnz27
    mixed = not args.f64
    r = run_steps(args, case, mixed, profile=True)
    info, info_e = r["info"], r["info_e"]
    head = step_summary(args, case, r)
    avg_ms = r["prof_ms"] / max(r["prof_launches"], 1)
    diags = info_e["diags"][0]
    bytes_launch = spmv_bytes(n, nnz, 8, info_e["col_bytes"][0], info_e["tiles"][0], diags)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    it_bytes = iteration_bytes(info_e, 4 if mixed else 8)
    it_ms = info["ms_ell"] / max(info["it_ell"], 1)
    it_gbs = it_bytes / (it_ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic_from_profile(n, nnz),
                    kernel=(("k_spmv_sdia<double, 8>" if diags else "k_spmv_stream<double, 8>")
                            + " (OP_CG_Q: outer q = A p on the fine operator, float64, with p^T q)"),
                    bytes_per_launch=bytes_launch, column_index_bytes=info_e["col_bytes"][0],
                    stored_diagonals=diags, avg_launch_ms=round(avg_ms, 5), launches=r["prof_launches"],
                    note="launches that did the product only (those enqueued past convergence return at once)")
    iteration = dict(bytes=it_bytes, ms=round(it_ms, 4), achieved=round(it_gbs, 1),
                     frac=round(it_gbs / PEAK_HBM_GBS, 4),
                     note="whole elliptic PCG iteration (outer product, V-cycle, CG updates) by the cost "
                          "model of iteration_bytes, over elliptic solve time / iterations")
    out = {
        "metric": "elliptic PCG-AMG DOF*iters/s",
        "value": head["value"],
        "unit": "DOF*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32-vcycle/f64" if mixed else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: Bidomain slab {case.nx}x{case.ny}x{case.nz} Q1 elements, n={n}, "
                        f"nnz={nnz}, Aliev-Panfilov + parabolic + elliptic AMG-PCG per step, "
                        + ("float32 V-cycles in float64 flexible CG" if mixed else "float64 AMG-PCG")
                        + f", rtol {args.rtol:g}"
                        + ("" if args.par_precond == "amg" else f"; parabolic CG preconditioner: {args.par_precond}"),
            "elliptic_levels": info_e["n"],
            "parabolic_levels": r["info_p"]["n"],
            "operator_complexity_ell": round(info_e["operator_complexity"], 3),
        },
        "phases_ms_per_step": head["phases_ms_per_step"],
        "iters_per_step": head["iters_per_step"],
        "rel_residual_last": head["rel_residual_last"],
        "setup_s": head["setup_s"],
        "roofline": roofline,
        "iteration_roofline": iteration,
    }
    if mixed and not args.no_f64_path:
        v_m, ue_m = r["v"], r["ue"]
        del r
        r64 = run_steps(args, case, False, profile=False)
        f64 = step_summary(args, case, r64)
        f64["rel_diff_vs_mixed"] = {
            "v": float(torch.linalg.norm(r64["v"] - v_m) / torch.linalg.norm(r64["v"])),
            "ue": float(torch.linalg.norm(r64["ue"] - ue_m) / torch.linalg.norm(r64["ue"])),
            "note": "after the same warm-up and timed steps, each solve at rtol 1e-8"}
        out["f64_path"] = f64
        del r64, v_m, ue_m
    else:
        del r
    torch.cuda.empty_cache()
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_serve:
        nc, ns, rate = args.bounded_serve.split(",")
        print("[bench] bounded serving stream", file=sys.stderr, flush=True)
        out["serving"] = serve_stream(args, int(nc), int(ns), float(rate))
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, tuple(int(v) for v in args.cpu_block.split(",")))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
