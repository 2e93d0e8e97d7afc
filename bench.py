"""Benchmark of the DG multigrid-Schwarz solver on one MI355X.

Workload (one step = one full solve to a 1e-10 relative residual):
  3D Poisson on [0,1]^3, 8x8x8 elements, p = 6 (175,616 DOFs), source from 16
  seeded random Fourier modes (seed 2), homogeneous Dirichlet, penalty C = 1.5,
  3-level multigrid V-cycle with 3+3 additive Schwarz steps (overlap 2)
  preconditioning flexible GMRES.  The headline runs the mixed-precision
  solver (FP32 MFMA subdomain solves, FP64 everywhere else); the plain FP64
  solver is timed beside it on the same inputs.

Also measured: operator-apply throughput (GDOF/s) with HIP events on the
stream the kernel runs on, on the same shape and on a 40^3, p = 7 shape whose
vectors (262 MB) exceed the 256 MB Infinity Cache; the ceilings the GPU
reaches outside the library (a 512 MiB copy, an FP32 torch.matmul) beside the
vendor peaks; and the oracle on the host CPU on a bounded sample (one solve of
the same workload).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time to 1e-10 rel residual & DG apply GDOF/s; mixed vs FP64; p50/p99"
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_FP64_PEAK_TFLOPS = 78.6

# HBM traffic per launch of the two roofline kernels, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs of this script, each scaled by what the same
# counter reads for the plain copy of COPY_BYTES made below.  A figure is
# reported only while the sources it was measured on are unchanged.
MEASURED_TRAFFIC = {
    "subdomain_gemm": {"sources": ["paper_2111_06767_amd/csrc/dgs_schwarz.hip",
                                   "paper_2111_06767_amd/csrc/dgs_internal.h"],
                       "sha256": "e938373551449a8ea1a3516b307afcd9e0cd77c4ed5ffdbada422dc884a1f3e7",
                       "bytes": 68707843},
    "apply": {"sources": ["paper_2111_06767_amd/csrc/dgs_apply.hip",
                          "paper_2111_06767_amd/csrc/dgs_internal.h"],
              "sha256": "cb7d0cf42f33170e20ac90f612691b41f7ab274968708ac41cdb48800bedb32f",
              "bytes": 633367037},
}


def _sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    t = MEASURED_TRAFFIC[kernel]
    if t["bytes"] is None or _sources_sha256(t["sources"]) != t["sha256"]:
        return None
    return t["bytes"]


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def build_c2(dg, precision, **opts):
    import torch
    import workloads as W
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (8, 8, 8), 6, penalty=1.5, mg_levels=3,
                      precision=precision, **opts)
    xyz = prob.node_coordinates()
    modes = W.fourier_modes(W.SEED_C2)
    x, y, z = (xyz[d].cpu().numpy() for d in range(3))
    f = torch.as_tensor(W.fourier_source(modes, x, y, z)).cuda()
    b = prob.apply_mass(f)
    uex = W.fourier_solution(modes, x, y, z)
    return prob, b, uex


def time_solves(prob, b, steps, warmup):
    import torch
    u = torch.zeros_like(b)
    for _ in range(warmup):
        u.zero_()
        prob.solve(b, u)
    torch.cuda.synchronize()
    times, stats = [], None
    t_all = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, stats = prob.solve(b, u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    total = time.perf_counter() - t_all
    return u, stats, times, total


def time_cg(prob, b, reps=10):
    """The same solve by preconditioned conjugate gradients (dgs_cg_solve),
    one V-cycle per iteration: p50 wall time and iterations."""
    import torch
    u = torch.zeros_like(b)
    prob.solve_cg(b, u)
    times, st = [], None
    for _ in range(reps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = prob.solve_cg(b, u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return dict(ms_p50=round(1e3 * _pct(times, 50), 3), iterations=st["iterations"],
                rel_residual=st["rel_residual"], converged=st["converged"])


def time_apply(dg, elements, p, reps=100, warm=10, calibration_copy=False, shape=None):
    """Average apply duration with HIP events on torch's current stream (the
    stream the library launches on).  With calibration_copy, one plain
    device-to-device copy of the input vector follows the timed applies: the
    known-size transfer the HBM counters are scaled by."""
    import torch
    import workloads as W
    prob = dg.Problem((0, 0, 0), (1, 1, 1), elements, p, mg_levels=1)
    if shape is not None:
        prob.set_apply_shape(shape)
    u = torch.as_tensor(W.random_normal(W.SEED_APPLY, prob.ndof)).cuda()
    out = torch.empty_like(u)
    for _ in range(warm):
        prob.apply(u, out)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        prob.apply(u, out)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    if calibration_copy:
        out.copy_(u)
        torch.cuda.synchronize()
    n = prob.ndof
    shape = prob.apply_shape()
    prob.close()
    del u, out
    torch.cuda.empty_cache()
    return dict(elements=list(elements), p=p, ndof=n, launch_shape=shape,
                ms_per_apply=ms, gdofs=n / (ms * 1e-3) / 1e9,
                algorithmic_bytes=16 * n, achieved_gbs=16 * n / (ms * 1e-3) / 1e9)


def time_subdomain_gemm(prob, reps=50, warm=5):
    """Average duration of the fine-level grouped subdomain-solve GEMM (one
    Schwarz sweep's du_S = s A_S^-1 r_S), HIP events on torch's current stream."""
    import torch
    s = torch.cuda.current_stream()
    prob.subdomain_solves(0, warm)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    flops = prob.subdomain_solves(0, reps)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return dict(flops_per_launch=flops, ms_per_launch=ms, achieved_tflops=flops / (ms * 1e-3) / 1e12)


def measured_ceilings():
    """What this GPU reaches outside the library, reported beside the vendor
    peaks: a device-to-device copy of 512 MiB (read and write counted), and
    an FP32 8192^3 product through torch.matmul (the vendor BLAS)."""
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = 1 << 26
    a = torch.empty(n, dtype=torch.float64, device="cuda").normal_()
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    e0.record(s)
    for _ in range(20):
        c.copy_(a)
    e1.record(s)
    e1.synchronize()
    copy_gbs = 2 * 8 * n * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, c
    m = 8192
    x = torch.randn(m, m, device="cuda", dtype=torch.float32)
    y = torch.randn(m, m, device="cuda", dtype=torch.float32)
    for _ in range(3):
        z = x @ y
    e0.record(s)
    for _ in range(10):
        z = x @ y
    e1.record(s)
    e1.synchronize()
    gemm_tflops = 2 * m ** 3 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del x, y, z
    return dict(copy_gbs=copy_gbs, fp32_gemm_tflops=gemm_tflops)


def time_c5(dg, steps=3):
    """The 16^3, p = 7 share (2.1 M DOFs, 4 levels): FP64 and mixed solves."""
    import torch
    import workloads as W
    out = {}
    for prec in ("mixed", "fp64"):
        prob = dg.Problem((0, 0, 0), (1, 1, 1), (16, 16, 16), 7, penalty=1.5, mg_levels=4,
                          precision=prec)
        xyz = prob.node_coordinates()
        modes = W.fourier_modes(W.SEED_C5)
        f = torch.as_tensor(W.fourier_source(modes, *(xyz[d].cpu().numpy() for d in range(3)))).cuda()
        b = prob.apply_mass(f)
        u, st, times, _ = time_solves(prob, b, steps, 1)
        out[prec] = dict(ms_p50=round(1e3 * _pct(times, 50), 3), iterations=st["iterations"],
                         rel_residual=st["rel_residual"], setup_s=round(st["t_setup_s"], 3),
                         u=u.cpu().numpy())
        prob.close()
    out["speedup_mixed_vs_fp64"] = round(out["fp64"]["ms_p50"] / out["mixed"]["ms_p50"], 3)
    out["mixed_vs_fp64_solution_rel_diff"] = float(
        np.linalg.norm(out["mixed"]["u"] - out["fp64"]["u"]) / np.linalg.norm(out["fp64"]["u"]))
    for prec in ("mixed", "fp64"):
        del out[prec]["u"]
    return out


def run_serving(dg, n_requests=256, max_active=16, precision="mixed", host_threads=0):
    """Poisson-process stream of solves (grids {2..6}^3, p in 3..8, cube sides
    1..4, random-Fourier sources): a closed-loop pass measures the saturation
    throughput, then requests arrive at 0.8 of it and p50/p99 latency and
    throughput are recorded."""
    import workloads as W
    reqs = W.request_stream(n_requests, rate=1.0)
    data = []
    for r in reqs:
        side = r.side
        xyz = dg.points((0, 0, 0), (side,) * 3, r.elements, r.p)
        f = W.fourier_source(W.fourier_modes(r.seed, (0, 0, 0), (side,) * 3), *xyz)
        data.append((r, f))

    def closed_loop():
        srv = dg.Server(hbm_budget_bytes=64e9, max_active=max_active, precision=precision, max_iter=60,
                    host_threads=host_threads)
        t0 = time.perf_counter()
        for r, f in data:
            srv.submit((0, 0, 0), (r.side,) * 3, r.elements, r.p, f)
        while srv.step() != (0, 0):
            pass
        dt = time.perf_counter() - t0
        its = []
        for rid in srv.finished():
            _, st, _ = srv.fetch(rid)
            its.append(st["iterations"])
        srv.close()
        return n_requests / dt, its

    cold_tput, _ = closed_loop()  # fills the inverse cache
    warm_tput, its = closed_loop()
    rate = 0.8 * warm_tput
    gaps = np.array([r.arrival for r, _ in data]) / rate  # unit-rate arrivals rescaled
    srv = dg.Server(hbm_budget_bytes=64e9, max_active=max_active, precision=precision, max_iter=60,
                    host_threads=host_threads)
    t0 = time.perf_counter()
    nxt = 0
    ids = {}
    peak_active = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < n_requests and gaps[nxt] <= now:
            r, f = data[nxt]
            ids[srv.submit((0, 0, 0), (r.side,) * 3, r.elements, r.p, f)] = nxt
            nxt += 1
        a, q = srv.step()
        peak_active = max(peak_active, a)
        if nxt == n_requests and a == 0 and q == 0:
            break
        if a == 0 and q == 0 and nxt < n_requests:
            time.sleep(max(0.0, min(0.001, gaps[nxt] - (time.perf_counter() - t0))))
    makespan = time.perf_counter() - t0
    lat, conv = [], 0
    for rid in srv.finished():
        _, st, times = srv.fetch(rid)
        lat.append(times[2] - times[0])
        conv += int(st["converged"] and st["rel_residual"] <= 1e-10)
    srv.close()
    return dict(requests=n_requests, precision=precision, max_active=max_active,
                saturation_solves_per_s_cold_cache=round(cold_tput, 2),
                saturation_solves_per_s=round(warm_tput, 2), arrival_rate_per_s=round(rate, 2),
                solves_per_s=round(n_requests / makespan, 2),
                latency_ms_p50=round(1e3 * _pct(lat, 50), 2), latency_ms_p99=round(1e3 * _pct(lat, 99), 2),
                converged_to_1e10=conv, peak_active=peak_active,
                iterations_p50=float(np.median(its)), iterations_max=int(max(its)))


def cpu_baseline():
    """The oracle solving the same workload once (setup not counted)."""
    import workloads as W
    from oracle import krylov, mesh, multigrid, operator
    m = mesh.BoxMesh((0, 0, 0), (1, 1, 1), (8, 8, 8), 6)
    x, y, z = m.node_coordinates()
    b = operator.apply_mass(m, W.fourier_source(W.fourier_modes(W.SEED_C2), x, y, z)).reshape(-1)
    N = m.N
    A = lambda v: operator.apply_operator(m, v.reshape(m.E, N, N, N), 1.5).reshape(-1)
    t0 = time.perf_counter()
    V = multigrid.VCycle(m, 1.5, levels=3)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    u, its, hist = krylov.fgmres(A, b, precondition=V, rtol=1e-10)
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=1.0 / t, unit="solves/s", cores=threads, kind="oracle",
                sample=f"one FP64 oracle solve of the 8^3 p=6 workload ({its} FGMRES iterations, "
                       f"{t:.1f} s; set-up of {t_setup:.1f} s not counted)"), u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large-apply", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    # the ceiling measurements include large copies; counter runs that are
    # calibrated by the one 262 MB copy leave them out
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    # host threads that issue the active requests' stages (0: the library default)
    ap.add_argument("--serve-threads", type=int, default=0)
    # pin the autotuned choices of the two roofline kernels (the 8^3 p=6 mixed
    # problem's fine-level GEMM variant, the 40^3 p=7 apply's launch shape), so
    # that a profiled run launches the kernels an unprofiled run chose
    ap.add_argument("--gemm-variant", type=int, default=None)
    ap.add_argument("--apply-shape", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2111_06767_amd as dg
    torch.cuda.set_device(0)

    res = {}
    for prec in ("mixed", "fp64"):
        _log(f"8^3 p=6 {prec}: set-up and {args.warmup}+{args.steps} solves")
        prob, b, uex = build_c2(dg, prec)
        if prec == "mixed" and args.gemm_variant is not None:
            prob.set_gemm_variant(args.gemm_variant, level=0)
        u, st, times, total = time_solves(prob, b, args.steps, args.warmup)
        un = u.cpu().numpy()
        res[prec] = dict(prob=prob, b=b, u=un, stats=st, times=times, total=total,
                         err_exact=float(np.sqrt(np.mean((un - uex) ** 2))),
                         setup_s=st["t_setup_s"])

    mixed, fp64 = res["mixed"], res["fp64"]
    sol_diff = float(np.linalg.norm(mixed["u"] - fp64["u"]) / np.linalg.norm(fp64["u"]))
    _log("8^3 p=6 by preconditioned conjugate gradients")
    cg = {prec: time_cg(res[prec]["prob"], res[prec]["b"]) for prec in ("mixed", "fp64")}
    _log("8^3 p=6 by restarted FGMRES(4)")
    rprob, rb, _ = build_c2(dg, "mixed", restart=4)
    _, rst, rtimes, _ = time_solves(rprob, rb, 10, 2)
    restarted = dict(restart=4, ms_p50=round(1e3 * _pct(rtimes, 50), 3),
                     iterations=rst["iterations"], rel_residual=rst["rel_residual"],
                     converged=rst["converged"])
    rprob.close()
    _log("8^3 p=6 with the W-cycle")
    wprob, wb, _ = build_c2(dg, "mixed", cycle=2)
    _, wst, wtimes, _ = time_solves(wprob, wb, 10, 2)
    wcycle = dict(ms_p50=round(1e3 * _pct(wtimes, 50), 3), iterations=wst["iterations"],
                  rel_residual=wst["rel_residual"], converged=wst["converged"])
    wprob.close()
    _log("8^3 p=6 with the F-cycle")
    fprob, fb, _ = build_c2(dg, "mixed", cycle=3)
    _, fst, ftimes, _ = time_solves(fprob, fb, 10, 2)
    fcycle = dict(ms_p50=round(1e3 * _pct(ftimes, 50), 3), iterations=fst["iterations"],
                  rel_residual=fst["rel_residual"], converged=fst["converged"])
    fprob.close()
    _log("8^3 p=6 with additive multigrid")
    aprob, ab, _ = build_c2(dg, "mixed", additive=1)
    _, ast_, atimes, _ = time_solves(aprob, ab, 10, 2)
    additive = dict(ms_p50=round(1e3 * _pct(atimes, 50), 3), iterations=ast_["iterations"],
                    rel_residual=ast_["rel_residual"], converged=ast_["converged"])
    aprob.close()
    _log("subdomain GEMM and apply timings")
    gemm = time_subdomain_gemm(mixed["prob"])
    apply_c2 = time_apply(dg, (8, 8, 8), 6)
    apply_c5 = time_apply(dg, (16, 16, 16), 7)
    # every degree at about 2 M DOFs (n^3 (p+1)^3)
    sweep = {}
    for p, n in ((3, 32), (4, 25), (5, 21), (6, 18), (7, 16), (8, 14)):
        r = time_apply(dg, (n, n, n), p, reps=50, warm=5)
        sweep[f"p{p}_{n}^3"] = dict(ndof=r["ndof"], gdofs=round(r["gdofs"], 1),
                                    achieved_gbs=round(r["achieved_gbs"], 1),
                                    launch_shape=r["launch_shape"])
    apply_big = None if args.no_large_apply else time_apply(dg, (40, 40, 40), 7, reps=50,
                                                             calibration_copy=True,
                                                             shape=args.apply_shape)
    roofline = {"bound": "mfma", "achieved": round(gemm["achieved_tflops"], 2),
                "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(gemm["achieved_tflops"] / MFMA_FP32_PEAK_TFLOPS, 4),
                "traffic": measured_traffic("subdomain_gemm"),
                "kernel": "grouped subdomain-solve GEMM (FP32 MFMA) of one Schwarz sweep on the "
                          "8^3 p=6 fine level, 2 sum_S n_S^2 = "
                          f"{gemm['flops_per_launch']:.4g} flop per launch, tile variant "
                          f"{mixed['prob'].gemm_variant(0)}",
                "gemm_variant": mixed["prob"].gemm_variant(0),
                "ms_per_launch": round(gemm["ms_per_launch"], 5)}
    roof_src = apply_big or apply_c5
    roofline_apply = {"bound": "hbm", "achieved": round(roof_src["achieved_gbs"], 1),
                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(roof_src["achieved_gbs"] / HBM_PEAK_GBS, 4),
                      "traffic": measured_traffic("apply") if apply_big else None,
                      "kernel": f"DG operator apply, {roof_src['elements']} elements "
                                f"p={roof_src['p']}, 16 B/DOF algorithmic (read u, write Au), "
                                "launch shape " + ("2x2x2 element bricks" if roof_src["launch_shape"] < 0
                                                   else f"{roof_src['launch_shape']} elements/workgroup"
                                                   " (0: default)"),
                      "ms_per_launch": round(roof_src["ms_per_apply"], 5)}
    roofline_apply["launch_shape"] = roof_src["launch_shape"]
    if apply_big:
        roofline_apply["calibration_copy_bytes"] = 8 * apply_big["ndof"]
    ceil = None if args.no_ceilings else measured_ceilings()
    if ceil:
        roofline["measured_ceiling"] = {
            "what": "FP32 8192^3 torch.matmul (vendor BLAS) on this GPU", "unit": "TFLOP/s",
            "value": round(ceil["fp32_gemm_tflops"], 1),
            "frac": round(gemm["achieved_tflops"] / ceil["fp32_gemm_tflops"], 4)}
        roofline_apply["measured_ceiling"] = {
            "what": "device-to-device copy of 512 MiB on this GPU (read + write)", "unit": "GB/s",
            "value": round(ceil["copy_gbs"], 1),
            "frac": round(roof_src["achieved_gbs"] / ceil["copy_gbs"], 4)}

    if not args.no_c5:
        _log("16^3 p=7 solves")
    c5 = None if args.no_c5 else time_c5(dg)
    if not args.no_serving:
        _log(f"serving stream of {args.serve_requests} requests")
    serving = None if args.no_serving else run_serving(dg, args.serve_requests,
                                                          host_threads=args.serve_threads)

    cpu = None
    u_oracle = None
    if not args.no_cpu_baseline:
        _log("oracle on the host CPU")
        cpu, u_oracle = cpu_baseline()

    out = {
        "metric": METRIC,
        "value": round(args.steps / mixed["total"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * mixed["total"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mfma subdomain solves + f64",
        "data": "synthetic",
        "config": {"workload": "3D Poisson [0,1]^3, 8x8x8 elements, p=6 (175616 DOFs), 16-mode "
                               "random-Fourier source seed 2, C=1.5, 3-level MG-Schwarz FGMRES, "
                               "rtol 1e-10",
                   "global_batch": 1, "parallelism": "single GPU"},
        "solve_ms_mixed": {"p50": round(1e3 * _pct(mixed["times"], 50), 3),
                           "p99": round(1e3 * _pct(mixed["times"], 99), 3)},
        "solve_ms_fp64": {"p50": round(1e3 * _pct(fp64["times"], 50), 3),
                          "p99": round(1e3 * _pct(fp64["times"], 99), 3)},
        "speedup_mixed_vs_fp64_p50": round(_pct(fp64["times"], 50) / _pct(mixed["times"], 50), 3),
        "iterations": {"mixed": mixed["stats"]["iterations"], "fp64": fp64["stats"]["iterations"]},
        "rel_residual": {"mixed": mixed["stats"]["rel_residual"], "fp64": fp64["stats"]["rel_residual"]},
        "mixed_vs_fp64_solution_rel_diff": sol_diff,
        "rms_error_vs_exact": {"mixed": mixed["err_exact"], "fp64": fp64["err_exact"]},
        "setup_s": {"mixed": round(mixed["setup_s"], 3), "fp64": round(fp64["setup_s"], 3)},
        "apply": {"c2_shape": apply_c2, "16^3_p7": apply_c5, "40^3_p7": apply_big,
                  "sweep_2M_dofs": sweep},
        "c2_conjugate_gradients": cg,
        "c2_restarted_fgmres_mixed": restarted,
        "c2_wcycle_mixed": wcycle,
        "c2_fcycle_mixed": fcycle,
        "c2_additive_mg_mixed": additive,
        "c5_16x16x16_p7": c5,
        "serving": serving,
        "roofline": roofline,
        "roofline_apply": roofline_apply,
        "cpu_baseline": cpu,
    }
    if u_oracle is not None:
        out["fp64_vs_oracle_solution_rel_diff"] = float(
            np.linalg.norm(fp64["u"] - u_oracle) / np.linalg.norm(u_oracle))
        out["mixed_vs_oracle_solution_rel_diff"] = float(
            np.linalg.norm(mixed["u"] - u_oracle) / np.linalg.norm(u_oracle))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
