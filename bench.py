"""Benchmark of the DG multigrid-Schwarz solver on one MI355X.

Headline workload (one step = one full solve to a 1e-10 relative residual):
  3D Poisson on [0,1]^3, 16x16x16 elements, p = 7 (2,097,152 DOFs), source
  from 16 seeded random Fourier modes (seed 5), homogeneous Dirichlet,
  penalty C = 1.5, 4-level multigrid V-cycle with 3+3 additive Schwarz steps
  (overlap 2) preconditioning flexible GMRES, every step in FP64.  The
  mixed-precision solver (FP32 MFMA subdomain solves, FP64 everywhere else)
  is timed beside it on the same inputs, to the same true residual.

Also measured:
  * the 2x2x2, p = 3 manufactured-solution solve (FP64), the 8x8x8, p = 6
    Fourier solve (FP64 and mixed) and its Krylov/cycle variants, the 6^3,
    p = 7 puncture Newton-Krylov solve (FP64 and mixed), and the serving
    stream of 256 requests;
  * operator-apply throughput (GDOF/s) with HIP events on the stream the
    kernel runs on, on the solve shapes, every p = 3..8 at about 2 M DOFs,
    and a 40^3, p = 7 shape whose vectors (262 MB) exceed the 256 MB
    Infinity Cache;
  * the ceilings the GPU reaches outside the library (a 512 MiB copy, an
    FP32 torch.matmul) beside the vendor peaks;
  * the oracle on the host CPU (cpu_baseline leg, a child process started
    before the GPU is touched): one V-cycle and one operator apply of the
    headline workload at 1 thread and at all cores, and the oracle's check of
    the GPU solutions (residuals through the oracle's own operator, the
    oracle's solution of the 2x2x2 case).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time to 1e-10 rel residual & DG apply GDOF/s; mixed vs FP64; p50/p99"
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_FP64_PEAK_TFLOPS = 78.6

C5 = dict(lower=(0, 0, 0), upper=(1, 1, 1), elements=(16, 16, 16), p=7, levels=4)
C2 = dict(lower=(0, 0, 0), upper=(1, 1, 1), elements=(8, 8, 8), p=6, levels=3)
C1 = dict(lower=(0, 0, 0), upper=(1, 1, 1), elements=(2, 2, 2), p=3, levels=2)
C3 = dict(lower=(-20, -20, -20), upper=(20, 20, 20), elements=(6, 6, 6), p=7, levels=2)

# HBM traffic per launch of the two roofline kernels, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs of this script, each scaled by what the same
# counter reads for the plain copy of the calibration bytes made below.  A
# figure is reported only while the sources it was measured on are unchanged.
MEASURED_TRAFFIC = {
    # the 16^3 p=7 FP64 fine-level GEMM, per tile variant (FETCH_SIZE KiB x
    # 1.99981 + WRITE_SIZE KiB): v0 k_sub_gemm<double, 2, 2, 1, 4, 16> 329993.7
    # + 39936.0; v1 <2, 2, 2, 4> 257093.4 + 80896.0; v2 <2, 2, 1, 2> 322041.5 +
    # 39936.0; v3 k_sub_gemm_db<double, 2, 2, 2, 2, 16> 258727.6 + 40448.0;
    # v4 k_sub_gemm_db<double, 2, 2, 1, 2, 16> 310040.1 + 39936.0
    "subdomain_gemm": {"sources": ["paper_2111_06767_amd/csrc/dgs_schwarz.hip",
                                   "paper_2111_06767_amd/csrc/dgs_internal.h"],
                       "sha256": "9f082964d70abd00e4cbcbbe58d8115eb0ad696728b23c76bdaaf50fce0348ba",
                       "bytes": {0: 716658737, 1: 609315841, 2: 700374145, 3: 571243620, 4: 675797563}},
    # the 40^3 p=7 apply per launch shape (k_apply<8, epb, 0, 0, brick, true>,
    # non-temporal stores): bricks (-1) 181232.1 + 256028.8, one element per
    # workgroup 181320.1, two 181312.5, four 181312.6 KiB fetched x 1.99982,
    # each + 256000.0 KiB written
    "apply": {"sources": ["paper_2111_06767_amd/csrc/dgs_apply.hip",
                          "paper_2111_06767_amd/csrc/dgs_elem.h",
                          "paper_2111_06767_amd/csrc/dgs_internal.h"],
              "sha256": "ef2f59d67748230c12f631ee4c19ec8cd2fd13e162e7b1790380da014a5b4985",
              "bytes": {-1: 633303488, 1: 633454205, 2: 633438641, 4: 633438846}},
}


def _sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, choice):
    """Counted bytes per launch, if measured on these sources for this tile
    variant / launch shape (the autotuner's choice of the run)."""
    t = MEASURED_TRAFFIC[kernel]
    if choice not in t["bytes"] or _sources_sha256(t["sources"]) != t["sha256"]:
        return None
    return t["bytes"][choice]


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def _ms(times):
    return {"p50": round(1e3 * _pct(times, 50), 3), "p99": round(1e3 * _pct(times, 99), 3)}


# ---------------------------------------------------------------------------
# cpu_baseline leg: the oracle in a child process
# ---------------------------------------------------------------------------
def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_child():
    """The cpu_baseline leg (runs in its own process, started by the parent
    before it touches the GPU).  Waits for the parent's GPU solutions (a .npz
    path on stdin, sent once every GPU leg is over), builds the oracle's
    V-cycle of the headline workload, checks the solutions through the
    oracle, then times one V-cycle and one operator apply at 1 thread and at
    all cores.  Prints one JSON line."""
    from threadpoolctl import threadpool_info, threadpool_limits

    import workloads as W
    from oracle import krylov, mesh, multigrid, newton, operator

    def log(msg):
        print(f"[bench:cpu] {msg}", file=sys.stderr, flush=True)

    n_all = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    # nothing runs here until the parent's GPU legs are over: the oracle's
    # multi-threaded set-up would otherwise compete with the host thread that
    # launches the GPU work, and stretch the timed GPU legs
    line = sys.stdin.readline().strip()
    if not line:
        return
    path, iters = line.split()
    iters = int(iters)
    t0 = time.perf_counter()
    m5 = mesh.BoxMesh(C5["lower"], C5["upper"], C5["elements"], C5["p"])
    x, y, z = m5.node_coordinates()
    b5 = operator.apply_mass(m5, W.fourier_source(W.fourier_modes(W.SEED_C5), x, y, z)).reshape(-1)
    log("building the oracle's 16^3 p=7 hierarchy")
    V5 = multigrid.VCycle(m5, 1.5, levels=C5["levels"],
                          on_level=lambda l, m: log(f"level {l} ({m.n} elements) set up"))
    t_setup = time.perf_counter() - t0
    log(f"oracle set-up done in {t_setup:.1f} s")
    data = np.load(path)
    checks = {}

    def A(m):
        N = m.N
        return lambda v: operator.apply_operator(m, v.reshape(m.E, N, N, N), 1.5).reshape(-1)

    # the GPU solutions through the oracle's own operator
    nb5 = np.linalg.norm(b5)
    A5 = A(m5)
    for prec in ("fp64", "mixed"):
        key = f"c5_{prec}"
        if key in data:
            checks[f"c5_{prec}_oracle_rel_residual"] = float(np.linalg.norm(b5 - A5(data[key])) / nb5)
    m2 = mesh.BoxMesh(C2["lower"], C2["upper"], C2["elements"], C2["p"])
    x, y, z = m2.node_coordinates()
    b2 = operator.apply_mass(m2, W.fourier_source(W.fourier_modes(W.SEED_C2), x, y, z)).reshape(-1)
    for prec in ("fp64", "mixed"):
        key = f"c2_{prec}"
        if key in data:
            checks[f"c2_{prec}_oracle_rel_residual"] = float(
                np.linalg.norm(b2 - A(m2)(data[key])) / np.linalg.norm(b2))
    m1 = mesh.BoxMesh(C1["lower"], C1["upper"], C1["elements"], C1["p"])
    x, y, z = m1.node_coordinates()
    b1 = operator.apply_mass(m1, W.sin_product_source(x, y, z)).reshape(-1)
    u1, its1, _ = krylov.fgmres(A(m1), b1, precondition=multigrid.VCycle(m1, 1.5, levels=2),
                                rtol=1e-10)
    if "c1_fp64" in data:
        checks["c1_fp64_vs_oracle_solution_rel_diff"] = float(
            np.linalg.norm(data["c1_fp64"] - u1) / np.linalg.norm(u1))
        checks["c1_oracle_iterations"] = int(its1)
    m3 = mesh.BoxMesh(C3["lower"], C3["upper"], C3["elements"], C3["p"])
    x, y, z = m3.node_coordinates()
    al, be = W.puncture_background(W.puncture_params(W.SEED_C3), x, y, z)
    al, be = al.reshape(-1), be.reshape(-1)
    N3 = m3.N

    def F3(v):
        src = newton.puncture_source(al, be, v).reshape(m3.E, N3, N3, N3)
        return operator.apply_operator(m3, v.reshape(m3.E, N3, N3, N3), 1.5, source=src).reshape(-1)

    r30 = np.linalg.norm(F3(np.zeros(m3.ndof)))
    for prec in ("fp64", "mixed"):
        key = f"c3_{prec}"
        if key in data:
            checks[f"c3_{prec}_oracle_rel_nonlinear_residual"] = float(np.linalg.norm(F3(data[key])) / r30)
    served = []
    reqs = W.request_stream(256, rate=1.0)
    for key in sorted(k for k in data.files if k.startswith("serve_")):
        r = reqs[int(key.split("_")[1])]
        ms = mesh.BoxMesh((0, 0, 0), (r.side,) * 3, r.elements, r.p)
        xs, ys, zs = ms.node_coordinates()
        fs = W.fourier_source(W.fourier_modes(r.seed, (0, 0, 0), (r.side,) * 3), xs, ys, zs)
        bs = operator.apply_mass(ms, fs).reshape(-1)
        served.append(float(np.linalg.norm(bs - A(ms)(data[key])) / np.linalg.norm(bs)))
    if served:
        checks["served_sample_oracle_rel_residual_max"] = max(served)
        checks["served_sample_size"] = len(served)
    log("oracle checks of the GPU solutions done; timing one V-cycle + apply")

    def one_pass():
        ta = time.perf_counter()
        zz = V5(b5)
        A5(zz)
        return time.perf_counter() - ta

    legs = {}
    for threads in (n_all, 1):
        with threadpool_limits(limits=threads):
            used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
            t = one_pass()
        legs[threads] = (t, used)
        log(f"{threads} thread(s): {t:.1f} s per V-cycle + apply")
    t_all, used_all = legs[n_all]
    t_one, _ = legs[1]
    sample = (f"one oracle V-cycle and one operator apply of the 16^3 p=7 headline workload "
              f"(FP64, {m5.ndof} DOFs), extrapolated by the {iters} FGMRES iterations of the "
              f"GPU FP64 solve; Gram-Schmidt and the oracle's set-up ({t_setup:.0f} s) not counted")
    out = dict(value=1.0 / (iters * t_all), unit="solves/s", cores=int(used_all), kind="oracle",
               sample=sample, cpu_model=_cpu_model(), seconds_per_vcycle_and_apply=round(t_all, 2),
               one_thread={"value": 1.0 / (iters * t_one), "cores": 1,
                           "seconds_per_vcycle_and_apply": round(t_one, 2)},
               oracle_checks=checks)
    print(json.dumps(out), flush=True)


def start_cpu_child():
    env = dict(os.environ)
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child"],
                            stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)


def finish_cpu_child(child, solutions, iters):
    path = os.path.join(tempfile.gettempdir(), f"dgs_bench_{os.getpid()}.npz")
    np.savez(path, **solutions)
    try:
        child.stdin.write(f"{path} {iters}\n")
        child.stdin.flush()
        out, _ = child.communicate(timeout=1200)
    finally:
        try:
            os.remove(path)
        except OSError:
            pass
    lines = [ln for ln in out.splitlines() if ln.startswith("{")]
    if child.returncode != 0 or not lines:
        raise RuntimeError(f"cpu_baseline child failed (exit {child.returncode})")
    return json.loads(lines[-1])


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------
def build_fourier(dg, cfg, seed, precision, **opts):
    import torch
    import workloads as W
    prob = dg.Problem(cfg["lower"], cfg["upper"], cfg["elements"], cfg["p"], penalty=1.5,
                      mg_levels=cfg["levels"], precision=precision, **opts)
    xyz = prob.node_coordinates()
    modes = W.fourier_modes(seed)
    x, y, z = (xyz[d].cpu().numpy() for d in range(3))
    f = torch.as_tensor(W.fourier_source(modes, x, y, z)).cuda()
    b = prob.apply_mass(f)
    uex = W.fourier_solution(modes, x, y, z)
    return prob, b, uex


def time_solves(prob, b, steps, warmup, cg=False):
    import torch
    u = torch.zeros_like(b)
    solve = prob.solve_cg if cg else prob.solve
    for _ in range(warmup):
        u.zero_()
        solve(b, u)
    torch.cuda.synchronize()
    times, stats = [], None
    t_all = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, stats = solve(b, u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    total = time.perf_counter() - t_all
    return u, stats, times, total


def solve_leg(dg, cfg, seed, precision, steps, warmup, **opts):
    prob, b, uex = build_fourier(dg, cfg, seed, precision, **opts)
    u, st, times, total = time_solves(prob, b, steps, warmup)
    un = u.cpu().numpy()
    return dict(prob=prob, b=b, u=un, stats=st, times=times, total=total,
                rms_err=float(np.sqrt(np.mean((un - uex) ** 2))), setup_s=st["t_setup_s"])


def summary(leg):
    st = leg["stats"]
    return dict(ms=_ms(leg["times"]), iterations=st["iterations"],
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


def system_leg(dg, precision, laplacian_bc, k, steps=5, warmup=1):
    """A coupled system of five variables on 8^3 elements, p = 6 (the shape
    of the linearised XCTS equations of Sec. IV.B on a flat box: variable 0
    with Neumann faces x-, y-, z-, variable 2 with Neumann face x+, the others
    Dirichlet; pointwise couplings D_ab = M c_ab), solved by FGMRES with the
    system V-cycle whose subdomain problems take k GMRES iterations with the
    matched or the Dirichlet Laplacian approximation."""
    import torch
    import workloads as W
    nv = len(W.SYSTEM_NEUMANN)
    el, p = C2["elements"], C2["p"]
    aux = dg.Problem(C2["lower"], C2["upper"], el, p, mg_levels=1)
    xyz = aux.node_coordinates()
    x, y, z = (xyz[d].cpu().numpy() for d in range(3))
    c = W.system_coupling(W.SEED_SYSTEM, nv, x, y, z)
    D = torch.empty(nv * nv * aux.ndof, dtype=torch.float64, device="cuda")
    for ab in range(nv * nv):
        aux.apply_mass(torch.as_tensor(c[ab // nv, ab % nv]).cuda(), out=D[ab * aux.ndof:(ab + 1) * aux.ndof])
    b = torch.empty(nv * aux.ndof, dtype=torch.float64, device="cuda")
    for a in range(nv):
        f = torch.as_tensor(W.fourier_source(W.fourier_modes(W.SEED_SYSTEM + 1 + a), x, y, z)).cuda()
        aux.apply_mass(f, out=b[a * aux.ndof:(a + 1) * aux.ndof])
    aux.close()
    S = dg.System(C2["lower"], C2["upper"], el, p, W.SYSTEM_NEUMANN, laplacian_bc=laplacian_bc,
                  mg_levels=C2["levels"], subdomain_iters=k, precision=precision, max_iter=100)
    S.set_coupling(D)
    u = torch.zeros_like(b)
    for _ in range(warmup):
        u.zero_()
        S.solve(b, u)
    times, st = [], None
    for _ in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = S.solve(b, u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    S.close()
    return dict(ms=_ms(times), iterations=st["iterations"], rel_residual=st["rel_residual"],
                converged=st["converged"])


def deformed_coordinates(dg, cfg, amplitude, elements=None, p=None):
    """Node coordinates of the box map x = X + a c prod_d sin(pi (X_d - lo_d)/L_d),
    c = (1, 0.7, 0.4) (the box boundary stays in place): a device tensor of
    3 * ndof (x, then y, then z)."""
    import torch
    el = elements or cfg["elements"]
    pp = p or cfg["p"]
    X = dg.points(cfg["lower"], cfg["upper"], el, pp)
    lo = np.asarray(cfg["lower"], float)
    L = np.asarray(cfg["upper"], float) - lo
    bump = np.prod([np.sin(np.pi * (X[d] - lo[d]) / L[d]) for d in range(3)], axis=0)
    xyz = X + amplitude * np.array([1.0, 0.7, 0.4])[:, None] * bump[None, :]
    return torch.as_tensor(xyz.reshape(-1)).cuda()


def curved_leg(dg, precision, amplitude=0.1, steps=10, warmup=2):
    """The 16^3 p=7 headline solve on a deformed grid: curved operator,
    V-cycle of the box grid as the preconditioner."""
    import torch
    import workloads as W
    prob = dg.Problem(C5["lower"], C5["upper"], C5["elements"], C5["p"], penalty=1.5,
                      mg_levels=C5["levels"], precision=precision)
    prob.set_geometry(deformed_coordinates(dg, C5, amplitude))
    xyz = deformed_coordinates(dg, C5, amplitude).view(3, -1)
    x, y, z = (xyz[d].cpu().numpy() for d in range(3))
    f = torch.as_tensor(W.fourier_source(W.fourier_modes(W.SEED_C5), x, y, z)).cuda()
    b = prob.apply_mass(f)
    u, st, times, total = time_solves(prob, b, steps, warmup)
    prob.close()
    return dict(ms=_ms(times), iterations=st["iterations"], rel_residual=st["rel_residual"],
                converged=st["converged"])


def metric_fields(xyz, cfg, amplitude):
    """g^ij (6 fields xx, xy, xz, yy, yz, zz) and sqrt(g) of the pullback
    metric of the box map with the given amplitude, at the node coordinates
    xyz (a device tensor of 3 * ndof): device tensors of 6 * ndof and ndof."""
    import torch
    import workloads as W
    X = xyz.view(3, -1).cpu().numpy()
    _, G, sg = W.pullback_metric(X, cfg["lower"], cfg["upper"], amplitude)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    return torch.as_tensor(six).cuda(), torch.as_tensor(sg).cuda()


def metric_leg(dg, precision, amplitude=0.1, metric_amplitude=0.15, steps=10, warmup=2):
    """The 16^3 p=7 headline solve on a deformed grid and a curved background
    metric (the pullback of the box map, amplitude 0.15, at the physical
    nodes): the Laplace-Beltrami operator with sqrt(g) in M, MD and ML,
    preconditioned by the box grid's flat V-cycle."""
    import torch
    import workloads as W
    prob = dg.Problem(C5["lower"], C5["upper"], C5["elements"], C5["p"], penalty=1.5,
                      mg_levels=C5["levels"], precision=precision)
    xyz = deformed_coordinates(dg, C5, amplitude)
    prob.set_geometry(xyz)
    six, sg = metric_fields(xyz, C5, metric_amplitude)
    prob.set_metric(six, sg)
    x, y, z = (xyz.view(3, -1)[d].cpu().numpy() for d in range(3))
    f = torch.as_tensor(W.fourier_source(W.fourier_modes(W.SEED_C5), x, y, z)).cuda()
    b = prob.apply_mass(f)
    u, st, times, total = time_solves(prob, b, steps, warmup)
    prob.close()
    return dict(ms=_ms(times), iterations=st["iterations"], rel_residual=st["rel_residual"],
                converged=st["converged"])


def lapse_leg(dg, precision, steps=3, warmup=1):
    """The lapse equation of the XCTS system on the Kerr-Schild background
    (psi = 1, shift fixed at its Kerr-Schild value) on one wedge of the shell
    (r from 2M to 10M) as 16^3 elements of p = 7: Newton with the power-law
    source c_-1/Phi + c_1 Phi + c_0 on the metric operator, Dirichlet data
    from the analytic lapse, flat initial guess Phi = 1, linear solves to
    1e-4 by FGMRES with the cube's V-cycle on the linearised operator."""
    import torch
    import workloads as W
    lower, upper = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    X = dg.points(lower, upper, C5["elements"], C5["p"])
    xyz = W.wedge_coordinates(X, 2.0, 10.0)
    G, sg, alpha, coefs, powers = W.kerr_schild_lapse(xyz)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    prob = dg.Problem(lower, upper, C5["elements"], C5["p"], penalty=1.5, mg_levels=C5["levels"],
                      precision=precision, subdomain_iters=3)
    prob.set_geometry(torch.as_tensor(xyz.reshape(-1)).cuda())
    prob.set_metric(torch.as_tensor(six).cuda(), torch.as_tensor(sg.reshape(-1)).cuda())
    cf = torch.as_tensor(coefs.reshape(-1)).cuda()
    ub = torch.as_tensor(alpha.reshape(-1)).cuda()
    u = torch.empty(prob.ndof, dtype=torch.float64, device="cuda")
    times, st = [], None
    for i in range(warmup + steps):
        u.fill_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = prob.newton_solve_powers(cf, powers, dirichlet=ub, u=u, newton_rtol=1e-10,
                                         linear_rtol=1e-4)
        torch.cuda.synchronize()
        if i >= warmup:
            times.append(time.perf_counter() - t0)
    err = float(np.abs(u.cpu().numpy() - alpha.reshape(-1)).max())
    prob.close()
    return dict(ms=_ms(times), newton_steps=st["newton_steps"], linear_iterations=st["iterations"],
                rel_residual=st["rel_residual"], converged=st["converged"],
                max_error_vs_analytic_lapse=err)


def xcts_leg(dg, precision, steps=2, warmup=1, laplacian_bc="matched", k=3, elements=None, p=None,
             levels=None):
    """The Hamiltonian and lapse equations of the XCTS system for psi and
    alpha psi on the Kerr-Schild background (shift held at its Kerr-Schild
    value) on one wedge (r from 2M to 10M) as 16^3 elements of p = 7: psi
    Neumann at the inner sphere (Sec. IV.B), Dirichlet data from the analytic
    solution elsewhere, flat initial guess; the system Newton with the
    BC-matched Laplacian approximation in the system V-cycle."""
    import torch
    import workloads as W
    lower, upper = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    elements = elements or C5["elements"]
    p = p or C5["p"]
    levels = levels or C5["levels"]
    X = dg.points(lower, upper, elements, p)
    xyz = W.wedge_coordinates(X, 2.0, 10.0)
    G, sg, alpha, terms = W.kerr_schild_xcts(xyz)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    S = dg.System(lower, upper, elements, p, [(4,), ()], laplacian_bc=laplacian_bc, penalty=1.5,
                  mg_levels=levels, precision=precision, subdomain_iters=k)
    S.set_geometry(torch.as_tensor(xyz.reshape(-1)).cuda())
    S.set_metric(torch.as_tensor(six).cuda(), torch.as_tensor(sg.reshape(-1)).cuda())
    n = S.ndof
    vars_ = [a for a in range(2) for _ in terms[a]]
    powers = [k for a in range(2) for _, k in terms[a]]
    coef = torch.as_tensor(np.concatenate([np.asarray(c, float).reshape(-1)
                                           for a in range(2) for c, _ in terms[a]])).cuda()
    ub = torch.as_tensor(np.concatenate([np.ones(n), alpha.reshape(-1)])).cuda()
    u = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    times, st = [], None
    for i in range(warmup + steps):
        u.fill_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = S.newton_solve_powers(coef, vars_, powers, dirichlet=ub, u=u, newton_rtol=1e-10,
                                      linear_rtol=1e-4)
        torch.cuda.synchronize()
        if i >= warmup:
            times.append(time.perf_counter() - t0)
    uh = u.cpu().numpy().reshape(2, n)
    S.close()
    return dict(ms=_ms(times), newton_steps=st["newton_steps"], linear_iterations=st["iterations"],
                rel_residual=st["rel_residual"], converged=st["converged"],
                max_error_psi=float(np.abs(uh[0] - 1.0).max()),
                max_error_lapse=float(np.abs(uh[1] - alpha.reshape(-1)).max()))


def wedge_leg(dg, precision, steps=5, warmup=1):
    """One wedge of the spherical shell of Sec. IV.B (r from 2 to 10,
    logarithmic radius, equiangular angles) as 16^3 elements of p = 7 on the
    logical cube [-1, 1]^3: the curved operator, FGMRES preconditioned by the
    cube's V-cycle, right-hand side M 1."""
    import torch
    import workloads as W
    lower, upper = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    X = dg.points(lower, upper, C5["elements"], C5["p"])
    xyz = torch.as_tensor(W.wedge_coordinates(X, 2.0, 10.0).reshape(-1)).cuda()
    prob = dg.Problem(lower, upper, C5["elements"], C5["p"], penalty=1.5, mg_levels=C5["levels"],
                      precision=precision)
    prob.set_geometry(xyz)
    b = prob.apply_mass(torch.ones(prob.ndof, dtype=torch.float64, device="cuda"))
    u, st, times, total = time_solves(prob, b, steps, warmup)
    prob.close()
    return dict(ms=_ms(times), iterations=st["iterations"], rel_residual=st["rel_residual"],
                converged=st["converged"])


def time_curved_apply(dg, elements, p, amplitude=0.1, metric_amplitude=None, reps=50, warm=5):
    """Curved-element apply (the gradient and operator kernels), HIP events;
    with metric_amplitude on the pullback background metric."""
    import torch
    import workloads as W
    cfg = dict(lower=(0, 0, 0), upper=(1, 1, 1), elements=elements, p=p)
    prob = dg.Problem(cfg["lower"], cfg["upper"], elements, p, mg_levels=1)
    xyz = deformed_coordinates(dg, cfg, amplitude)
    prob.set_geometry(xyz)
    if metric_amplitude is not None:
        prob.set_metric(*metric_fields(xyz, cfg, metric_amplitude))
    del xyz
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
    n = prob.ndof
    prob.close()
    del u, out
    torch.cuda.empty_cache()
    # algorithmic: read u and the element metric (9 inverse-Jacobian entries
    # and the determinant), write A u: 96 B per DOF; the background metric
    # adds g^ij (6), sqrt(g) and d ln sqrt(g) (3): 176 B per DOF
    bpd = 96 if metric_amplitude is None else 176
    return dict(elements=list(elements), p=p, ndof=n, ms_per_apply=ms, gdofs=n / (ms * 1e-3) / 1e9,
                algorithmic_bytes_per_dof=bpd, achieved_gbs=bpd * n / (ms * 1e-3) / 1e9)


def hp_workload():
    """hp-nonuniform mesh of the unit cube: 2 x 2 x 2 blocks in a checkerboard
    of refinement levels 3 (8^3 elements of degree 5) and 2 (4^3 elements of
    degree 7), so that every block face is nonconforming in both h and p:
    2304 elements, 573440 DOFs."""
    levels, degrees = [], []
    for b in range(8):
        fine = (b % 2 + (b // 2) % 2 + b // 4) % 2 == 0
        L = 3 if fine else 2
        levels.append((L, L, L))
        degrees += [(5, 5, 5) if fine else (7, 7, 7)] * (8 ** L)
    return levels, degrees


def hp_leg(dg, precision="fp64", steps=5, warmup=1, reps=50):
    """FGMRES with the hp V-cycle on the hp workload, and the hp operator
    apply timed with HIP events on the launch stream."""
    import torch
    import workloads as W
    levels, degrees = hp_workload()
    t0 = time.perf_counter()
    prob = dg.HpProblem((0, 0, 0), (1, 1, 1), (2, 2, 2), levels, degrees, penalty=1.5, mg_levels=4,
                        precision=precision)
    setup_s = time.perf_counter() - t0
    xyz = prob.node_coordinates()
    x, y, z = (xyz[d].cpu().numpy() for d in range(3))
    b = prob.apply_mass(torch.as_tensor(W.fourier_source(W.fourier_modes(W.SEED_C5), x, y, z)).cuda())
    u = torch.zeros_like(b)
    for _ in range(warmup):
        u.zero_()
        prob.solve(b, u)
    times, st = [], None
    for _ in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st = prob.solve(b, u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    out = torch.empty_like(b)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        prob.apply(b, out)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n = prob.ndof
    res = dict(elements=len(degrees), ndof=n, levels=prob.levels,
               subdomain_inverses_per_level=[prob.num_classes(l) for l in range(prob.levels)],
               setup_s=round(setup_s, 3), ms=_ms(times), iterations=st["iterations"],
               rel_residual=st["rel_residual"], converged=st["converged"],
               apply=dict(ms_per_apply=round(ms, 5), gdofs=round(n / (ms * 1e-3) / 1e9, 2),
                          achieved_gbs=round(16 * n / (ms * 1e-3) / 1e9, 1)))
    prob.close()
    return res


def newton_leg(dg, precision, steps=10, warmup=2):
    """The 6^3, p = 7 puncture problem on [-20, 20]^3 by Newton-Krylov with the
    multigrid-Schwarz preconditioner (subdomain GMRES(3))."""
    import torch
    import workloads as W
    prob = dg.Problem(C3["lower"], C3["upper"], C3["elements"], C3["p"], mg_levels=C3["levels"],
                      subdomain_iters=3, precision=precision)
    xyz = [v.cpu().numpy() for v in prob.node_coordinates()]
    al, be = W.puncture_background(W.puncture_params(W.SEED_C3), *xyz)
    al, be = torch.as_tensor(al).cuda(), torch.as_tensor(be).cuda()
    u = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        u.zero_()
        prob.newton_solve(al, be, u=u)
    times, st = [], None
    for _ in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = prob.newton_solve(al, be, u=u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    out = dict(ms=_ms(times), newton_steps=st["newton_steps"], linear_iterations=st["iterations"],
               backtracks=st["backtracks"], rel_nonlinear_residual=st["rel_residual"],
               converged=st["converged"], setup_s=round(st["t_setup_s"], 3))
    un = u.cpu().numpy()
    prob.close()
    return out, un


def run_serving(dg, n_requests=256, max_active=16, precision="mixed", host_threads=0,
                batched=True, paced=True, keep=8):
    """Poisson-process stream of solves (grids {2..6}^3, p in 3..8, cube sides
    1..4, random-Fourier sources): a closed-loop pass measures the saturation
    throughput, then requests arrive at 0.8 of it and p50/p99 latency and
    throughput are recorded.  batched: the cross-request batch engine (one
    launch per phase over all active requests), else one stream per request.
    Returns the summary and the solutions of the first `keep` requests of
    the paced pass (for the oracle's check)."""
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
                        host_threads=host_threads, batched=batched)
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
        counters = srv.counters() + srv.timings()
        srv.close()
        return n_requests / dt, its, counters

    cold_tput, _, _ = closed_loop()  # fills the inverse cache
    warm_tput, its, counters = closed_loop()
    summary = dict(requests=n_requests, precision=precision, max_active=max_active,
                   batched=batched, saturation_solves_per_s_cold_cache=round(cold_tput, 2),
                   saturation_solves_per_s=round(warm_tput, 2),
                   iterations_p50=float(np.median(its)), iterations_max=int(max(its)))
    steps, bsteps, launches, peak, t_work, t_issue, t_wait, t_host, t_ret = counters
    summary["host_seconds_warm_loop"] = dict(admission_setup_and_workers=round(t_work, 3),
                                             engine_issue=round(t_issue, 3),
                                             engine_wait=round(t_wait, 3),
                                             engine_host_part=round(t_host, 3),
                                             retire=round(t_ret, 3))
    if batched:
        summary["batch_engine"] = dict(steps=bsteps, launches_per_step=round(launches / max(bsteps, 1), 1),
                                       most_requests_per_step=peak)
    if not paced:
        return summary, {}
    rate = 0.8 * warm_tput
    gaps = np.array([r.arrival for r, _ in data]) / rate  # unit-rate arrivals rescaled
    srv = dg.Server(hbm_budget_bytes=64e9, max_active=max_active, precision=precision, max_iter=60,
                    host_threads=host_threads, batched=batched)
    t0 = time.perf_counter()
    nxt = 0
    index = {}
    peak_active = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < n_requests and gaps[nxt] <= now:
            r, f = data[nxt]
            index[srv.submit((0, 0, 0), (r.side,) * 3, r.elements, r.p, f)] = nxt
            nxt += 1
        a, q = srv.step()
        peak_active = max(peak_active, a)
        if nxt == n_requests and a == 0 and q == 0:
            break
        if a == 0 and q == 0 and nxt < n_requests:
            time.sleep(max(0.0, min(0.001, gaps[nxt] - (time.perf_counter() - t0))))
    makespan = time.perf_counter() - t0
    lat, conv, kept = [], 0, {}
    for rid in srv.finished():
        u, st, times = srv.fetch(rid)
        lat.append(times[2] - times[0])
        conv += int(st["converged"] and st["rel_residual"] <= 1e-10)
        if index[rid] < keep:
            kept[f"serve_{index[rid]}"] = u
    srv.close()
    summary.update(arrival_rate_per_s=round(rate, 2), solves_per_s=round(n_requests / makespan, 2),
                   latency_ms_p50=round(1e3 * _pct(lat, 50), 2),
                   latency_ms_p99=round(1e3 * _pct(lat, 99), 2),
                   converged_to_1e10=conv, peak_active=peak_active)
    return summary, kept


def roofline_kernels(args):
    """Counter-collection mode for rocprofv3 --pmc runs: the 16^3 p=7 FP64
    problem's set-up and 5 + 50 launches of its fine-level GEMM, then the
    40^3 p=7 apply timing followed by its calibration copy, and nothing else,
    so that each counter pass sees few dispatches.  Prints the two launch
    times (not a benchmark line)."""
    import torch
    import paper_2111_06767_amd as dg
    torch.cuda.set_device(0)
    prob, _, _ = build_fourier(dg, C5, 5, "fp64")
    if args.gemm_variant is not None:
        prob.set_gemm_variant(args.gemm_variant, level=0)
    gemm = time_subdomain_gemm(prob)
    variant = prob.gemm_variant(0)
    prob.close()
    ap = time_apply(dg, (40, 40, 40), 7, reps=50, calibration_copy=True, shape=args.apply_shape)
    print(json.dumps({"mode": "roofline kernels only", "gemm_variant": variant,
                      "gemm_ms_per_launch": gemm["ms_per_launch"],
                      "gemm_tflops": gemm["achieved_tflops"], "apply_shape": ap["launch_shape"],
                      "apply_ms": ap["ms_per_apply"], "calibration_copy_bytes": 8 * ap["ndof"]}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large-apply", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    # the ceiling measurements include large copies; counter runs that are
    # calibrated by the one 262 MB copy leave them out
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256)
    # host threads that issue the active requests' stages (0: the library default)
    ap.add_argument("--serve-threads", type=int, default=0)
    # pin the autotuned choices of the two roofline kernels (the headline FP64
    # problem's fine-level GEMM variant, the 40^3 p=7 apply's launch shape), so
    # that a profiled run launches the kernels an unprofiled run chose
    ap.add_argument("--gemm-variant", type=int, default=None)
    ap.add_argument("--apply-shape", type=int, default=None)
    # counter collection: only the launches the two roofline objects come from
    ap.add_argument("--roofline-kernels-only", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_child()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.roofline_kernels_only:
        roofline_kernels(args)
        return

    # the oracle's child starts before anything here touches the GPU
    child = None if args.no_cpu_baseline else start_cpu_child()

    import torch
    import paper_2111_06767_amd as dg
    torch.cuda.set_device(0)
    solutions = {}

    # -- headline: 16^3 p=7, FP64 and mixed ---------------------------------
    legs = {}
    for prec in ("fp64", "mixed"):
        _log(f"16^3 p=7 {prec}: set-up and {args.warmup}+{args.steps} solves")
        prob, b, uex = build_fourier(dg, C5, 5, prec)
        if prec == "fp64" and args.gemm_variant is not None:
            prob.set_gemm_variant(args.gemm_variant, level=0)
        u, st, times, total = time_solves(prob, b, args.steps, args.warmup)
        un = u.cpu().numpy()
        legs[prec] = dict(prob=prob, u=un, stats=st, times=times, total=total,
                          rms_err=float(np.sqrt(np.mean((un - uex) ** 2))), setup_s=st["t_setup_s"])
        solutions[f"c5_{prec}"] = un
    fp64, mixed = legs["fp64"], legs["mixed"]
    _log("16^3 p=7 subdomain GEMMs")
    gemm64 = time_subdomain_gemm(fp64["prob"])
    gemm32 = time_subdomain_gemm(mixed["prob"])
    variant64 = fp64["prob"].gemm_variant(0)
    variant32 = mixed["prob"].gemm_variant(0)
    headline_iters = fp64["stats"]["iterations"]
    for leg in legs.values():
        leg["prob"].close()

    # -- c1: 2^3 p=3 manufactured solution, FP64 -----------------------------
    _log("2^3 p=3 FP64 solves")
    import workloads as W
    p1 = dg.Problem(C1["lower"], C1["upper"], C1["elements"], C1["p"], penalty=1.5,
                    mg_levels=C1["levels"])
    xyz = p1.node_coordinates()
    b1 = p1.apply_mass(torch.as_tensor(W.sin_product_source(*(xyz[d].cpu().numpy() for d in range(3)))).cuda())
    u1, st1, t1, _ = time_solves(p1, b1, 50, 5)
    solutions["c1_fp64"] = u1.cpu().numpy()
    c1 = dict(ms=_ms(t1), iterations=st1["iterations"], rel_residual=st1["rel_residual"],
              converged=st1["converged"])
    p1.close()

    # -- c2: 8^3 p=6, FP64 and mixed, and its variants -----------------------
    c2 = {}
    for prec in ("fp64", "mixed"):
        _log(f"8^3 p=6 {prec}")
        leg = solve_leg(dg, C2, 2, prec, 20, 3)
        c2[prec] = summary(leg)
        c2[prec]["rms_error_vs_exact"] = leg["rms_err"]
        solutions[f"c2_{prec}"] = leg["u"]
        leg["prob"].close()
    c2["speedup_mixed_vs_fp64_p50"] = round(c2["fp64"]["ms"]["p50"] / c2["mixed"]["ms"]["p50"], 3)
    variants = None
    if not args.no_variants:
        variants = {}
        for name, opts in (("cg", dict(cg=True)), ("restarted_fgmres_4", dict(restart=4)),
                           ("wcycle", dict(cycle=2)), ("fcycle", dict(cycle=3)),
                           ("additive_mg", dict(additive=1))):
            _log(f"8^3 p=6 mixed, {name}")
            cg = opts.pop("cg", False)
            prob, b, _ = build_fourier(dg, C2, 2, "mixed", **opts)
            _, st, times, _ = time_solves(prob, b, 10, 2, cg=cg)
            variants[name] = dict(ms_p50=round(1e3 * _pct(times, 50), 3), iterations=st["iterations"],
                                  rel_residual=st["rel_residual"], converged=st["converged"])
            prob.close()

    # -- c3: puncture Newton-Krylov, FP64 and mixed ---------------------------
    c3 = {}
    for prec in ("fp64", "mixed"):
        _log(f"6^3 p=7 puncture Newton {prec}")
        c3[prec], solutions[f"c3_{prec}"] = newton_leg(dg, prec)
    c3["speedup_mixed_vs_fp64_p50"] = round(c3["fp64"]["ms"]["p50"] / c3["mixed"]["ms"]["p50"], 3)
    c3["mixed_vs_fp64_solution_rel_diff"] = float(
        np.linalg.norm(solutions["c3_mixed"] - solutions["c3_fp64"]) / np.linalg.norm(solutions["c3_fp64"]))

    # -- a coupled five-variable system: matched vs Dirichlet Laplacian approximation
    systems = None
    if not args.no_variants:
        systems = {}
        for k in (3, 1):
            for bc in ("matched", "dirichlet"):
                for prec in (("fp64", "mixed") if k == 3 else ("fp64",)):
                    _log(f"8^3 p=6 five-variable system, {bc} k={k} {prec}")
                    systems[f"k{k}_{bc}_{prec}"] = system_leg(dg, prec, bc, k)

    # -- curved elements: the headline solve on a deformed grid ----------------
    curved = None
    if not args.no_variants:
        curved = {}
        for prec in ("fp64", "mixed"):
            _log(f"16^3 p=7 deformed grid {prec}")
            curved[prec] = curved_leg(dg, prec)
        _log("curved apply 40^3 p=7")
        curved["apply_40^3_p7"] = time_curved_apply(dg, (40, 40, 40), 7)
        for prec in ("fp64", "mixed"):
            _log(f"wedge of a spherical shell, 16^3 p=7 {prec}")
            curved[f"wedge_16^3_p7_{prec}"] = wedge_leg(dg, prec)
        for prec in ("fp64", "mixed"):
            _log(f"16^3 p=7 deformed grid on a background metric {prec}")
            curved[f"metric_16^3_p7_{prec}"] = metric_leg(dg, prec)
        for prec in ("fp64", "mixed"):
            _log(f"Kerr-Schild lapse equation on a wedge, 16^3 p=7 {prec}")
            curved[f"kerr_schild_lapse_16^3_p7_{prec}"] = lapse_leg(dg, prec)
        for prec in ("fp64", "mixed"):
            _log(f"XCTS Hamiltonian and lapse equations on a wedge, 16^3 p=7 {prec}")
            curved[f"xcts_psi_lapse_16^3_p7_{prec}"] = xcts_leg(dg, prec)
        # the boundary-matched Laplacian approximation against the Dirichlet
        # one on the same solve, and one subdomain GMRES iteration instead of 3
        for bc, k in (("dirichlet", 3), ("matched", 1), ("dirichlet", 1)):
            _log(f"XCTS Hamiltonian and lapse, fp64, {bc} Laplacian approximation, k={k}")
            curved[f"xcts_psi_lapse_16^3_p7_fp64_{bc}_k{k}"] = xcts_leg(dg, "fp64", steps=1,
                                                                         laplacian_bc=bc, k=k)
        # scale independence: FGMRES iterations of the whole Newton solve as
        # the wedge is refined (p = 5, matched approximation, k = 1)
        scaling = {}
        for n, lv in ((4, 2), (8, 3), (16, 4), (32, 5)):
            _log(f"XCTS Hamiltonian and lapse, {n}^3 p=5 (scale independence)")
            r = xcts_leg(dg, "fp64", steps=1, k=1, elements=(n, n, n), p=5, levels=lv)
            scaling[f"{n}^3"] = {key: r[key] for key in ("ms", "newton_steps", "linear_iterations",
                                                          "max_error_psi", "max_error_lapse")}
        curved["xcts_psi_lapse_p5_refinement"] = scaling
        _log("curved apply on a background metric 24^3 p=7")
        curved["metric_apply_24^3_p7"] = time_curved_apply(dg, (24, 24, 24), 7, metric_amplitude=0.15)

    # -- hp-nonuniform mesh ---------------------------------------------------
    hp_out = None
    if not args.no_variants:
        hp_out = {}
        for prec in ("fp64", "mixed"):
            _log(f"hp-nonuniform mesh, 573440 DOFs, {prec}")
            hp_out[prec] = hp_leg(dg, prec)

    # -- applies --------------------------------------------------------------
    _log("operator applies")
    apply_c2 = time_apply(dg, (8, 8, 8), 6)
    apply_c5 = time_apply(dg, (16, 16, 16), 7)
    sweep = {}
    for p, n in ((3, 32), (4, 25), (5, 21), (6, 18), (7, 16), (8, 14)):
        r = time_apply(dg, (n, n, n), p, reps=50, warm=5)
        sweep[f"p{p}_{n}^3"] = dict(ndof=r["ndof"], gdofs=round(r["gdofs"], 1),
                                    achieved_gbs=round(r["achieved_gbs"], 1),
                                    launch_shape=r["launch_shape"])
    apply_big = None if args.no_large_apply else time_apply(dg, (40, 40, 40), 7, reps=50,
                                                             calibration_copy=True,
                                                             shape=args.apply_shape)

    serving = None
    if not args.no_serving:
        _log(f"serving stream of {args.serve_requests} requests (batched)")
        serving, kept = run_serving(dg, args.serve_requests, host_threads=args.serve_threads)
        solutions.update(kept)
        _log(f"serving stream of {args.serve_requests} requests (one stream per request)")
        serving["per_request_streams"], _ = run_serving(dg, args.serve_requests,
                                                        host_threads=args.serve_threads,
                                                        batched=False, paced=False)
    ceil = None if args.no_ceilings else measured_ceilings()

    roofline = {"bound": "mfma", "achieved": round(gemm64["achieved_tflops"], 2),
                "peak": MFMA_FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(gemm64["achieved_tflops"] / MFMA_FP64_PEAK_TFLOPS, 4),
                "traffic": measured_traffic("subdomain_gemm", variant64),
                "kernel": "grouped subdomain-solve GEMM (FP64 MFMA) of one Schwarz sweep on the "
                          "16^3 p=7 fine level, 2 sum_S n_S^2 = "
                          f"{gemm64['flops_per_launch']:.4g} flop per launch, tile variant {variant64}",
                "gemm_variant": variant64,
                "ms_per_launch": round(gemm64["ms_per_launch"], 5)}
    roofline_mixed_gemm = {"bound": "mfma", "achieved": round(gemm32["achieved_tflops"], 2),
                           "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(gemm32["achieved_tflops"] / MFMA_FP32_PEAK_TFLOPS, 4),
                           "kernel": "the same GEMM in FP32 (mixed-precision solver), tile variant "
                                     f"{variant32}",
                           "ms_per_launch": round(gemm32["ms_per_launch"], 5)}
    roof_src = apply_big or apply_c5
    roofline_apply = {"bound": "hbm", "achieved": round(roof_src["achieved_gbs"], 1),
                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(roof_src["achieved_gbs"] / HBM_PEAK_GBS, 4),
                      "traffic": (measured_traffic("apply", roof_src["launch_shape"])
                                  if apply_big else None),
                      "kernel": f"DG operator apply, {roof_src['elements']} elements "
                                f"p={roof_src['p']}, 16 B/DOF algorithmic (read u, write Au), "
                                f"launch shape {roof_src['launch_shape']}",
                      "gdofs": round(roof_src["gdofs"], 1),
                      "ms_per_launch": round(roof_src["ms_per_apply"], 5),
                      "launch_shape": roof_src["launch_shape"]}
    if apply_big:
        roofline_apply["calibration_copy_bytes"] = 8 * apply_big["ndof"]
    if ceil:
        roofline_mixed_gemm["measured_ceiling"] = {
            "what": "FP32 8192^3 torch.matmul (vendor BLAS) on this GPU", "unit": "TFLOP/s",
            "value": round(ceil["fp32_gemm_tflops"], 1),
            "frac": round(gemm32["achieved_tflops"] / ceil["fp32_gemm_tflops"], 4)}
        roofline_apply["measured_ceiling"] = {
            "what": "device-to-device copy of 512 MiB on this GPU (read + write)", "unit": "GB/s",
            "value": round(ceil["copy_gbs"], 1),
            "frac": round(roof_src["achieved_gbs"] / ceil["copy_gbs"], 4)}

    cpu = None
    if child is not None:
        _log("cpu_baseline leg: the oracle's checks and timing")
        cpu = finish_cpu_child(child, solutions, headline_iters)

    c5_out = {
        "solve_ms_fp64": _ms(fp64["times"]), "solve_ms_mixed": _ms(mixed["times"]),
        "speedup_mixed_vs_fp64_p50": round(_pct(fp64["times"], 50) / _pct(mixed["times"], 50), 3),
        "iterations": {"fp64": fp64["stats"]["iterations"], "mixed": mixed["stats"]["iterations"]},
        "rel_residual": {"fp64": fp64["stats"]["rel_residual"], "mixed": mixed["stats"]["rel_residual"]},
        "rms_error_vs_exact": {"fp64": fp64["rms_err"], "mixed": mixed["rms_err"]},
        "mixed_vs_fp64_solution_rel_diff": float(
            np.linalg.norm(mixed["u"] - fp64["u"]) / np.linalg.norm(fp64["u"])),
        "setup_s": {"fp64": round(fp64["setup_s"], 3), "mixed": round(mixed["setup_s"], 3)},
        "mixed_solves_per_s": round(args.steps / mixed["total"], 3),
    }
    if cpu:
        checks = cpu.get("oracle_checks", {})
        c5_out["oracle_rel_residual"] = {p: checks.get(f"c5_{p}_oracle_rel_residual")
                                         for p in ("fp64", "mixed")}
        for p in ("fp64", "mixed"):
            c2[p]["oracle_rel_residual"] = checks.get(f"c2_{p}_oracle_rel_residual")
            c3[p]["oracle_rel_nonlinear_residual"] = checks.get(f"c3_{p}_oracle_rel_nonlinear_residual")
        c1["vs_oracle_solution_rel_diff"] = checks.get("c1_fp64_vs_oracle_solution_rel_diff")
        if serving is not None and "served_sample_oracle_rel_residual_max" in checks:
            serving["oracle_check"] = {
                "sample": f"the first {checks['served_sample_size']} requests of the paced pass",
                "max_oracle_rel_residual": checks["served_sample_oracle_rel_residual_max"]}
        c1["oracle_iterations"] = checks.get("c1_oracle_iterations")

    out = {
        "metric": METRIC,
        "value": round(args.steps / fp64["total"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * fp64["total"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D Poisson [0,1]^3, 16x16x16 elements, p=7 (2097152 DOFs), 16-mode "
                               "random-Fourier source seed 5, C=1.5, 4-level multigrid V-cycle with "
                               "3+3 additive Schwarz steps (overlap 2) preconditioning FGMRES, "
                               "rtol 1e-10, FP64 throughout",
                   "global_batch": 1, "parallelism": "single GPU"},
        "c5_16x16x16_p7": c5_out,
        "c1_2x2x2_p3": c1,
        "c2_8x8x8_p6": c2,
        "c2_variants_mixed": variants,
        "c3_puncture_6x6x6_p7": c3,
        "system_5var_8x8x8_p6": systems,
        "curved_16x16x16_p7": curved,
        "hp_checkerboard_2304_elements": hp_out,
        "apply": {"c2_shape": apply_c2, "16^3_p7": apply_c5, "40^3_p7": apply_big,
                  "sweep_2M_dofs": sweep},
        "serving": serving,
        "roofline": roofline,
        "roofline_mixed_gemm": roofline_mixed_gemm,
        "roofline_apply": roofline_apply,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
