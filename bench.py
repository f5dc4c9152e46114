#!/usr/bin/env python3
"""Benchmark of the enriched Taylor-Hood Stokes solver on one MI355X.

Workload (one "step" = one complete preconditioned MINRES solve of an already
assembled, HBM-resident right-hand side to |eta|/gamma_1 <= 1e-6):
  Stokes lid-driven cavity on the unit square, n x n Q2 elements (default
  n = 256: 526k velocity, 66k Q1 + 65.5k P0 pressure unknowns), lid (1,0),
  f = 0, block-diagonal preconditioner = one geometric-multigrid V(2,2)
  Chebyshev-smoothed cycle for the velocity block + 20 Chebyshev-SGS steps for
  the singular pressure mass matrix with the null-vector projection.
  `value` is the mixed-precision solver (FP32 preconditioner inside FP64
  MINRES); the FP64 solver is timed on the same input and reported beside it.

Prints ONE JSON line.  --gpus N with N > 1 is refused: the solver runs on one
GPU (the method would shard by mesh blocks with halo exchanges).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = {"k_mq_cheb_fused": "k_mq.hip", "k_apply": "k_apply.hip", "k_cheb_step": "k_gmg.hip"}


def measured_traffic(kernel, n, variant):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a
    plain copy of known size), or None when there is none for this workload,
    the counters were read on another template variant (`variant`, the full
    kernel name), or the kernel source changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_stokes{n}_traffic.json")
    src = KERNEL_SOURCES.get(kernel)
    if not src or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2303_10233_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha or (variant and rec.get("kernel") != variant):
        return None
    return rec.get("bytes_per_launch")


def time_solves(P, b, steps, warmup, rtol, use_graph):
    import torch
    x = torch.empty_like(b)
    info = None
    for _ in range(warmup):
        _, info = P.solve(b, rtol=rtol, maxit=2000, use_graph=use_graph, out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(steps):
        _, info = P.solve(b, rtol=rtol, maxit=2000, use_graph=use_graph, out=x)
        its.append(info[0]["iterations"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, its, info


def cpu_identity():
    """What the host baseline ran on: core counts, affinity, CPU model and the
    BLAS / OpenMP thread settings."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    return {"os_cpu_count": os.cpu_count(), "affinity": affinity, "cpu_model": model,
            "thread_env": {k: v for k, v in env.items() if v is not None}}


def cpu_baseline(n, iterations_per_solve, cpu_iters):
    """The oracle (NumPy/SciPy, FP64, as it stands) on the same workload: a
    bounded sample of `cpu_iters` MINRES iterations with the same
    preconditioner algorithm, scaled to one solve by the GPU's iteration
    count."""
    from oracle.assemble import Mesh, System, lid_dirichlet
    from oracle.krylov import minres
    from oracle.precond import StokesBlockDiag

    t0 = time.perf_counter()
    m = Mesh(n)
    s = System(m)
    b = s.to_interior(s.rhs(None, lid_dirichlet(m)))
    # same Chebyshev-SGS interval as the GPU default: [min(0.01, 0.4/n), 1]
    P = StokesBlockDiag(s, "gmg", "cheb_sgs", mq_lo=min(0.01, 0.4 / n), mq_steps=20)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    minres(lambda v: s.K @ v, b, P, tol=1e-30, maxit=cpu_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / cpu_iters
    per_solve = per_iter * iterations_per_solve
    return {
        "value": 1.0 / per_solve,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "host": cpu_identity(),
        "sample": (f"{cpu_iters} MINRES iterations of the NumPy/SciPy oracle at n={n} "
                   f"(GMG V(2,2) + 20 Chebyshev-SGS steps, FP64; {dt:.1f} s, setup "
                   f"{t_setup:.1f} s excluded), scaled by the GPU iteration count "
                   f"{iterations_per_solve}; single-threaded SciPy sparse kernels"),
        "seconds_per_iteration": per_iter,
    }


def _pool_minres_sample(args):
    """Worker of the k-core oracle pool: MINRES iterations of the oracle at
    n x n with one Gaussian-bump forcing (GMG + Chebyshev-SGS, FP64)."""
    n, seed, iters = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)          # one core per worker: k workers on k cores
    from oracle.assemble import Mesh, System, lid_dirichlet
    from oracle.krylov import minres
    from oracle.precond import StokesBlockDiag
    from paper_2303_10233_amd.workloads import gaussian_bumps
    m = Mesh(n)
    s = System(m)
    b = s.to_interior(s.rhs(gaussian_bumps(n, seed), lid_dirichlet(m)))
    P = StokesBlockDiag(s, "gmg", "cheb_sgs", mq_lo=min(0.01, 0.4 / n), mq_steps=20)
    t0 = time.perf_counter()
    minres(lambda v: s.K @ v, b, P, tol=1e-30, maxit=iters)
    return time.perf_counter() - t0


def cpu_other(gpu):
    """Oracle baselines of the other configurations, timed on this host beside
    the GPU figures (`gpu`: the GPU results they are compared with):
    config 1 (16^2, exact velocity block, diagonal M_Q): direct solve with the
    factorisation and the solve timed apart, and the oracle's own MINRES;
    the 64-RHS batch at 128^2: a pool of k worker processes, each running a
    bounded MINRES sample, scaled to solves/s on k cores; Oseen 128^2
    (nu = 1/100): a bounded sample of the oracle's two-stage FGMRES with the
    GPU's inexact pieces, scaled by the GPU's iteration count.  The direct
    factorisation at 128^2 (SuperLU, about 250 s and 10-14 GB on the build
    host) does not fit the bench's time budget and is not run here."""
    import multiprocessing as mp
    import numpy as np
    from oracle.assemble import Mesh, System, lid_dirichlet, recirculating_wind
    from oracle.direct import BorderedLU, canonicalize, rel_err
    from oracle.krylov import minres
    from oracle import precond as opc
    out = {"host": cpu_identity()}
    # config 1
    m = Mesh(16)
    s = System(m)
    b = s.rhs(None, lid_dirichlet(m))
    t0 = time.perf_counter()
    lu = BorderedLU(s)
    t_fact = time.perf_counter() - t0
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        xd = canonicalize(lu.solve(b), m)
    t_solve = (time.perf_counter() - t0) / reps
    P = opc.StokesBlockDiag(s, "exact", "diag")
    t0 = time.perf_counter()
    _, info = minres(lambda v: s.K @ v, s.to_interior(b), P, tol=1e-6, maxit=3000)
    t_minres = time.perf_counter() - t0
    c1 = {"cores": 1, "direct_factor_s": round(t_fact, 4), "direct_solve_s": round(t_solve, 5),
          "direct_solves_per_s": round(1.0 / t_solve, 2), "minres_iterations": info["iterations"],
          "minres_s": round(t_minres, 3), "minres_solves_per_s": round(1.0 / t_minres, 2)}
    if gpu.get("c1_x") is not None:
        c1["gpu_rel_err_vs_direct"] = float(rel_err(gpu["c1_x"], xd))
    out["config1_stokes16"] = c1
    # 64-RHS batch at 128^2 on a pool of k cores
    k = max(1, min(8, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1))
    iters = 10
    with mp.get_context("fork").Pool(k) as pool:
        t0 = time.perf_counter()
        times = pool.map(_pool_minres_sample, [(128, 1000 + i, iters) for i in range(k)])
        wall = time.perf_counter() - t0
    per_iter = float(np.mean(times)) / iters
    its = gpu.get("batch64_iterations") or 62
    out["batch64_stokes128"] = {
        "cores": k, "solves_per_s": round(k / (per_iter * its), 4),
        "sample": (f"{k} processes (one BLAS thread each) x {iters} MINRES iterations of the oracle at "
                   f"128^2 (one bump forcing each, {wall:.1f} s wall with set-up), scaled by the GPU "
                   f"iteration count {its}"),
        "seconds_per_iteration": round(per_iter, 4)}
    # Oseen 128^2, nu = 1/100, two-stage with the GPU's inexact pieces
    n = 128
    m = Mesh(n, -1, 1, -1, 1)
    s = System(m, nu=0.01, wind=recirculating_wind(m))
    b = s.rhs(None, lid_dirichlet(m))
    vel, _ = opc.oseen_velocity_gmg(s)
    P1 = opc.PCDStage1Inexact(s, vel)
    P2 = opc.OseenM1(s, velocity_solve=vel, mq=opc.MQChebSGS(m, s.MQ, min(0.01, 0.4 / n), 1.0, 20))
    sample = 20
    t0 = time.perf_counter()
    opc.two_stage(s, b, eta=1e-30, maxit=sample // 2, stage1_prec=P1, stage2_prec=P2)
    dt = time.perf_counter() - t0
    its = gpu.get("oseen128_iterations") or 60
    out["oseen128_nu100"] = {"cores": 1, "solves_per_s": round(1.0 / (dt / sample * its), 5),
                             "sample": (f"{sample} two-stage FGMRES iterations of the oracle ({dt:.1f} s), "
                                        f"scaled by the GPU iteration count {its}"),
                             "seconds_per_iteration": round(dt / sample, 4)}
    # flow over a step, m = 32 (the paper's intermediate grid, 11264 squares):
    # a bounded sample of the oracle's two-stage FGMRES with the GPU's inexact
    # pieces; the wind is the channel profile (1 - y^2)/2 (the oracle's direct
    # Stokes solve at this size takes about 100 s, and the cost of an
    # iteration does not depend on the wind)
    from oracle import step as ostep
    sm = 32
    M = ostep.StepMesh(sm)
    X, Y = M.q2_coords()
    wind = np.concatenate([0.5 * (1.0 - Y ** 2), np.zeros(M.nv)])
    s = System(M, nu=0.02, wind=wind)
    b = s.rhs(None, ostep.inflow_dirichlet(M))
    vel, _ = ostep.velocity_gmg(s)
    P1 = ostep.PCDStage1(s, velocity_solve=vel, inexact=True)
    P2 = opc.OseenM1(s, velocity_solve=vel, mq=ostep.MQChebSGS(s))
    sample = 40
    t0 = time.perf_counter()
    ostep.two_stage(s, b, eta=1e-30, maxit=sample // 2, stage1_prec=P1, stage2_prec=P2)
    dt = time.perf_counter() - t0
    its = gpu.get("step32_iterations") or 150
    out["step32_nu50"] = {"cores": 1, "solves_per_s": round(1.0 / (dt / sample * its), 5),
                          "sample": (f"{sample} two-stage FGMRES iterations of the oracle at m = {sm} "
                                     f"({dt:.1f} s, channel-profile wind), scaled by the GPU iteration "
                                     f"count {its}"),
                          "seconds_per_iteration": round(dt / sample, 4)}
    return out


def bench_oseen(n, nu, prec, steps, rtol, maxit=1000, peclet_max=0.0):
    """Two-stage PCD FGMRES(50) on the recirculating-wind Oseen problem."""
    import torch
    from paper_2303_10233_amd import eth
    from paper_2303_10233_amd.workloads import recirculating_wind
    w = torch.as_tensor(recirculating_wind(n), dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    P = eth.Problem(n, domain=(-1.0, 1.0, -1.0, 1.0), nu=nu, kind=eth.OSEEN, wind=w, precision=prec,
                    gmg_peclet_max=peclet_max)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    b = P.assemble_rhs()
    x, info = P.solve(b, rtol=rtol, maxit=maxit, method=eth.TWO_STAGE, raise_on_error=False)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, info = P.solve(b, rtol=rtol, maxit=maxit, method=eth.TWO_STAGE, out=x, raise_on_error=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    i = info[0]
    P.close()
    return dict(n=n, nu=nu, solves_per_s=round(1.0 / dt, 4), ms_per_solve=round(1e3 * dt, 3),
                iterations=i["iterations"], stage1_iterations=i["stage1_iterations"],
                rel_residual=i["rel_residual_true"], status=i["status"], setup_s=round(setup, 3))


def bench_picard(n, nu, prec, steps, rtol, picard_steps=5, maxit=1000):
    """Enclosed flow on [-1, 1]^2 with the regularised lid 1 - x^4 (Re = 2/nu):
    Stokes start, `picard_steps` fixed-point steps (each a two-stage PCD
    solve from the previous iterate), then the Oseen system they produce is
    solved from zero `steps` times."""
    import torch
    from paper_2303_10233_amd import eth
    dom = (-1.0, 1.0, -1.0, 1.0)
    S = eth.Problem(n, domain=dom, nu=nu, corner_mode=2, precision=prec)
    x, _ = S.solve(S.assemble_rhs(), rtol=rtol, maxit=maxit)
    S.close()
    P = eth.Problem(n, domain=dom, nu=nu, kind=eth.OSEEN, wind=x[: 2 * (2 * n + 1) ** 2].contiguous(),
                    corner_mode=2, precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, pinfo = P.picard(x, picard_steps, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    t_picard = time.perf_counter() - t0
    b = P.assemble_rhs()
    y, info = P.solve(b, rtol=rtol, maxit=maxit)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        y, info = P.solve(b, rtol=rtol, maxit=maxit, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    i = info[0]
    P.close()
    return dict(n=n, nu=nu, reynolds=round(2.0 / nu, 3), solves_per_s=round(1.0 / dt, 4),
                ms_per_solve=round(1e3 * dt, 3), iterations=i["iterations"],
                stage1_iterations=i["stage1_iterations"], rel_residual=i["rel_residual_true"],
                status=i["status"], picard_seconds=round(t_picard, 4),
                picard_iterations=[p["iterations"] for p in pinfo])


def bench_step(m, prec, steps, rtol, picard_steps=5, maxit=2000):
    """Flow over a step (Sec. 3, the inflow-outflow example, nu = 1/50): the
    Stokes solution and `picard_steps` Picard steps on the GPU, then the
    Oseen system they produce solved from zero `steps` times by the
    two-stage PCD method; the volume flux through every vertical grid line
    of the solution against the inflow flux 2/3 (mass conservation)."""
    import numpy as np
    import torch
    from paper_2303_10233_amd import eth
    t0 = time.perf_counter()
    P = eth.StepProblem(m, nu=1.0 / 50, precision=prec)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, pinfo = P.picard(picard_steps, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    t_picard = time.perf_counter() - t0
    b = P.rhs()
    y, info = P.solve(b, rtol=rtol, maxit=maxit, raise_on_error=False)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        y, info = P.solve(b, rtol=rtol, maxit=maxit, out=y, raise_on_error=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    lay = eth.step_host_layout(m)
    yh = y.cpu().numpy()
    # flux through the vertical element lines by Simpson's rule on every edge
    nqx, nqy = 2 * 6 * m + 1, 4 * m + 1
    ux = np.zeros((nqy, nqx))
    ux[lay["q2_ij"][:, 1], lay["q2_ij"][:, 0]] = yh[: lay["nv"]]
    h = 1.0 / m
    fl = h / 6.0 * (ux[0:-1:2, 0::2] + 4.0 * ux[1::2, 0::2] + ux[2::2, 0::2]).sum(axis=0)
    P.close()
    return dict(m=m, nu=0.02, unknowns=lay["N"], elements=lay["n0"], solves_per_s=round(1.0 / dt, 4),
                ms_per_solve=round(1e3 * dt, 3), iterations=info["iterations"],
                stage1_iterations=info["stage1_iterations"], rel_residual=info["rel_residual_true"],
                status=info["status"], setup_s=round(setup, 3), picard_seconds=round(t_picard, 3),
                picard_iterations=[p["iterations"] for p in pinfo],
                max_flux_error=float(np.abs(fl - 2.0 / 3.0).max()))


def bench_batch(n, nrhs, prec, steps, rtol):
    """Lockstep MINRES over nrhs bump-forced right-hand sides on one mesh."""
    import torch
    from paper_2303_10233_amd import eth
    from paper_2303_10233_amd.workloads import gaussian_bumps
    P = eth.Problem(n, precision=prec, max_batch=nrhs)
    F = torch.stack([torch.as_tensor(gaussian_bumps(n, 1000 + k), dtype=torch.float64, device="cuda:0")
                     for k in range(nrhs)])
    B = P.assemble_rhs(F, batch=nrhs)
    X = torch.empty_like(B)
    P.solve(B, rtol=rtol, maxit=2000, use_graph=True, out=X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = P.solve(B, rtol=rtol, maxit=2000, use_graph=True, out=X)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    its = [i["iterations"] for i in info]
    P.close()
    return dict(n=n, rhs=nrhs, solves_per_s=round(nrhs / dt, 3), ms_per_batch=round(1e3 * dt, 3),
                iterations_max=max(its), iterations_min=min(its),
                all_converged=all(i["status"] == 0 for i in info))


def bench_ragged(prec, steps, rtol):
    """32 cavities n_i = 32 + 16 (i mod 15) solved together."""
    import torch
    from paper_2303_10233_amd import eth
    sizes = [32 + 16 * (i % 15) for i in range(32)]
    t0 = time.perf_counter()
    R = eth.RaggedBatch(sizes, precision=prec)
    setup = time.perf_counter() - t0
    bs = R.assemble_rhs()
    xs, infos = R.solve(bs, rtol=rtol, maxit=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xs, infos = R.solve(bs, rtol=rtol, maxit=2000, out=xs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # every member's iterations in one captured graph per chunk (use_graph = 2)
    xs, _ = R.solve(bs, rtol=rtol, maxit=2000, out=xs, use_graph=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xs, _ = R.solve(bs, rtol=rtol, maxit=2000, out=xs, use_graph=2)
    torch.cuda.synchronize()
    dt_joint = (time.perf_counter() - t0) / steps
    # the same problems one after another on one stream, for comparison
    t0 = time.perf_counter()
    for p, b, x in zip(R.problems, bs, xs):
        p.solve(b, rtol=rtol, maxit=2000, use_graph=True, out=x)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    dofs = sum(p.N for p in R.problems)
    R.close()
    return dict(cavities=len(sizes), total_dofs=dofs, solves_per_s=round(len(sizes) / dt, 3),
                ms_per_batch=round(1e3 * dt, 3), ms_joint_graph=round(1e3 * dt_joint, 3),
                ms_sequential=round(1e3 * seq, 3),
                iterations_max=max(i["iterations"] for i in infos),
                all_converged=all(i["status"] == 0 for i in infos), setup_s=round(setup, 2))


def bench_adjoint(kind, n, prec, steps, rtol):
    """One gradient evaluation = forward solve at f0 + misfit + adjoint solve +
    dJ/df + dJ/dnu, for J = 1/2 ||u - u_t||^2_{M_v} with u_t the solution for
    bumps(seed 5000) and f0 = 1/2 bumps(seed 4999)."""
    import torch
    from paper_2303_10233_amd import eth
    from paper_2303_10233_amd.workloads import gaussian_bumps, recirculating_wind
    if kind == "oseen":
        dom = (-1.0, 1.0, -1.0, 1.0)
        w = torch.as_tensor(recirculating_wind(n), dtype=torch.float64, device="cuda:0")
        P = eth.Problem(n, domain=dom, nu=0.01, kind=eth.OSEEN, wind=w, precision=prec)
    else:
        dom = (0.0, 1.0, 0.0, 1.0)
        P = eth.Problem(n, precision=prec)
    ft = torch.as_tensor(gaussian_bumps(n, 5000, *dom), dtype=torch.float64, device="cuda:0")
    f0 = torch.as_tensor(0.5 * gaussian_bumps(n, 4999, *dom), dtype=torch.float64, device="cuda:0")
    # MINRES replays captured iterations; FGMRES measured faster launched eagerly
    gr = kind == "stokes"
    xt, _ = P.solve(P.assemble_rhs(ft), rtol=rtol, maxit=2000, use_graph=gr)
    b0 = P.assemble_rhs(f0)

    def gradient():
        x, i1 = P.solve(b0, rtol=rtol, maxit=2000, use_graph=gr)
        J, g = P.misfit(x, xt)
        lam, i2 = P.solve_adjoint(g, rtol=rtol, maxit=2000, use_graph=gr)
        return P.grad_forcing(lam), P.grad_viscosity(lam, x), i1[0], i2[0]

    gradient()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gf, gnu, i1, i2 = gradient()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    P.close()
    return dict(kind=kind, n=n, gradients_per_s=round(1.0 / dt, 4), ms_per_gradient=round(1e3 * dt, 3),
                forward_iterations=i1["iterations"], adjoint_iterations=i2["iterations"],
                forward_status=i1["status"], adjoint_status=i2["status"], dJdnu=float(gnu))


def microbench(reps):
    """Kernel bandwidth at sizes whose vectors exceed the 256 MB Infinity Cache:
    Stokes n = 2048 (one FP64 vector 336 MB) and n = 512 x 16 right-hand sides,
    Oseen n = 2048.  Algorithmic bytes per launch / average launch time."""
    import torch
    from paper_2303_10233_amd import eth
    from paper_2303_10233_amd.workloads import recirculating_wind
    out = []
    stokes_k = [eth.K_SADDLE_APPLY, eth.K_CHEB_STEP, eth.K_RESTRICT, eth.K_PROLONG, eth.K_MQ_CHEB_STEP,
                eth.K_DOT, eth.K_MINRES_V, eth.K_MINRES_WX]
    cases = [("stokes", 2048, 1, eth.FP64), ("stokes", 2048, 1, eth.MIXED),
             ("stokes", 512, 16, eth.FP64), ("stokes", 512, 16, eth.MIXED),
             ("oseen", 2048, 1, eth.FP64), ("oseen", 2048, 1, eth.MIXED)]
    for kind, n, nrhs, prec in cases:
        if kind == "stokes":
            P = eth.Problem(n, precision=prec, max_batch=nrhs)
            ks = stokes_k if prec == eth.FP64 else [eth.K_CHEB_STEP, eth.K_RESTRICT, eth.K_PROLONG,
                                                     eth.K_MQ_CHEB_STEP]
        else:
            w = torch.as_tensor(recirculating_wind(n), dtype=torch.float64, device="cuda:0")
            P = eth.Problem(n, domain=(-1.0, 1.0, -1.0, 1.0), nu=0.01, kind=eth.OSEEN, wind=w,
                            precision=prec, max_batch=nrhs)
            ks = ([eth.K_OSEEN_APPLY, eth.K_CD_STEP, eth.K_GM_MDOT, eth.K_GM_MAXPY] if prec == eth.FP64
                  else [eth.K_CD_STEP])
        torch.cuda.synchronize()
        for k in ks:
            ms, by = P.profile_kernel(k, reps=reps, batch=nrhs)
            gbs = by / (ms * 1e-3) / 1e9
            out.append(dict(workload=f"{kind} n={n} rhs={nrhs}", precision="mixed" if prec else "fp64",
                            kernel=eth.KERNEL_NAMES[k], avg_us=round(1e3 * ms, 2), bytes=by,
                            gbs=round(gbs, 1), frac=round(gbs / MI355X_HBM_GBS, 4)))
            log(f"micro {kind} n={n} x{nrhs} {out[-1]['precision']} {out[-1]['kernel']}: "
                f"{out[-1]['avg_us']} us, {out[-1]['gbs']} GB/s")
        P.close()
        del P
        torch.cuda.empty_cache()
    return out


def counters_run(n, reps, tile, which="mq"):
    """The launches that the byte counters are read on (run under
    `rocprofv3 --pmc FETCH_SIZE` and then `--pmc WRITE_SIZE`), `reps` each,
    with plain copies of known size for the calibration (at n and at n = 2048:
    336 MB per vector, beyond every cache).
    which = "mq": the dominant kernel of the headline workload (the fused
    Chebyshev-SGS step, mixed, n x n).  The tile side of the fused step is
    fixed (`tile`, the one set-up picks for this workload when timed without
    a profiler: under the counters every launch is serialised and
    timing-based choices would differ between runs).
    which = "apply": the FP64 saddle apply with its fused dot at n = 2048, the
    stencil bandwidth figure (one 336 MB vector in, one out).
    which = "oseen": the Oseen saddle apply (FP64) and the damped-Jacobi F
    smoothing step (FP64 and FP32) at n = 2048.
    Prints the launch record the reduction script needs."""
    import torch
    from paper_2303_10233_amd import eth
    rec = {"n": n, "reps": reps, "launches": [], "which": which}
    if which == "apply":
        plan = ((2048, eth.FP64, (eth.K_SADDLE_APPLY, eth.K_COPY)),)
    elif which == "oseen":
        plan = ((2048, eth.FP64, (eth.K_OSEEN_APPLY, eth.K_CD_STEP, eth.K_COPY)),
                (2048, eth.MIXED, (eth.K_CD_STEP,)))
    else:
        plan = ((n, eth.MIXED, (eth.K_MQ_CHEB_STEP, eth.K_COPY)), (2048, eth.MIXED, (eth.K_COPY,)))
    for nn, prec, kernels in plan:
        if which == "oseen":
            from paper_2303_10233_amd.workloads import recirculating_wind
            w = torch.as_tensor(recirculating_wind(nn), dtype=torch.float64, device="cuda:0")
            P = eth.Problem(nn, domain=(-1.0, 1.0, -1.0, 1.0), nu=0.01, kind=eth.OSEEN, wind=w, precision=prec,
                            device="cuda:0", gmres_restart=8)
        else:
            P = eth.Problem(nn, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_CHEB_SGS, device="cuda:0",
                            mq_tile=tile)
        torch.cuda.synchronize()
        for k in kernels:
            ms, by = P.profile_kernel(k, reps=reps)
            var = P.mq_variant() if which != "oseen" else (0, 0)
            rec["launches"].append(dict(n=nn, kernel=eth.KERNEL_NAMES[k], bytes_per_launch=by,
                                        avg_us=round(1e3 * ms, 3), mq_tile=var[0],
                                        mq_steps_per_launch=var[1],
                                        precision="mixed" if prec == eth.MIXED else "fp64"))
            log(f"counters n={nn} {eth.KERNEL_NAMES[k]}: {by:.0f} B, {1e3 * ms:.2f} us")
        P.close()
        del P
        torch.cuda.empty_cache()
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=100)
    ap.add_argument("--profile-reps", type=int, default=50)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the Oseen, 64-RHS and ragged-batch measurements")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--no-micro", action="store_true",
                    help="skip the kernel bandwidth measurements at n = 2048 and 512 x 16")
    ap.add_argument("--counters", action="store_true",
                    help="only the launches read by the rocprofv3 byte counters (see counters_run)")
    ap.add_argument("--mq-tile", type=int, default=16, help="tile side of the fused M_Q step in --counters")
    ap.add_argument("--counters-kernel", choices=["mq", "apply", "oseen"], default="mq",
                    help="kernel of --counters: the fused M_Q step (headline), the FP64 apply at n = 2048, "
                         "or the Oseen apply and F smoothing step at n = 2048")
    ap.add_argument("--step-only", type=int, default=0, metavar="M",
                    help="only the flow-over-a-step workload at m elements per unit length (mixed and FP64; "
                         "the command of the step's kernel statistics)")
    ap.add_argument("--mq-variant", default="auto",
                    help="fused M_Q step of the headline solves as TILExSTEPS (e.g. 16x1), or auto (set-up "
                         "timing); a profiler serialises the two preconditioner branches, so a profiled run "
                         "fixes the variant the unprofiled run picks")
    args = ap.parse_args()
    mq_kw = {}
    if args.mq_variant != "auto":
        t, st = args.mq_variant.lower().split("x")
        mq_kw = dict(mq_tile=int(t), mq_fuse_steps=int(st))
    if args.counters:
        counters_run(args.n, args.profile_reps, args.mq_tile, args.counters_kernel)
        return
    if args.step_only:
        from paper_2303_10233_amd import eth
        res = []
        for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
            r = bench_step(args.step_only, prec, args.extra_steps, args.rtol)
            r["precision"] = name
            res.append(r)
            log(f"step m={args.step_only} {name}: {r['solves_per_s']} solves/s, {r['iterations']} its")
        print(json.dumps({"step": res}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 "
                          "(sharding over several GPUs is described, not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2303_10233_amd import eth

    n = args.n
    use_graph = not args.no_graph
    log(f"n={n} steps={args.steps} warmup={args.warmup} graph={use_graph}")
    results = {}
    problems = {}
    for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
        t0 = time.perf_counter()
        P = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_CHEB_SGS, device="cuda:0",
                        **mq_kw)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        b = P.assemble_rhs()
        dt, its, info = time_solves(P, b, args.steps, args.warmup, args.rtol, use_graph)
        _, tinfo = P.solve(b, rtol=args.rtol, maxit=2000, use_graph=use_graph, true_residual=True)
        results[name] = dict(seconds=dt, iterations=its, setup_s=setup_s,
                             true_residual=tinfo[0]["rel_residual_true"],
                             status=tinfo[0]["status"])
        problems[name] = P
        log(f"{name}: {args.steps / dt:.2f} solves/s, {1e3 * dt / args.steps:.2f} ms/solve, "
            f"iterations {its[-1]}, true rel. residual {tinfo[0]['rel_residual_true']:.2e}, "
            f"setup {setup_s:.2f} s")

    mixed, fp64 = results["mixed"], results["fp64"]
    equal_residual_ok = mixed["true_residual"] <= 2.0 * fp64["true_residual"]
    # set-up with the tuning cache warm (the first set-up above timed its
    # choices unless the cache already held them)
    t0 = time.perf_counter()
    Pw = eth.Problem(n, precision=eth.MIXED, velocity=eth.VEL_GMG, mq=eth.MQ_CHEB_SGS, device="cuda:0", **mq_kw)
    torch.cuda.synchronize()
    setup_info = {"first_s": round(mixed["setup_s"], 4), "warm_cache_s": round(time.perf_counter() - t0, 4),
                  "first_tuning_timed_cached": list(problems["mixed"].tuning_source()),
                  "warm_tuning_timed_cached": list(Pw.tuning_source())}
    Pw.close()
    log(f"set-up: {setup_info}")

    # --- kernel timing (HIP events on the problem's stream) -------------------
    Pm = problems["mixed"]
    its_m = mixed["iterations"][-1]
    levels, _ = Pm.levels()
    # launches of each kernel per MINRES iteration (mixed solver, finest level
    # for the multigrid kernels): V(2,2) with degree-2 Chebyshev = 1 pre-step
    # kernel + 2 post-step kernels on the finest level; 20 fused Chebyshev-SGS
    # steps; 1 saddle apply, 1 dot, 1 v update, 1 w/x update (the last two
    # run as one launch inside MINRES, the v update making the previous
    # iteration's w/x update; timed here as two, with the same bytes).
    per_iter = {eth.K_SADDLE_APPLY: 1, eth.K_CHEB_STEP: 3, eth.K_RESTRICT: 1, eth.K_PROLONG: 1,
                eth.K_MQ_CHEB_STEP: 20 // Pm.mq_variant()[1], eth.K_DOT: 1, eth.K_MINRES_V: 1,
                eth.K_MINRES_WX: 1,
                eth.K_COPY: 0}   # the plain copy calibrates the byte counters of a profiler run
    kernels = {}
    for k, cnt in per_iter.items():
        ms, by = Pm.profile_kernel(k, reps=args.profile_reps)
        kernels[eth.KERNEL_NAMES[k]] = dict(avg_us=1e3 * ms, bytes=by, gbs=by / (ms * 1e-3) / 1e9,
                                            launches_per_iteration=cnt,
                                            us_per_iteration=1e3 * ms * cnt)
    dom = max(kernels, key=lambda k: kernels[k]["us_per_iteration"])
    dk = kernels[dom]
    s_mixed = 4.0
    n_p = (n + 1) ** 2 + n * n
    N_u = 2 * (2 * n + 1) ** 2
    N_all = N_u + n_p
    # the bytes the roofline counts: the cost model's per-unit figure for the
    # dominant kernel (a Chebyshev-SGS step moves 10 s n_p: r, z, d and the
    # symmetric sweep's reads and writes), the kernel's own fused minimum
    # (read r, z, d; write z, d: 5 s n_p) reported beside it
    if dom == "k_mq_cheb_fused":
        steps_per_launch = Pm.mq_variant()[1]
        model_bytes = 10.0 * s_mixed * n_p * steps_per_launch
    else:
        model_bytes = dk["bytes"]
    achieved = model_bytes / (dk["avg_us"] * 1e-6) / 1e9
    working_set = 8.0 * N_all * 8    # eight FP64 Krylov vectors
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2),
                "peak": MI355X_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / MI355X_HBM_GBS, 5),
                "traffic": measured_traffic(dom, n, "k_mq_cheb_fused<float, %d, %d>" % Pm.mq_variant()[:2]
                                            if dom == "k_mq_cheb_fused" else None),
                "bytes_per_launch": model_bytes, "bytes_fused_min": dk["bytes"],
                "avg_launch_us": round(dk["avg_us"], 3),
                "mall_resident": working_set < 256e6,
                "note": ("working set below the 256 MB Infinity Cache: the figure is a cache/latency "
                         "rate, not an HBM one; HBM-scale kernel rates are in microbench")}

    def iteration_roofline(s_bytes, seconds, iterations):
        # cost model per MINRES iteration: Krylov vectors (FP64) + one V-cycle
        # + 20 Chebyshev-SGS steps
        by = 104.0 * N_all + s_bytes * N_u * 21 + 16.0 * N_u + 10.0 * s_bytes * n_p * 20
        t = seconds / args.steps / iterations
        return {"bytes": by, "us": round(t * 1e6, 2), "achieved": round(by / t / 1e9, 1),
                "frac": round(by / t / 1e9 / MI355X_HBM_GBS, 4), "unit": "GB/s"}
    iter_roof = {"mixed": iteration_roofline(4.0, mixed["seconds"], its_m),
                 "fp64": iteration_roofline(8.0, fp64["seconds"], fp64["iterations"][-1])}
    log("kernels: " + ", ".join(f"{k} {v['avg_us']:.1f}us {v['gbs']:.0f}GB/s"
                                for k, v in kernels.items()))
    # persistent kernel or kernel boundaries: one step of a ring dependency
    # over one block per CU, as dependent launches replayed from a graph and
    # as rounds of one cooperative launch separated by grid-wide barriers
    sync_probe = {"graph_launch_us": round(1e3 * Pm.profile_kernel(eth.K_SYNC_GRAPH, reps=1000)[0], 3),
                  "grid_barrier_us": round(1e3 * Pm.profile_kernel(eth.K_SYNC_GRID, reps=1000)[0], 3)}
    log(f"sync probe: {sync_probe}")

    extra = None
    if not args.no_extra:
        extra = {"oseen": [], "batch64": {}, "ragged": {}}
        for on in (128, 256):
            for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
                r = bench_oseen(on, 0.01, prec, args.extra_steps, args.rtol)
                r["precision"] = name
                extra["oseen"].append(r)
                log(f"oseen n={on} nu=1/100 {name}: {r['solves_per_s']} solves/s, "
                    f"{r['iterations']} its ({r['stage1_iterations']} stage I)")
        # nu = 1/1000: the plain F multigrid makes no headway (status no-progress);
        # with the Peclet cap the solve progresses but, as with exact pieces in
        # the oracle, does not reach 1e-6 within 4096 iterations
        r = bench_oseen(128, 0.001, eth.MIXED, 1, args.rtol, maxit=300)
        r["precision"] = "mixed"
        r["note"] = "nu = 1/1000 (element Peclet 15.6), plain damped-Jacobi F multigrid, maxit 300"
        extra["oseen"].append(r)
        log(f"oseen n=128 nu=1/1000 plain: status {r['status']}, residual {r['rel_residual']:.2e}")
        for on in (128, 256):
            for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
                r = bench_oseen(on, 0.001, prec, 1, args.rtol, maxit=4096, peclet_max=4.0)
                r["precision"] = name
                r["note"] = ("nu = 1/1000, F multigrid with element Peclet cap 4, maxit 4096 (exact pieces "
                             "in the oracle need more than 4096 per stage at 64^2 and 128^2)")
                extra["oseen"].append(r)
                log(f"oseen n={on} nu=1/1000 cap 4 {name}: status {r['status']}, {r['iterations']} its, "
                    f"residual {r['rel_residual']:.2e}, {r['ms_per_solve']} ms")
        extra["oseen_picard"] = []
        for on in (128, 256):
            for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
                r = bench_picard(on, 0.01, prec, args.extra_steps, args.rtol)
                r["precision"] = name
                extra["oseen_picard"].append(r)
                log(f"cavity Re=200 n={on} {name}: {r['solves_per_s']} solves/s, {r['iterations']} its "
                    f"({r['stage1_iterations']} stage I); 5 Picard steps {r['picard_seconds']} s "
                    f"{r['picard_iterations']}")
        extra["step"] = []
        for sm in (32, 64, 128):
            for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
                r = bench_step(sm, prec, args.extra_steps, args.rtol)
                r["precision"] = name
                extra["step"].append(r)
                log(f"step m={sm} {name}: {r['solves_per_s']} solves/s, {r['iterations']} its "
                    f"({r['stage1_iterations']} stage I), flux error {r['max_flux_error']:.1e}, "
                    f"Picard {r['picard_seconds']} s {r['picard_iterations']}")
        extra["stokes_schur_mq"] = {}
        for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
            Ps = eth.Problem(n, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_SCHUR_GMG)
            bs = Ps.assemble_rhs()
            dt, its, _ = time_solves(Ps, bs, args.steps, args.warmup, args.rtol, use_graph)
            _, ti = Ps.solve(bs, rtol=args.rtol, maxit=2000, use_graph=use_graph, true_residual=True)
            extra["stokes_schur_mq"][name] = dict(
                solves_per_s=round(args.steps / dt, 4), ms_per_solve=round(1e3 * dt / args.steps, 3),
                iterations=its[-1], true_rel_residual=ti[0]["rel_residual_true"],
                note="pressure mass by P0 elimination + Q1 multigrid for S_k (mesh independent)")
            log(f"stokes n={n} schur-gmg M_Q {name}: {extra['stokes_schur_mq'][name]}")
            Ps.close()
        # the larger configured cavity, same solver settings as the headline
        extra["stokes512"] = {}
        for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
            P5 = eth.Problem(512, precision=prec, velocity=eth.VEL_GMG, mq=eth.MQ_CHEB_SGS)
            b5 = P5.assemble_rhs()
            dt, its, _ = time_solves(P5, b5, args.extra_steps, 1, args.rtol, use_graph)
            _, ti = P5.solve(b5, rtol=args.rtol, maxit=2000, use_graph=use_graph, true_residual=True)
            extra["stokes512"][name] = dict(
                solves_per_s=round(args.extra_steps / dt, 4), ms_per_solve=round(1e3 * dt / args.extra_steps, 3),
                iterations=its[-1], true_rel_residual=ti[0]["rel_residual_true"],
                mq_variant=list(P5.mq_variant()[:2]))
            log(f"stokes n=512 {name}: {extra['stokes512'][name]}")
            P5.close()
        extra["adjoint"] = []
        for kind, an in (("stokes", 512), ("oseen", 256)):
            for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
                r = bench_adjoint(kind, an, prec, max(1, args.extra_steps - 1), args.rtol)
                r["precision"] = name
                extra["adjoint"].append(r)
                log(f"adjoint {kind} n={an} {name}: {r['gradients_per_s']} gradients/s "
                    f"({r['forward_iterations']} + {r['adjoint_iterations']} its)")
        for name, prec in (("mixed", eth.MIXED), ("fp64", eth.FP64)):
            extra["batch64"][name] = bench_batch(128, 64, prec, args.extra_steps, args.rtol)
            log(f"batch64 {name}: {extra['batch64'][name]}")
            extra["ragged"][name] = bench_ragged(prec, args.extra_steps, args.rtol)
            log(f"ragged {name}: {extra['ragged'][name]}")

    micro = None if args.no_micro else microbench(20)

    # configuration 1 on the GPU (16^2, exact velocity block, diagonal M_Q,
    # FP64 MINRES to 1e-6): rate, and the solution for the error against the
    # oracle's direct solve
    P1 = eth.Problem(16, precision=eth.FP64, velocity=eth.VEL_EXACT, mq=eth.MQ_DIAG)
    b1 = P1.assemble_rhs()
    dt1, its1, _ = time_solves(P1, b1, args.steps, args.warmup, args.rtol, use_graph)
    x1, _ = P1.solve(b1, rtol=args.rtol, maxit=3000, use_graph=use_graph)
    c1_gpu = {"solves_per_s": round(args.steps / dt1, 2), "iterations": its1[-1]}
    c1_x = x1.cpu().numpy()
    P1.close()

    cpu = None
    cpu_more = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        cpu = cpu_baseline(n, its_m, args.cpu_iters)
        log(f"oracle: {cpu['value']:.4g} solves/s ({cpu['seconds_per_iteration']:.2f} s/iteration)")
        g = {"c1_x": c1_x}
        if extra:
            g["batch64_iterations"] = extra["batch64"]["mixed"]["iterations_max"]
            g["oseen128_iterations"] = extra["oseen"][0]["iterations"]
            g["step32_iterations"] = extra["step"][0]["iterations"]
        cpu_more = cpu_other(g)
        log(f"oracle, other configurations: {json.dumps(cpu_more)}")

    value = args.steps / mixed["seconds"]
    out = {
        "metric": "Krylov solves/sec at 1e-6 residual, mixed vs FP64 on 1 GPU; stencil HBM GB/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * mixed["seconds"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 Krylov + f32 preconditioner",
        "data": "synthetic",
        "config": {
            "workload": f"Stokes lid-driven cavity, unit square, {n}x{n} Q2 elements, "
                        f"Q1+P0 pressure frame, MINRES rtol {args.rtol:g}, GMG V(2,2) Chebyshev "
                        f"+ 20-step Chebyshev-SGS pressure mass, mixed precision",
            "n": n,
            "unknowns": 2 * (2 * n + 1) ** 2 + (n + 1) ** 2 + n * n,
            "hip_graph": use_graph,
            "mq_tile": {"mixed": problems["mixed"].mq_tile()[0], "fp64": problems["fp64"].mq_tile()[0]},
            "mq_steps_per_launch": {"mixed": problems["mixed"].mq_variant()[1],
                                    "fp64": problems["fp64"].mq_variant()[1]},
        },
        "iterations": its_m,
        "true_rel_residual": mixed["true_residual"],
        "fp64": {"value": round(args.steps / fp64["seconds"], 4), "unit": "solves/s",
                 "ms_per_step": round(1e3 * fp64["seconds"] / args.steps, 4),
                 "iterations": fp64["iterations"][-1], "true_rel_residual": fp64["true_residual"]},
        "mixed_over_fp64": round(fp64["seconds"] / mixed["seconds"], 4),
        "setup": setup_info,
        "equal_residual_ok": bool(equal_residual_ok),
        "roofline": roofline,
        "iteration_roofline": iter_roof,
        "sync_probe": sync_probe,
        "config1_stokes16": c1_gpu,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "cpu_baseline": cpu,
        "cpu_other": cpu_more,
        "other_workloads": extra,
        "microbench": micro,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
